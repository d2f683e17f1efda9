// qh3d.h -- records shared by the 3D kernels and the host topology step.
//
// The 3D path keeps the facets of the current hull on the host (their
// corners, neighbours and planes: a few hundred bytes per facet, small next to
// the point data) and the points on the device.  Every round the device finds
// the apex of every facet that still has outside points, the host picks
// apexes whose visible regions do not touch and replaces each region by its
// cone, and the device moves the points of the removed facets to the new
// facets or drops them.
#pragma once

#include "qh_device.h"

namespace qh3 {

constexpr int kBlock = 256;
constexpr int kItems = 4;
constexpr int kTile = kBlock * kItems;   // points per tile
constexpr int kGroupLds = 512;           // cone facets counted in LDS per block
constexpr int32_t kCoordMax = 1 << 19;   // |coordinate| bound of the exact int64 predicates
constexpr int64_t kInitSmall = 32768;    // instances up to this size get one init block each

// A facet as the kernels see it: outward normal n = (b - a) x (c - a),
// off = n . a (a point p is strictly above iff n . p > off), the corner a and
// the edge vectors b - a, c - a for the tie keys of the apex.
struct FacetRec {
    int64_t nx, ny, nz, off;
    int32_t ax, ay, az;
    int32_t ebx, eby, ebz;
    int32_t ecx, ecy, ecz;
    int32_t pad[3];
};

// A range of points to classify against a group of new facets.
struct SrcRec {
    int64_t start;    // first point (pool position, or input index)
    int32_t len;      // points
    int32_t gfirst;   // first facet of its group in the round's facet table
    int32_t gcount;   // facets in the group
    int32_t tile0;    // first tile of this range in the launch's tile space
};

// A range of points whose apex is wanted (one facet's outside set).
struct SegRec {
    int64_t start;   // first point in the pool
    int32_t len;
    int32_t facet;   // index into the round's facet table
    int32_t tile0;
    int32_t pad;
};

// Apex key: distance descending, then t1 = (p - a).(b - a), t2 = (p - a).(c - a)
// and the index ascending.
struct ApexKey {
    int64_t d, t1, t2;
    int32_t idx;
    int32_t x, y, z;
    int32_t pad;
};

// Initial simplex search results (device -> host).
struct InitRes {
    int32_t a, b, c, d;        // point indices (-1 = none)
    int32_t coords[4][3];
    int32_t error;             // 1 = coordinate out of range
    int32_t pad[3];
};

// Totals of the scan of the new facets' counts (device -> host).
struct ScanTot {
    int64_t written;   // points in the new outside sets
    int32_t nseg;      // facets with points
    int32_t ntiles;    // apex tiles of those facets
};

struct Pool {
    int32_t *x, *y, *z, *idx;
};

hipError_t launch_init(const int32_t *x, const int32_t *y, const int32_t *z, int32_t n,
                       void *scratch, InitRes *res, int grid, hipStream_t st);
hipError_t launch_classify(int pass, const int32_t *ix, const int32_t *iy, const int32_t *iz,
                           int from_input, Pool in, Pool out, const SrcRec *src, int32_t nsrc,
                           int32_t ntiles, const FacetRec *fac, uint32_t *counts,
                           uint32_t *cursor, const int64_t *range, int mode,
                           unsigned long long *filter_ctr, hipStream_t st);
// The outside-set ranges of the nf new facets from pass 1's counts:
// range[j] = top + (points of facets before j); the facets with points in
// facet order as seg records; cursor[j] = 0; totals in *tot (all of its
// fields written).  part: 3 * ceil(nf / kScanChunk) words of scratch.
constexpr int kScanChunk = kBlock * 8;
hipError_t launch_scan(const uint32_t *counts, int32_t nf, int64_t top, int64_t *range, SegRec *seg,
                       uint32_t *cursor, uint32_t *part, ScanTot *tot, hipStream_t st);
// The apex of each facet of seg[0 .. tot->nseg) over tot->ntiles tiles;
// nseg_max and ntiles_max bound those and size the grids.
hipError_t launch_apex(Pool pool, const SegRec *seg, int32_t nseg_max, int32_t ntiles_max,
                       const ScanTot *tot, const FacetRec *fac, ApexKey *tile_keys,
                       ApexKey *seg_keys, hipStream_t st);
hipError_t launch_gather(Pool in, Pool out, const SegRec *seg, int32_t nseg, int32_t ntiles,
                         const int64_t *dst, hipStream_t st);
size_t init_scratch_bytes(int grid);
// the first simplex of the instances list[0..count) (each [off[i], off[i+1]),
// at least 4 and at most kInitSmall points), one block each, results at res[i]
hipError_t launch_init_small(const int32_t *x, const int32_t *y, const int32_t *z, const int64_t *off,
                             const int32_t *list, int32_t count, InitRes *res, hipStream_t st);

}  // namespace qh3
