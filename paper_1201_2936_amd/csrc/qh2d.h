// qh2d.h -- workspace view and launch wrappers of the 2D Quickhull kernels.
#pragma once

#include "qh_device.h"

namespace qh {

constexpr int kBlock = 256;              // threads per block
constexpr int kItems = 8;                // points per thread
constexpr int kTile = kBlock * kItems;   // points per tile
constexpr int kSlots = 128;              // segments per LDS window (multi-segment tiles)
constexpr int kPieceItems = 8;           // tile counts per thread of the piece scan
constexpr int kSegBlock = 256;           // segments per tile of the segment phase
constexpr int kRankSmallCap = 8192;      // hull ids ranked inside one block's LDS (64 KB)
constexpr int kFinCap = 1024;            // points of a segment one block finishes in LDS
constexpr int kFinUnit = kFinCap / 2;     // points of a run of small segments finished together
constexpr int kFinUnitsPerBlock = 8;      // runs per finishing block that a round may need
constexpr int32_t kCoordMax2D = (1 << 30) - 1;
constexpr int kMaxStamps = 256;

// What a tile of the survivor array needs to know before it reads a point:
// the segment holding its first point (whose geometry is in the segment
// table) and whether that segment covers the whole tile (the common case).
struct TileInfo {
    int32_t seg;     // segment of the tile's first point (index in the region's table)
    int32_t single;  // 1: that segment covers the whole tile
    int32_t start, end;
};

// Device pointers of one workspace (passed by value to every kernel).  The
// buffers indexed by round parity p and region r are laid out back to back
// and addressed arithmetically, so no array of pointers is indexed at run
// time (that would force a copy of this struct into scratch memory).
struct Ws2 {
    Control *ctl;
    int32_t *pts_;      // survivors: [parity][region][plane x, y, index][cap_pts]
    SegGeo *geo_;       // segment tables: [parity][region][scap]
    SegTop *top_;       // [parity][region][scap]
    TileInfo *tinfo_;   // tile records: [parity][region][tcap]
    uint32_t *tcnt_;    // survivors per tile of a round (child 0 | child 1 << 16): [parity][tcap]
    int32_t *pv_;       // pieces of a round's input: virtual start [parity][region][tcap + 2]
    int32_t *pp_;       // ... physical start [parity][region][tcap + 2]
    int32_t *kf_;       // first piece of every tile [parity][region][tcap + 2]
    int32_t *ml_;       // tiles of a round that hold several segments: [parity][tcap]
    uint64_t *st5_;     // look-back words of the piece scan (counts): [parity][s5cap]
    uint64_t *st5b_;    // ... (non-empty pieces): [parity][s5cap]
    uint64_t *st4_;     // look-back words of the segment phase: [parity][s4cap]
    uint64_t *st4b_;    // ... of its second scan (child offsets): [parity][s4cap]
    int32_t *succ_;     // list ranking: [2][hcap]
    int32_t *dist_;     // [2][hcap]
    // per segment of the current round (global id = region-0 ids, then region 1)
    Best *adir;    // [seg][child] argmax of the segment
    // per tile of the current round
    Best *recF;    // [tile][child] partial argmax of the tile's first segment
    Best *recL;    // [tile][child] ... of its last segment
    // extremes (set-up)
    Best *recF0, *recL0, *dir0;
    int32_t *inst_rank;
    // hull: compact vertex ids
    int32_t *V;       // input index of the vertex
    int32_t *hinst;   // its instance
    int32_t *nxt;     // next vertex counter-clockwise (-1 = unused id)
    int64_t cap_pts;  // points per survivor plane
    int32_t scap;     // segments per table
    int32_t hcap;     // compact hull ids
    int32_t tcap;     // tiles per round
    int32_t s4cap;    // look-back words of the segment phase
    int32_t s5cap;    // look-back words of the piece scan

    __host__ __device__ int32_t *px(int p, int r) const { return pts_ + (size_t)((p * 2 + r) * 3 + 0) * cap_pts; }
    __host__ __device__ int32_t *py(int p, int r) const { return pts_ + (size_t)((p * 2 + r) * 3 + 1) * cap_pts; }
    __host__ __device__ int32_t *pi(int p, int r) const { return pts_ + (size_t)((p * 2 + r) * 3 + 2) * cap_pts; }
    __host__ __device__ SegGeo *geo(int p, int r) const { return geo_ + (size_t)(p * 2 + r) * scap; }
    __host__ __device__ SegTop *top(int p, int r) const { return top_ + (size_t)(p * 2 + r) * scap; }
    __host__ __device__ TileInfo *tinfo(int p, int r) const { return tinfo_ + (size_t)(p * 2 + r) * tcap; }
    __host__ __device__ uint32_t *tcnt(int p) const { return tcnt_ + (size_t)p * tcap; }
    __host__ __device__ int32_t *pv(int p, int r) const { return pv_ + (size_t)(p * 2 + r) * (tcap + 2); }
    __host__ __device__ int32_t *pp(int p, int r) const { return pp_ + (size_t)(p * 2 + r) * (tcap + 2); }
    __host__ __device__ int32_t *kf(int p, int r) const { return kf_ + (size_t)(p * 2 + r) * (tcap + 2); }
    __host__ __device__ int32_t *ml(int p) const { return ml_ + (size_t)p * tcap; }
    __host__ __device__ uint64_t *st5(int p) const { return st5_ + (size_t)p * s5cap; }
    __host__ __device__ uint64_t *st5b(int p) const { return st5b_ + (size_t)p * s5cap; }
    __host__ __device__ uint64_t *st4(int p) const { return st4_ + (size_t)p * s4cap; }
    __host__ __device__ uint64_t *st4b(int p) const { return st4b_ + (size_t)p * s4cap; }
    __host__ __device__ int32_t *succ(int p) const { return succ_ + (size_t)p * hcap; }
    __host__ __device__ int32_t *dist(int p) const { return dist_ + (size_t)p * hcap; }
};

struct HullArgs {
    const int32_t *x;
    const int32_t *y;
    const int64_t *offsets;
    int32_t *hull_idx;
    int64_t *hull_offsets;
    int32_t n;
    int32_t k;
    int32_t vec_ok;      // the planes are 4-byte aligned: 4-point vector loads
    int32_t timing;
    int32_t max_rounds;
    int32_t fin_cap;   // finish every segment in one block once none is larger (0: off)
    int32_t fin_segs;  // ... and there are at most this many segments
    int32_t grid_split;  // blocks of the split and of the round after it (0: the
    int32_t grid_ro1;    // round kernel's grid)
    int32_t fin_from;    // first round whose finishing kernel is launched (earlier
                         // rounds never finish: their segments go on as rounds)
    int32_t fin_pts;     // or finish runs of segments, kFinUnit points per block at
                         // a time, once none is larger and the round holds at most
                         // this many points (0: off)
};

hipError_t launch_setup(const Ws2 &ws, const HullArgs &a, int grid, hipStream_t st);
hipError_t launch_extremes(const Ws2 &ws, const HullArgs &a, int grid, hipStream_t st);
hipError_t launch_round(const Ws2 &ws, const HullArgs &a, int mode, int32_t r, int grid,
                        int grid_multi, int grid_fin, hipStream_t st);
hipError_t launch_segments(const Ws2 &ws, const HullArgs &a, int32_t r, int grid, hipStream_t st);
hipError_t launch_output(const Ws2 &ws, const HullArgs &a, int32_t H, hipStream_t st);
// resident blocks on the whole device of the split, the round after it and
// the later rounds' kernel
hipError_t round_grids(int mode, int cus, int (&grids)[3]);
// resident blocks of the extremes kernel
hipError_t extremes_grid(int cus, int *grid);

}  // namespace qh
