// qh2d.h -- workspace view and launch wrappers of the 2D Quickhull kernels.
#pragma once

#include "qh_device.h"

namespace qh {

constexpr int kBlock = 256;              // threads of the round kernel
constexpr int kItems = 8;                // points per thread
constexpr int kTile = kBlock * kItems;   // points per tile
constexpr int kSlots = 256;              // segments per LDS window
constexpr int kSegBlock = 256;           // threads (= segments) of the segment kernel
constexpr int kRankSmallCap = 8192;      // hull ids ranked inside one block's LDS
constexpr int32_t kCoordMax2D = (1 << 30) - 1;

// Device pointers of one workspace (passed by value to every kernel).
struct Ws2 {
    Control *ctl;
    // survivors: [round parity][region] planes x, y and input index
    int32_t *px[2][2];
    int32_t *py[2][2];
    int32_t *pi[2][2];
    // segment tables and tile maps: [round parity][region]
    SegGeo *geo[2][2];
    SegTop *top[2][2];
    int32_t *tmap[2][2];
    // per segment of the current round (global id = region-0 ids, then region 1)
    int2 *pst;     // global offsets (child 0, child 1) at the segment's first point
    int2 *pen;     // ... after its last point
    Best *adir;    // [seg][child] argmax of segments inside one tile
    // per tile of the current round
    Best *recF;    // [tile][child] partial argmax of the tile's first segment
    Best *recL;    // [tile][child] ... of its last segment
    uint64_t *st2[2];  // look-back status of the round kernel, by parity
    uint64_t *st4[2];  // look-back status of the segment kernel, by parity
    // extremes (set-up)
    Best *recF0, *recL0, *dir0;
    int32_t *inst_rank;
    // hull: compact vertex ids
    int32_t *V;       // input index of the vertex
    int32_t *hinst;   // its instance
    int32_t *nxt;     // next vertex counter-clockwise (-1 = unused id)
    int32_t *succ[2];
    int32_t *dist[2];
    int64_t cap_pts;  // points per survivor plane
    int32_t scap;     // segments per table
    int32_t hcap;     // compact hull ids
    int32_t tcap;     // tiles per round
    int32_t s4cap;    // look-back words of the segment kernel
};

hipError_t launch_instances(const Ws2 &ws, const int64_t *offsets, int64_t n_total, int32_t k,
                            hipStream_t st);
hipError_t launch_setup(const Ws2 &ws, const int64_t *offsets, int32_t k, int32_t ntiles, int grid,
                        hipStream_t st);
hipError_t launch_extremes(const Ws2 &ws, const int32_t *x, const int32_t *y, int32_t n,
                           int32_t vec_ok, int grid, int32_t nseg_max, hipStream_t st);
hipError_t launch_round(const Ws2 &ws, int32_t r, bool init, int mode, const int32_t *x,
                        const int32_t *y, int32_t vec_ok, int grid, hipStream_t st);
hipError_t launch_segments(const Ws2 &ws, int32_t r, int grid, hipStream_t st);
hipError_t launch_output(const Ws2 &ws, int32_t H, int32_t k, const int64_t *offsets,
                         int64_t *hull_offsets, int32_t *hull_idx, int64_t n_total, hipStream_t st);

}  // namespace qh
