// qh_ctx.h -- the workspace context behind the opaque qh_ctx handle (library
// internal).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/qh.h"
#include "qh2d.h"

namespace qh3 {
struct Ctx3;
}

// launch configuration of a 2D call
struct QhLaunch {
    int grid;        // blocks of the round kernel
    int grid_multi;  // blocks of the multi-segment kernel
    int fin_segs;    // most segments a round may finish, one workgroup each
};

// a captured batch of launches (QH_FLAG_GRAPH)
struct QhGraph {
    int prefix;  // 1: set-up and extremes come first
    int r0, len; // rounds r0 .. r0 + len - 1
    hipGraphExec_t exec;
};

// a tuned size class (QH_FLAG_AUTOTUNE)
struct QhTuned {
    uint64_t key;
    QhLaunch cfg;
};

struct qh_ctx {
    int device = 0;
    int cus = 256;
    // capacities of the current allocation
    int64_t cap_pts = 0;
    int32_t scap = 0, hcap = 0, tcap = 0, s4cap = 0, s5cap = 0, kcap = 0;
    // pending growth requests after a capacity overflow
    int32_t want_scap = 0, want_hcap = 0;
    void *dmem = nullptr;
    size_t dbytes = 0;
    qh::Ws2 ws = {};
    qh::Control *ctl_host = nullptr;  // pinned copy of the control block
    int64_t *h_host = nullptr;        // pinned: hull count of a single call
    int64_t *single_off = nullptr;    // device int64[2]
    int64_t *single_hoff = nullptr;   // device int64[2]
    std::vector<hipEvent_t> ev;       // timing events (pairs)
    int grid[2] = {0, 0};             // resident blocks of the round kernel, per mode
    int grid_pre[2][2] = {{0, 0}, {0, 0}};  // ... of the split and of the round after it
    int grid_ext = 0;                 // resident blocks of the extremes kernel
    int hint_rounds = 0;              // rounds the last 2D call needed (first batch size)
    int fin_hint = 0;                 // the round it finished in (0: none or unknown),
    int64_t fin_hint_n = -1;          // ... for this point count,
    int32_t fin_hint_k = -1;          // ... instance count
    int fin_hint_mode = -1;           // ... and arithmetic
    qh3::Ctx3 *c3 = nullptr;          // 3D workspace, made on the first 3D call
    std::vector<unsigned char> gkey;  // launch arguments of the cached graphs
    std::vector<QhGraph> graphs;
    std::vector<QhTuned> tuned;
    unsigned long long *digest = nullptr;  // device: output digest of the autotuner's check
};

namespace qhi {

qh_status ctx_init(qh_ctx *c);
void ctx_free(qh_ctx *c);
void ctx3_free(qh3::Ctx3 *c3);

// A caller's context, or a temporary one freed at scope exit.
struct TempCtx {
    qh_ctx *c = nullptr;
    bool owned = false;
    ~TempCtx() {
        if (owned) ctx_free(c);
    }
};

qh_status get_ctx(const qh_opts *o, TempCtx &t);

}  // namespace qhi
