// qh2d_kernels.hip -- the 2D segmented Quickhull on gfx950.
//
// The permute-and-segment Quickhull (Tzeng & Owens, Section 3.1; the 2D
// driver of Algorithm 4) as a short sequence of kernels per call:
//
//   set-up       non-empty instances become the first segments, tile records
//   extremes     lexicographic min / max of every instance (first split's
//                extrema, Algorithm 4) and the coordinate range check
//   round r      one pass over the survivors: each point is tested against the
//                two new edges u->f and f->v of its segment (the triangle test
//                and the "which edge" state), points inside the triangle are
//                dropped (compact, Section 4.2), the others are written to the
//                two child segments (a 2-state flagPermute, Section 4.1) using
//                a single-pass decoupled look-back scan, and the farthest point
//                of every child (next round's apex) is found on the way.
//                Round 0 is the first split (its input is the caller's array).
//   segments r   one thread per segment: the apex joins the hull, multi-tile
//                argmax partials are merged, the next segment table is written
//   output       list ranking of the hull cycles, CCW index lists
//
// Every kernel reads the round state from device memory and does nothing once
// no segment is left, so the host enqueues rounds in batches and reads the
// state back once per batch.
//
// Survivors are structure-of-arrays int32 x[], y[], idx[] in two regions per
// round (children of state 0 and of state 1); a segment is a range
// [start, start+len) of one region in compacted order.  Each block of the
// round kernel takes a fixed contiguous range of 2048-point tiles (no atomics)
// and writes the survivors of tile t at t * 2048 of each region (a piece);
// the segment kernel's scans (decoupled look-back over dynamically claimed
// scan tiles) turn the pieces' counts into the next round's piece table.
#include "../../include/qh.h"
#include "qh2d.h"

#include <algorithm>

namespace qh {

// FP32 filter constant: |fl(a b - c d) - (a b - c d)| <= 4.0000004 eps
// (|fl(a b)| + |fl(c d)|) for a, b, c, d rounded from int32 (eps = 2^-24);
// 5 eps also covers the rounding of the bound itself.
constexpr float kErrC = 5.0f / 16777216.0f;
constexpr int kNW = kBlock / kWave;

// Four consecutive int32 coordinates.  Only 4-byte alignment is assumed: the
// y plane starts n values after the x plane, and dword-aligned multi-dword
// global loads are legal on gfx9 and later (one instruction still moves 16
// bytes per lane).
typedef int32_t i32x4u __attribute__((ext_vector_type(4), aligned(4)));
constexpr int kQ = kItems / 4;

// ---------------------------------------------------------------------------
// arithmetic
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t cross_i64(int32_t px, int32_t py, int32_t ax, int32_t ay,
                                             int32_t bx, int32_t by) {
    // (p - a) x (b - a): > 0 when p lies strictly right of a -> b
    const int32_t dx = px - ax, dy = py - ay, ex = bx - ax, ey = by - ay;
    return (int64_t)dx * (int64_t)ey - (int64_t)dy * (int64_t)ex;
}

__device__ __forceinline__ float cross_f32(int32_t px, int32_t py, int32_t ax, int32_t ay,
                                           int32_t bx, int32_t by, float &bound) {
    const int32_t dx = px - ax, dy = py - ay, ex = bx - ax, ey = by - ay;
    const float p1 = __fmul_rn((float)dx, (float)ey);
    const float p2 = __fmul_rn((float)dy, (float)ex);
    bound = __fmul_rn(__fadd_rn(fabsf(p1), fabsf(p2)), kErrC);
    return __fsub_rn(p1, p2);
}

// The same estimate without its own bound, for callers that use a bound
// valid for every point of the input (static_bound).
__device__ __forceinline__ float cross_f32_nb(int32_t px, int32_t py, int32_t ax, int32_t ay,
                                              int32_t ex, int32_t ey) {
    const int32_t dx = px - ax, dy = py - ay;
    return __fsub_rn(__fmul_rn((float)dx, (float)ey), __fmul_rn((float)dy, (float)ex));
}

// A bound on the error of cross_f32_nb for every input point against an edge
// with direction (ex, ey): with |coordinate| <= C, |dx| and |dy| are at most
// 2C, so the error is at most about 4 eps 2C (|ex| + |ey|) (two conversions,
// a product and the difference each round once); kErrC = 5 eps also covers
// the rounding of c2 = fl(2C) and of this product.
__device__ __forceinline__ float static_bound(int32_t ex, int32_t ey, float c2) {
    return __fmul_rn(__fmul_rn(c2, __fadd_rn(fabsf((float)ex), fabsf((float)ey))), kErrC);
}

// Tie-break key of a point for the argmax over a child with edge direction
// (ex, ey): among equally far points (a line parallel to the edge) the one
// with the smallest t = (p - u).e, then the lowest index.  Along such a line
// t is monotone in x (or in y when ex = 0), so one 32-bit coordinate does.
__device__ __forceinline__ uint64_t tie_key(int32_t px, int32_t py, int32_t idx, int32_t ex,
                                            int32_t ey) {
    const int32_t s = ex > 0 ? px : ex < 0 ? -px : (ey > 0 ? py : -py);
    return ((uint64_t)((uint32_t)s ^ 0x80000000u) << 32) | (uint64_t)(uint32_t)idx;
}

__device__ __forceinline__ uint32_t fkey(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ uint64_t coord_key(int32_t x, int32_t y) {
    return ((uint64_t)((uint32_t)x ^ 0x80000000u) << 32) | (uint64_t)((uint32_t)y ^ 0x80000000u);
}

// A load through the scalar data cache (uniform address; the data was
// written by an earlier kernel and is not written by this one).
template <typename T>
__device__ __forceinline__ T scalar_load(const T *ptr) {
    return *(const __attribute__((address_space(4))) T *)(ptr);
}

// 2C as a float, from the control block's coordinate span
__device__ __forceinline__ float coord_c2(const Control *ctl) {
    const uint32_t cs = scalar_load(&ctl->cspan);
    const uint32_t c = cs > (uint32_t)kCoordMax2D ? cs - (uint32_t)kCoordMax2D : 0u;
    return (float)(2.0 * (double)c);
}

// largest i in [0, m) with s[i] <= v  (s[0] <= v, s nondecreasing)
__device__ __forceinline__ int slot_of(const int32_t *s, int m, int32_t v) {
    int a = 0, b = m;
    while (b - a > 1) {
        const int c = (a + b) >> 1;
        if (s[c] <= v) a = c; else b = c;
    }
    return a;
}

__device__ __forceinline__ Best best_none() {
    Best b;
    b.key1 = 0;
    b.key2 = ~0ull;
    b.x = b.y = b.idx = b.cnt = 0;
    return b;
}

__device__ __forceinline__ void best_merge(Best &acc, const Best &b) {
    if (best_better(b, acc)) {
        acc.key1 = b.key1;
        acc.key2 = b.key2;
        acc.x = b.x;
        acc.y = b.y;
        acc.idx = b.idx;
        acc.cnt = b.cnt;
    }
}

// merge of argmax records that also sums the child counts
__device__ __forceinline__ void rec_merge(Best &acc, const Best &b) {
    const int32_t c = acc.cnt + b.cnt;
    if (best_better(b, acc)) {
        acc.key1 = b.key1;
        acc.key2 = b.key2;
        acc.x = b.x;
        acc.y = b.y;
        acc.idx = b.idx;
    }
    acc.cnt = c;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// butterfly all-reduce of a Best over the 64 lanes of a wave
__device__ __forceinline__ void wave_best(Best &b) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        Best o;
        o.key1 = shfl_xor_u64(b.key1, m);
        o.key2 = shfl_xor_u64(b.key2, m);
        o.x = __shfl_xor(b.x, m);
        o.y = __shfl_xor(b.y, m);
        o.idx = __shfl_xor(b.idx, m);
        o.cnt = 0;
        if (best_better(o, b)) b = o;
    }
}

__device__ __forceinline__ void wave_rec(Best &b) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        Best o;
        o.key1 = shfl_xor_u64(b.key1, m);
        o.key2 = shfl_xor_u64(b.key2, m);
        o.x = __shfl_xor(b.x, m);
        o.y = __shfl_xor(b.y, m);
        o.idx = __shfl_xor(b.idx, m);
        o.cnt = __shfl_xor(b.cnt, m);
        rec_merge(b, o);
    }
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m));
    return v;
}

// number of set bits of a wave mask in the lanes below this one
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// DPP reductions (row shifts and row broadcasts, no LDS): the result is
// complete in lane 63 only.  A lane whose source is outside its row, or
// whose row is masked off, receives the operation's identity.
template <int Ctrl, int RowMask>
__device__ __forceinline__ uint32_t dpp_or0(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, RowMask, 0xf, true);
}

template <int Ctrl, int RowMask>
__device__ __forceinline__ void rec_step(Best &b) {
    Best o;
    o.key1 = ((uint64_t)dpp_or0<Ctrl, RowMask>((uint32_t)(b.key1 >> 32)) << 32) |
             (uint64_t)dpp_or0<Ctrl, RowMask>((uint32_t)b.key1);
    o.key2 = ((uint64_t)dpp_or0<Ctrl, RowMask>((uint32_t)(b.key2 >> 32)) << 32) |
             (uint64_t)dpp_or0<Ctrl, RowMask>((uint32_t)b.key2);
    o.x = (int32_t)dpp_or0<Ctrl, RowMask>((uint32_t)b.x);
    o.y = (int32_t)dpp_or0<Ctrl, RowMask>((uint32_t)b.y);
    o.idx = (int32_t)dpp_or0<Ctrl, RowMask>((uint32_t)b.idx);
    o.cnt = (int32_t)dpp_or0<Ctrl, RowMask>((uint32_t)b.cnt);
    rec_merge(b, o);  // a zero record (key1 = 0) never wins; it adds no count
}

// argmax record with summed counts over the wave, complete in lane 63
__device__ __forceinline__ void wave_rec63(Best &b) {
    rec_step<0x111, 0xf>(b);   // row_shr:1
    rec_step<0x112, 0xf>(b);   // row_shr:2
    rec_step<0x114, 0xf>(b);   // row_shr:4
    rec_step<0x118, 0xf>(b);   // row_shr:8
    rec_step<0x142, 0xa>(b);   // row_bcast:15 -> rows 1 and 3
    rec_step<0x143, 0xc>(b);   // row_bcast:31 -> rows 2 and 3
}

template <int Ctrl, int RowMask>
__device__ __forceinline__ float dpp_fmax_step(float v) {
    const uint32_t ninf = 0xff800000u;  // -inf: the identity of max
    const float o = __uint_as_float((uint32_t)__builtin_amdgcn_update_dpp(
        (int)ninf, (int)__float_as_uint(v), Ctrl, RowMask, 0xf, false));
    return fmaxf(v, o);
}

// A lighter running argmax for the one-segment path: the exact distance, the
// tie key (its low 32 bits are the point's index) and the count; the
// point's coordinates are read back from the input when the record is made.
struct RunBest {
    uint64_t k1, k2;
    int32_t cnt;
};

__device__ __forceinline__ RunBest rb_none() {
    RunBest b;
    b.k1 = 0;
    b.k2 = ~0ull;
    b.cnt = 0;
    return b;
}

__device__ __forceinline__ void rb_offer(RunBest &b, uint64_t d, int32_t x, int32_t y, int32_t idx,
                                         int32_t ex, int32_t ey) {
    if (d < b.k1) return;
    const uint64_t k2 = tie_key(x, y, idx, ex, ey);
    if (d > b.k1 || k2 < b.k2) {
        b.k1 = d;
        b.k2 = k2;
    }
}

// the same update without branches (take = the point belongs to the child)
__device__ __forceinline__ void rb_offer_nb(RunBest &b, bool take, uint64_t d, int32_t x, int32_t y,
                                            int32_t idx, int32_t ex, int32_t ey) {
    const uint64_t k2 = tie_key(x, y, idx, ex, ey);
    const bool better = take && (d > b.k1 || (d == b.k1 && k2 < b.k2));
    b.k1 = better ? d : b.k1;
    b.k2 = better ? k2 : b.k2;
}

__device__ __forceinline__ void rb_merge(RunBest &acc, const RunBest &o) {
    const int32_t c = acc.cnt + o.cnt;
    if (o.k1 > acc.k1 || (o.k1 == acc.k1 && o.k1 != 0 && o.k2 < acc.k2)) {
        acc.k1 = o.k1;
        acc.k2 = o.k2;
    }
    acc.cnt = c;
}

template <int Ctrl, int RowMask>
__device__ __forceinline__ void rb_step(RunBest &b) {
    RunBest o;
    o.k1 = ((uint64_t)dpp_or0<Ctrl, RowMask>((uint32_t)(b.k1 >> 32)) << 32) |
           (uint64_t)dpp_or0<Ctrl, RowMask>((uint32_t)b.k1);
    o.k2 = ((uint64_t)dpp_or0<Ctrl, RowMask>((uint32_t)(b.k2 >> 32)) << 32) |
           (uint64_t)dpp_or0<Ctrl, RowMask>((uint32_t)b.k2);
    o.cnt = (int32_t)dpp_or0<Ctrl, RowMask>((uint32_t)b.cnt);
    rb_merge(b, o);  // a zero record (k1 = 0) never wins; it adds no count
}

// complete in lane 63
__device__ __forceinline__ void wave_rb63(RunBest &b) {
    rb_step<0x111, 0xf>(b);
    rb_step<0x112, 0xf>(b);
    rb_step<0x114, 0xf>(b);
    rb_step<0x118, 0xf>(b);
    rb_step<0x142, 0xa>(b);
    rb_step<0x143, 0xc>(b);
}

// maximum over the wave, returned to every lane
__device__ __forceinline__ float wave_max_f_dpp(float v) {
    v = dpp_fmax_step<0x111, 0xf>(v);
    v = dpp_fmax_step<0x112, 0xf>(v);
    v = dpp_fmax_step<0x114, 0xf>(v);
    v = dpp_fmax_step<0x118, 0xf>(v);
    v = dpp_fmax_step<0x142, 0xa>(v);
    v = dpp_fmax_step<0x143, 0xc>(v);
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), kWave - 1));
}

// candidate update of a running best with an exact distance d > 0
__device__ __forceinline__ void best_offer(Best &b, uint64_t d, int32_t x, int32_t y, int32_t idx,
                                           int32_t ex, int32_t ey) {
    if (d < b.key1) return;
    const uint64_t k2 = tie_key(x, y, idx, ex, ey);
    if (d > b.key1 || k2 < b.key2) {
        b.key1 = d;
        b.key2 = k2;
        b.x = x;
        b.y = y;
        b.idx = idx;
    }
}

// ---------------------------------------------------------------------------
// LDS layouts of the phases (they share one buffer)
// ---------------------------------------------------------------------------
struct RoundSmem {
    int32_t s_m;
    uint32_t s_tot;
    uint32_t stat[4];
    uint32_t scan[kQ * kNW];
    int32_t sstart[kTile + 4];      // segment starts of a multi-segment tile
    int32_t pvs[kTile + 4];         // virtual starts of the tile's input pieces
    int32_t pps[kTile + 4];         // ... their physical starts
    int32_t lgeo[kSlots][6];
    uint64_t k1[2][kSlots];
    uint64_t k2[2][kSlots];
    uint32_t lm[2][kSlots];
    uint32_t scnt[2][kSlots];
    int32_t res[2][kSlots][3];
    Best wrec[kNW][2];              // per-wave argmax records of a one-segment tile
    uint32_t wcnt[kNW];             // per-wave survivor counts (child 0 | child 1 << 16)
    uint32_t woff[kNW];             // their tile-local offsets
};

struct FastSmem {
    uint32_t stat[4];
    int32_t pvs[2][kTile + 4];      // virtual starts of a tile's input pieces (by tile parity)
    int32_t pps[2][kTile + 4];      // ... their physical starts
    RunBest wrb[kNW][2];            // per-wave argmax of a run
    uint32_t wcnt[2][kNW];          // per-wave survivor counts (child 0 | child 1 << 16)
};

struct ExtSmem {
    int32_t s_m, pad;
    Best red[kNW][2];
    int32_t sstart[kTile + 4];
    uint64_t kmin1[kSlots], kmin2[kSlots], kmax1[kSlots], kmax2[kSlots];
    int32_t rmin[kSlots][3], rmax[kSlots][3];
};

struct SegSmem {
    uint32_t pscan[4 * (kSegBlock / kWave)];
    uint32_t scan[2 * (kSegBlock / kWave)];
    uint32_t scan2[2 * (kSegBlock / kWave)];
    int32_t s_tile, qn_apex, qn_map, pad;
    uint64_t s_ex, s_ex2;
    int16_t q_apex[kSegBlock];
    int16_t q_map[2 * kSegBlock];
    int32_t o_t0[kSegBlock], o_t1[kSegBlock];
    int32_t o_ka[2 * kSegBlock], o_kb[2 * kSegBlock], o_id[2 * kSegBlock];
    int32_t o_st[2 * kSegBlock], o_en[2 * kSegBlock];
    Best qres[2 * kSegBlock];   // merged records of the queued segments (by owner)
    Best red[2 * kNW];
};

struct RankSmem {
    int32_t su[kRankSmallCap];
    int32_t di[kRankSmallCap];
};

struct ScanSmem {
    uint32_t scratch[32];
    unsigned long long carry;
    int32_t bad;
    int32_t maxlen;
};

template <typename A, typename B>
constexpr size_t cmax(A a, B b) { return a > b ? a : b; }
constexpr size_t kSmemBytes =
    cmax(cmax(cmax(sizeof(RoundSmem), sizeof(ExtSmem)), cmax(sizeof(SegSmem), sizeof(RankSmem))),
         sizeof(ScanSmem));


// Append tile t to the list of multi-segment tiles (wave-aggregated atomic).
// Called by every lane of a wave; lanes with want == false add nothing.
__device__ __forceinline__ void ml_append(const Ws2 &ws, int p, RoundState *rsp, bool want, int t) {
    const uint64_t m = __ballot(want);
    if (m == 0) return;
    const int leader = __builtin_ctzll(m);
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(&rsp->nmulti, (int)__popcll(m));
    base = __builtin_amdgcn_readlane(base, leader);
    if (want) {
        const int l = lane_id();
        const uint64_t below = l ? (m & (~0ull >> (64 - l))) : 0ull;
        const int slot = base + (int)__popcll(below);
        if (slot < ws.tcap) ws.ml(p)[slot] = t;
        else atomicOr(&ws.ctl->error, kErrInternal);
    }
}

// ---------------------------------------------------------------------------
// set-up
// ---------------------------------------------------------------------------
// block 0: compact the non-empty instances into the first segment table.
// Each thread takes kInstPer consecutive instances per pass (their offsets
// requested together), one block scan per pass
constexpr int kInstPer = 16;
__device__ __forceinline__ void phase_instances(const Ws2 &ws, const HullArgs &a, char *smem) {
    if (blockIdx.x != 0) return;
    ScanSmem *sm = reinterpret_cast<ScanSmem *>(smem);
    Control *ctl = ws.ctl;
    const int k = a.k;
    if (threadIdx.x == 0) { sm->carry = 0; sm->bad = 0; sm->maxlen = 0; }
    __syncthreads();
    for (int base = 0; base < k; base += kBlock * kInstPer) {
        const int i0 = base + (int)threadIdx.x * kInstPer;
        int64_t off[kInstPer + 1];
#pragma unroll
        for (int j = 0; j <= kInstPer; ++j) off[j] = i0 + j <= k ? a.offsets[i0 + j] : 0;
        uint32_t cnt = 0;
        bool bad = false;
        int mx = 0;
#pragma unroll
        for (int j = 0; j < kInstPer; ++j) {
            const int i = i0 + j;
            if (i >= k) continue;
            const int64_t lo = off[j], hi = off[j + 1];
            if (lo < 0 || hi < lo || hi > a.n || (i == 0 && lo != 0) || (i == k - 1 && hi != a.n)) bad = true;
            if (hi > lo) {
                ++cnt;
                mx = max(mx, (int)min<int64_t>(hi - lo, INT32_MAX));
            }
        }
        if (bad) atomicOr(&sm->bad, 1);
        if (mx > 0) atomicMax(&sm->maxlen, mx);
        uint32_t v[1] = {cnt}, tot[1];
        block_excl_scan<kBlock, 1>(v, tot, sm->scratch);
        uint32_t jn = (uint32_t)sm->carry + v[0];
#pragma unroll
        for (int j = 0; j < kInstPer; ++j) {
            const int i = i0 + j;
            if (i >= k) continue;
            const int64_t lo = off[j], hi = off[j + 1];
            const bool ne = hi > lo;
            ws.inst_rank[i] = ne ? (int32_t)jn : -1;
            ws.nxt[i] = -1;
            ws.nxt[k + i] = -1;
            if (ne) {
                SegGeo g;
                g.start = (int32_t)lo;
                g.len = (int32_t)(hi - lo);
                g.ux = g.uy = g.fx = g.fy = g.vx = g.vy = 0;
                ws.geo(0, 0)[jn] = g;
                SegTop t;
                t.fidx = 0;
                t.uc = i;
                t.vc = i;
                t.inst = i;
                ws.top(0, 0)[jn] = t;
                ++jn;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) sm->carry += tot[0];
        __syncthreads();
    }
    if (threadIdx.x < 64) ctl->cspan_slot[threadIdx.x] = (uint32_t)kCoordMax2D;
    for (int i = threadIdx.x; i < 4 * kAccSlots; i += blockDim.x) (&ctl->nacc[0][0][0])[i] = 0;
    for (int i = threadIdx.x; i < 3 * kAccSlots; i += blockDim.x) (&ctl->fstat[0][0])[i] = 0;
    if (threadIdx.x == 0) {
        RoundState z = {};
        ctl->rs[1] = z;
        RoundState r0 = {};
        r0.n[0] = a.n;
        r0.n[1] = 0;
        r0.s[0] = (int32_t)sm->carry;
        r0.s[1] = 0;
        r0.hbase = k;
        ctl->rs[0] = r0;
        ctl->error = sm->bad ? kErrOffsets : 0;
        ctl->setup_error = sm->bad ? kErrOffsets : 0;
        ctl->rounds_done = 0;
        ctl->max_segments = (int32_t)sm->carry;
        ctl->final_round = 0;
        ctl->points_in = ctl->points_out = ctl->first_in = ctl->first_out = 0;
        ctl->second_in = ctl->second_out = 0;
        ctl->cspan = (uint32_t)kCoordMax2D;
        ctl->rounds_with_work = 0;
        ctl->H = 0;
        ctl->h_total = 0;
        ctl->maxseg[0] = sm->maxlen;
        ctl->maxseg[1] = 0;
        ctl->fin_ids = 0;
        ctl->fin_round = -1;
        ctl->fin_runs = 0;
    }
}

// tile records of the input (tile -> instance segment) and clean look-back words
__device__ __forceinline__ void phase_setup(const Ws2 &ws, const HullArgs &a) {
    const int stride = gridDim.x * blockDim.x;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = tid; i < ws.s5cap; i += stride) {
        ws.st5(0)[i] = 0;
        ws.st5(1)[i] = 0;
        ws.st5b(0)[i] = 0;
        ws.st5b(1)[i] = 0;
    }
    for (int i = tid; i < ws.s4cap; i += stride) {
        ws.st4(0)[i] = 0;
        ws.st4(1)[i] = 0;
        ws.st4b(0)[i] = 0;
        ws.st4b(1)[i] = 0;
    }
    if (ws.ctl->error) return;
    const int ntiles = (a.n + kTile - 1) / kTile;
    // every wave iterates in lock step (ml_append is wave-collective)
    for (int t0 = tid - lane_id(); t0 < ntiles; t0 += stride) {
        const int t = t0 + lane_id();
        if (t >= ntiles) {
            ml_append(ws, 0, &ws.ctl->rs[0], false, 0);
            continue;
        }
        const int64_t v = (int64_t)t * kTile;
        // largest i with offsets[i] <= v: that instance holds v and is non-empty
        int lo = 0, hi = a.k;
        while (hi - lo > 1) {
            const int c = (lo + hi) >> 1;
            if (a.offsets[c] <= v) lo = c; else hi = c;
        }
        const int64_t st = a.offsets[lo], en = a.offsets[lo + 1];
        TileInfo ti = {};
        ti.seg = ws.inst_rank[lo];
        ti.start = (int32_t)st;
        ti.end = (int32_t)en;
        ti.single = en >= min(v + kTile, (int64_t)a.n) ? 1 : 0;
        ws.tinfo(0, 0)[t] = ti;
        ml_append(ws, 0, &ws.ctl->rs[0], !ti.single, t);
    }
}

// ---------------------------------------------------------------------------
// extremes: lexicographic min and max of every instance, range check
// ---------------------------------------------------------------------------
__device__ __forceinline__ void phase_extremes(const Ws2 &ws, const HullArgs &a, char *smem) {
    Control *ctl = ws.ctl;
    if (ctl->error) return;
    ExtSmem *sm = reinterpret_cast<ExtSmem *>(smem);
    const int n = a.n;
    const int S = ctl->rs[0].s[0];
    const int ntiles = (n + kTile - 1) / kTile;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
    // Every block takes a contiguous range of tiles.  Consecutive tiles of
    // one instance form a run whose minimum and maximum stay in registers;
    // the block reduces once per run and writes the run's record at its first
    // tile (the other tiles of the run get empty records).  Tiles that hold
    // several instances are reduced per instance in LDS.
    const int T = (ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
    if (blockIdx.x == 0 && tid == 0) ctl->tper_ext = T;
    const int tb = blockIdx.x * T, te = min(tb + T, ntiles);
    // a run's extremes per lane: the smallest and largest coordinate key and
    // the first index that has it (each lane sees its points in index order)
    uint64_t kmn = ~0ull, kmx = 0ull;
    int32_t imn = -1, imx = -1;
    uint32_t span = 0;   // largest coordinate + bound seen, for the range check
    uint32_t nspan = 0;  // largest bound - coordinate (the other side)
    int cur = -1, run0 = 0, cst = 0, cen = 0;
    auto as_best = [](uint64_t key1, uint64_t ck, int32_t idx) {
        Best b = best_none();
        if (idx >= 0) {
            b.key1 = key1;
            b.key2 = (uint32_t)idx;
            b.x = (int32_t)((uint32_t)(ck >> 32) ^ 0x80000000u);
            b.y = (int32_t)((uint32_t)ck ^ 0x80000000u);
            b.idx = idx;
            b.cnt = 0;
        }
        return b;
    };
    auto flush = [&](int tend) {
        Best rmn = as_best(~kmn, kmn, imn), rmx = as_best(kmx, kmx, imx);
        wave_rec63(rmn);
        wave_rec63(rmx);
        if (lane == kWave - 1) { sm->red[wv][0] = rmn; sm->red[wv][1] = rmx; }
        __syncthreads();
        if (tid == 0) {
            Best m0 = sm->red[0][0], m1 = sm->red[0][1];
            for (int w = 1; w < kNW; ++w) {
                best_merge(m0, sm->red[w][0]);
                best_merge(m1, sm->red[w][1]);
            }
            ws.recF0[run0 * 2 + 0] = m0; ws.recF0[run0 * 2 + 1] = m1;
            ws.recL0[run0 * 2 + 0] = m0; ws.recL0[run0 * 2 + 1] = m1;
            if (cst >= run0 * kTile && cen <= min(tend * kTile, n)) {
                ws.dir0[cur * 2 + 0] = m0;
                ws.dir0[cur * 2 + 1] = m1;
            }
        }
        __syncthreads();
        kmn = ~0ull;
        kmx = 0ull;
        imn = -1;
        imx = -1;
    };
    // the points of a tile (4-point vectors where the input allows) and its record
    auto load_tile = [&](int tile, int32_t (&X)[kItems], int32_t (&Y)[kItems], TileInfo &ti, bool whole) {
        const int lo = tile * kTile;
        const int hi = min(lo + kTile, n);
#pragma unroll
        for (int qq = 0; qq < kQ; ++qq) {
            const int v0 = lo + qq * kBlock * 4 + tid * 4;
            if (whole || (a.vec_ok && v0 + 3 < hi)) {
                const i32x4u p = *reinterpret_cast<const i32x4u *>(a.x + v0);
                const i32x4u q = *reinterpret_cast<const i32x4u *>(a.y + v0);
                X[qq * 4 + 0] = p.x; X[qq * 4 + 1] = p.y; X[qq * 4 + 2] = p.z; X[qq * 4 + 3] = p.w;
                Y[qq * 4 + 0] = q.x; Y[qq * 4 + 1] = q.y; Y[qq * 4 + 2] = q.z; Y[qq * 4 + 3] = q.w;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int v = v0 + j;
                    X[qq * 4 + j] = v < hi ? a.x[v] : 0;
                    Y[qq * 4 + j] = v < hi ? a.y[v] : 0;
                }
            }
        }
        // the record through the scalar cache: a vector load here would make
        // the wait for it also wait for the points just requested
        const int32_t *rec = reinterpret_cast<const int32_t *>(ws.tinfo(0, 0) + tile);
        ti.seg = scalar_load(rec + 0);
        ti.single = scalar_load(rec + 1);
        ti.start = scalar_load(rec + 2);
        ti.end = scalar_load(rec + 3);
    };
    // one tile's points: the run's extremes in registers, or several
    // instances reduced per instance in LDS
    auto reduce_tile = [&](int tile, const int32_t (&X)[kItems], const int32_t (&Y)[kItems], const TileInfo &ti)
        __attribute__((always_inline)) {
        const int lo = tile * kTile;
        const int hi = min(lo + kTile, n);
        const bool full = hi - lo == kTile;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            // |c| <= bound  <=>  c + bound in [0, 2 bound], modulo 2^32 (points
            // past the end load as 0)
            span = max(span, (uint32_t)X[i] + (uint32_t)kCoordMax2D);
            span = max(span, (uint32_t)Y[i] + (uint32_t)kCoordMax2D);
            nspan = max(nspan, (uint32_t)kCoordMax2D - (uint32_t)X[i]);
            nspan = max(nspan, (uint32_t)kCoordMax2D - (uint32_t)Y[i]);
        }
        if (ti.single) {
            if (ti.seg != cur) {
                if (cur >= 0) flush(tile);
                cur = ti.seg;
                run0 = tile;
                cst = ti.start;
                cen = ti.end;
            }
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                const int v = lo + (i >> 2) * kBlock * 4 + tid * 4 + (i & 3);
                if (!full && v >= hi) continue;
                const uint64_t ck = coord_key(X[i], Y[i]);
                if (ck < kmn) { kmn = ck; imn = v; }
                if (ck > kmx) { kmx = ck; imx = v; }
            }
            return;
        }
        if (cur >= 0) {
            flush(tile);
            cur = -1;
        }
        // several instances in the tile: per-slot LDS reduction
        const int s0 = ti.seg;
        if (tid == 0) sm->s_m = 0;
        __syncthreads();
        for (int b = 0; b <= kTile; b += kBlock) {
            const int j = b + tid;
            bool in = false;
            if (j <= kTile) {
                const int si = s0 + j;
                const int st = si < S ? ws.geo(0, 0)[si].start : n;
                sm->sstart[j] = st;
                in = st < hi;
            }
            const int cnt = __syncthreads_count(in);
            if (tid == 0) sm->s_m += cnt;
            if (cnt < kBlock) break;
        }
        __syncthreads();
        const int m = sm->s_m;
        for (int w0 = 0; w0 < m; w0 += kSlots) {
            const int wn = min(kSlots, m - w0);
            for (int j = tid; j < kSlots; j += kBlock) {
                sm->kmin1[j] = 0; sm->kmin2[j] = ~0ull; sm->kmax1[j] = 0; sm->kmax2[j] = ~0ull;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                const int v = lo + (i >> 2) * kBlock * 4 + tid * 4 + (i & 3);
                if (v >= hi) continue;
                const int sl = slot_of(sm->sstart, m, v);
                if (sl < w0 || sl >= w0 + wn) continue;
                const uint64_t ck = coord_key(X[i], Y[i]);
                atomicMax(&sm->kmin1[sl - w0], ~ck);
                atomicMax(&sm->kmax1[sl - w0], ck);
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                const int v = lo + (i >> 2) * kBlock * 4 + tid * 4 + (i & 3);
                if (v >= hi) continue;
                const int sl = slot_of(sm->sstart, m, v);
                if (sl < w0 || sl >= w0 + wn) continue;
                const uint64_t ck = coord_key(X[i], Y[i]);
                if (~ck == sm->kmin1[sl - w0]) atomicMin(&sm->kmin2[sl - w0], (uint64_t)(uint32_t)v);
                if (ck == sm->kmax1[sl - w0]) atomicMin(&sm->kmax2[sl - w0], (uint64_t)(uint32_t)v);
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                const int v = lo + (i >> 2) * kBlock * 4 + tid * 4 + (i & 3);
                if (v >= hi) continue;
                const int sl = slot_of(sm->sstart, m, v);
                if (sl < w0 || sl >= w0 + wn) continue;
                if ((uint64_t)(uint32_t)v == sm->kmin2[sl - w0]) {
                    sm->rmin[sl - w0][0] = X[i]; sm->rmin[sl - w0][1] = Y[i]; sm->rmin[sl - w0][2] = v;
                }
                if ((uint64_t)(uint32_t)v == sm->kmax2[sl - w0]) {
                    sm->rmax[sl - w0][0] = X[i]; sm->rmax[sl - w0][1] = Y[i]; sm->rmax[sl - w0][2] = v;
                }
            }
            __syncthreads();
            for (int j = tid; j < wn; j += kBlock) {
                const int sl = w0 + j;
                Best bmn, bmx;
                bmn.key1 = sm->kmin1[j]; bmn.key2 = sm->kmin2[j];
                bmn.x = sm->rmin[j][0]; bmn.y = sm->rmin[j][1]; bmn.idx = sm->rmin[j][2]; bmn.cnt = 0;
                bmx.key1 = sm->kmax1[j]; bmx.key2 = sm->kmax2[j];
                bmx.x = sm->rmax[j][0]; bmx.y = sm->rmax[j][1]; bmx.idx = sm->rmax[j][2]; bmx.cnt = 0;
                const bool inside = sm->sstart[sl] >= lo && sm->sstart[sl + 1] <= hi;
                if (inside) {
                    ws.dir0[(s0 + sl) * 2 + 0] = bmn;
                    ws.dir0[(s0 + sl) * 2 + 1] = bmx;
                }
                if (sl == 0) { ws.recF0[tile * 2 + 0] = bmn; ws.recF0[tile * 2 + 1] = bmx; }
                if (sl == m - 1) { ws.recL0[tile * 2 + 0] = bmn; ws.recL0[tile * 2 + 1] = bmx; }
            }
            __syncthreads();
        }
    };
    // software pipelined over the full tiles: the next tile's points are
    // requested before this tile is reduced, unconditionally (the last
    // iteration reloads its own tile), so the wait for this tile's points
    // never waits for them; the input's ragged last tile comes after the loop
    const int tfe = max(tb, min(te, n / kTile));
    int32_t Xn[kItems], Yn[kItems];
    TileInfo tin = {};
    if (tb < tfe) load_tile(tb, Xn, Yn, tin, true);
    for (int tile = tb; tile < tfe; ++tile) {
        int32_t X[kItems], Y[kItems];
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            X[i] = Xn[i];
            Y[i] = Yn[i];
        }
        const TileInfo ti = tin;
        load_tile(min(tile + 1, tfe - 1), Xn, Yn, tin, true);
        reduce_tile(tile, X, Y, ti);
    }
    for (int tile = tfe; tile < te; ++tile) {
        int32_t X[kItems], Y[kItems];
        TileInfo ti;
        load_tile(tile, X, Y, ti, false);
        reduce_tile(tile, X, Y, ti);
    }
    if (cur >= 0) flush(te);
    const bool bad = span > 2u * (uint32_t)kCoordMax2D || nspan > 2u * (uint32_t)kCoordMax2D;
    if (__syncthreads_or(bad) && threadIdx.x == 0) {
        atomicOr(&ctl->error, kErrRange);
        atomicOr(&ctl->setup_error, kErrRange);
    }
    // the largest |coordinate| (plus the bound) of the input, for the FP32
    // filter's static error bound: per wave, then into one of 64 slots (few
    // atomics per address), merged by the extremes' final kernel
    uint32_t cs = max(span, nspan);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) cs = max(cs, (uint32_t)__shfl_xor((int)cs, m));
    if (lane == 0 && cs > (uint32_t)kCoordMax2D) atomicMax(&ctl->cspan_slot[(blockIdx.x * kNW + wv) & 63], cs);
}

// Merge the per-tile partials of one segment over tiles t0 .. t1 (the whole
// block cooperates; every thread gets the result).  In tile t0 the segment is
// the tile's last one, in the later tiles its first one.
// The argmax records of a segment of region R whose points span the tiles
// t0 < t1 of round p (global tile indices): slot 0 is tile t0 (its last
// segment's record if t0 holds several segments, else the record of the run
// that starts there); slot 1 + j is the run head in the j-th range of T tiles
// the segment meets (the round kernel keeps one record per run, at the run's
// first tile); the last slot is tile t1 if it holds several segments.  Only
// t0 and t1 can hold several segments (s0, s1: whether each holds one), so
// a slot is one record load.  Returns the record's tile and array (recF /
// recL), or -1 for a slot without a record.
__device__ __forceinline__ int seg_slot(int T, int t0, int t1, bool s0, bool s1, int k, bool &last) {
    const int nb = t1 / T - t0 / T + 1;
    last = false;
    if (k == 0) {
        last = !s0;
        return t0;
    }
    if (k <= nb) {
        const int b = t0 / T + (k - 1);
        const int st = max(b * T, t0 + 1);
        if (st > t1 || st >= (b + 1) * T || (st == t1 && !s1)) return -1;
        if (st != b * T && s0) return -1;  // same run as t0
        return st;
    }
    if (k == nb + 1 && !s1) return t1;
    return -1;
}

__device__ __forceinline__ int seg_slots(int T, int t0, int t1) { return t1 / T - t0 / T + 3; }

// The extremes records of an instance over tiles t0 < t1, slot by slot as
// for the segments' argmax records (seg_slot): tile t0, the run heads of the
// ranges of T tiles, tile t1 if it holds several instances.
__device__ __forceinline__ void block_merge_ext(const Ws2 &ws, int T, int t0, int t1, Best *red,
                                                Best &mn, Best &mx) {
    const TileInfo *ti = ws.tinfo(0, 0);
    const bool s0 = ti[t0].single != 0, s1 = ti[t1].single != 0;
    Best a0 = best_none(), a1 = best_none();
    const int ns = seg_slots(T, t0, t1);
    // four slots per thread requested at a time, then merged (order-free)
    for (int k0 = threadIdx.x; k0 < ns; k0 += 4 * kBlock) {
        Best c0[4], c1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            c0[u] = best_none();
            c1[u] = best_none();
            bool last;
            const int k = k0 + u * kBlock;
            const int t = k < ns ? seg_slot(T, t0, t1, s0, s1, k, last) : -1;
            if (t >= 0) {
                const Best *rec = last ? ws.recL0 : ws.recF0;
                c0[u] = rec[t * 2 + 0];
                c1[u] = rec[t * 2 + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            best_merge(a0, c0[u]);
            best_merge(a1, c1[u]);
        }
    }
    wave_best(a0);
    wave_best(a1);
    if (lane_id() == 0) {
        red[2 * (threadIdx.x / kWave) + 0] = a0;
        red[2 * (threadIdx.x / kWave) + 1] = a1;
    }
    __syncthreads();
    mn = red[0];
    mx = red[1];
    for (int w = 1; w < kNW; ++w) {
        best_merge(mn, red[2 * w + 0]);
        best_merge(mx, red[2 * w + 1]);
    }
    __syncthreads();
}

// Every instance segment: finish its extremes, write the first-split segment
// (edge a -> a with apex b, so the round splits the points by the line ab) and
// the geometry of its tiles.
__device__ __forceinline__ void phase_extremes_final(const Ws2 &ws, const HullArgs &a, char *smem) {
    Control *ctl = ws.ctl;
    if (ctl->error) return;
    if (blockIdx.x == 0 && threadIdx.x < kWave) {
        uint32_t cs = ctl->cspan_slot[threadIdx.x];
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) cs = max(cs, (uint32_t)__shfl_xor((int)cs, m));
        if (threadIdx.x == 0) ctl->cspan = cs;
    }
    SegSmem *sm = reinterpret_cast<SegSmem *>(smem);
    const int S = ctl->rs[0].s[0];
    for (int s = blockIdx.x; s < S; s += gridDim.x) {
        SegGeo g = ws.geo(0, 0)[s];
        const SegTop tp = ws.top(0, 0)[s];
        const int t0 = g.start / kTile;
        const int t1 = (g.start + g.len - 1) / kTile;
        Best mn, mx;
        if (t0 == t1) {
            mn = ws.dir0[s * 2 + 0];
            mx = ws.dir0[s * 2 + 1];
        } else {
            const int T = max(1, ctl->tper_ext);
            block_merge_ext(ws, T, t0, t1, sm->red, mn, mx);
        }
        // (the first split reads the instance's geometry from this table;
        // its tile records come from the set-up kernel)
        if (threadIdx.x == 0) {
            g.ux = mn.x; g.uy = mn.y;
            g.vx = mn.x; g.vy = mn.y;
            g.fx = mx.x; g.fy = mx.y;
            ws.geo(0, 0)[s] = g;
            SegTop t = tp;
            t.fidx = mx.idx;
            ws.top(0, 0)[s] = t;
            ws.V[tp.uc] = mn.idx;
            ws.hinst[tp.uc] = tp.inst;
        }
    }
}

// ---------------------------------------------------------------------------
// one round over the survivors
// ---------------------------------------------------------------------------
// Every tile of a round is classified, reduced and scattered by one block in
// one pass: the survivors of child c of tile t go to region c at t * kTile
// (a "piece"), so no tile waits for another.  The next round reads its input
// in compacted order through the piece table that the segment kernel builds
// from the tiles' survivor counts (an exclusive scan), which is the order the
// child segments are laid out in.  Tiles are dealt to the resident blocks in
// a fixed stride, with no atomics.  A tile covered by one segment (the common
// case) is processed by each wave on its own quarter; a tile with several
// segments is processed by the whole block in point order.

// items of a thread: v = lo + (i >> 2) * kBlock * 4 + tid * 4 + (i & 3)
__device__ __forceinline__ int item_pos(int lo, int i) {
    return lo + (i >> 2) * kBlock * 4 + (int)threadIdx.x * 4 + (i & 3);
}

// the first split reads the caller's array (index = position)
__device__ __forceinline__ void load_input(const HullArgs &a, int lo, int hi, int32_t (&X)[kItems],
                                           int32_t (&Y)[kItems], int32_t (&I)[kItems]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int qq = 0; qq < kQ; ++qq) {
        const int v0 = lo + qq * kBlock * 4 + tid * 4;
        if (a.vec_ok && v0 + 3 < hi) {
            const i32x4u pa = *reinterpret_cast<const i32x4u *>(a.x + v0);
            const i32x4u pb = *reinterpret_cast<const i32x4u *>(a.y + v0);
            X[qq * 4 + 0] = pa.x; X[qq * 4 + 1] = pa.y; X[qq * 4 + 2] = pa.z; X[qq * 4 + 3] = pa.w;
            Y[qq * 4 + 0] = pb.x; Y[qq * 4 + 1] = pb.y; Y[qq * 4 + 2] = pb.z; Y[qq * 4 + 3] = pb.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int v = v0 + j;
                X[qq * 4 + j] = v < hi ? a.x[v] : 0;
                Y[qq * 4 + j] = v < hi ? a.y[v] : 0;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) I[qq * 4 + j] = v0 + j;
    }
}

// later rounds: the tile's virtual range [lo, hi) of region R, gathered from
// the pieces kA .. kB the previous round wrote.  Returns false (and raises
// an internal error) if the piece table does not fit the tile.
__device__ __forceinline__ bool load_pieces(const Ws2 &ws, int p, int R, int lt, int ntR, int npc,
                                            int lo, int hi, int32_t *pvs, int32_t *pps,
                                            int32_t (&X)[kItems], int32_t (&Y)[kItems],
                                            int32_t (&I)[kItems]) {
    const int tid = threadIdx.x;
    const int32_t *kf = ws.kf(p, R);
    const int kA = kf[lt];
    const int kB = (lt + 1 < ntR) ? kf[lt + 1] : npc - 1;
    const int K = kB - kA + 1;
    const bool ok = kA >= 0 && K >= 1 && K <= kTile + 2 && kB < npc;
    if (ok) {
        const int32_t *pv = ws.pv(p, R) + kA;
        const int32_t *pp = ws.pp(p, R) + kA;
        for (int j = tid; j < K; j += kBlock) {
            pvs[j] = pv[j];
            pps[j] = pp[j];
        }
    }
    __syncthreads();
    const int32_t *sx = ws.px(p, R), *sy = ws.py(p, R), *si = ws.pi(p, R);
    const int64_t cap = ws.cap_pts;
    bool bad = !ok;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int v = item_pos(lo, i);
        X[i] = Y[i] = I[i] = 0;
        if (!ok || v >= hi) continue;
        const int j = slot_of(pvs, K, v);
        const int64_t ph = (int64_t)pps[j] + (v - pvs[j]);
        if (ph < 0 || ph >= cap) { bad = true; continue; }
        X[i] = sx[ph];
        Y[i] = sy[ph];
        I[i] = si[ph];
    }
    if (bad) atomicOr(&ws.ctl->error, kErrInternal);
    return ok;
}

__device__ __forceinline__ uint32_t row_count(uint32_t stbits, int qq) {
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t st = (stbits >> (2 * (qq * 4 + j))) & 3u;
        c += st == 0 ? 1u : (st == 1 ? 0x10000u : 0u);
    }
    return c;
}

// exclusive in-tile ranks of the survivors of both children in point order
// (packed child 0 | child 1 << 16): cnt[qq] before this thread's group of
// row qq, rowbase[qq] before row qq; returns the tile totals
__device__ __forceinline__ uint32_t tile_ranks(uint32_t stbits, uint32_t (&cnt)[kQ],
                                               uint32_t (&rowbase)[kQ], uint32_t *scan) {
    uint32_t tot[kQ];
#pragma unroll
    for (int qq = 0; qq < kQ; ++qq) cnt[qq] = row_count(stbits, qq);
    block_excl_scan<kBlock, kQ>(cnt, tot, scan);
    uint32_t acc = 0;
#pragma unroll
    for (int qq = 0; qq < kQ; ++qq) { rowbase[qq] = acc; acc += tot[qq]; }
    return acc;
}

// exact distance of a point to its child's edge (child 0: u->f, 1: f->v)
__device__ __forceinline__ int64_t child_d(int32_t x, int32_t y, uint32_t st, const int32_t *g) {
    return st == 0 ? cross_i64(x, y, g[0], g[1], g[2], g[3]) : cross_i64(x, y, g[2], g[3], g[4], g[5]);
}

// Round r ends the recursion in one pass when no segment has more than
// fin_cap points and there are at most fin_segs segments (a workgroup takes
// one segment at a time), or, from round 2 on, when no segment has more
// than kFinUnit points and the round holds at most fin_pts points (a
// workgroup takes runs of consecutive segments of up to kFinUnit points
// together); decided alike by every kernel of the round.  Never in round 1,
// whose segments are the split's children, kept as input ranges rather than
// as points.
__device__ __forceinline__ bool fin_each(const Control *ctl, int r, const HullArgs &a) {
    const int p = r & 1;
    const RoundState &rs = ctl->rs[p];
    const int S = rs.s[0] + rs.s[1];
    return S <= a.fin_segs && ctl->maxseg[p] <= a.fin_cap;
}

__device__ __forceinline__ bool fin_mode(const Control *ctl, int r, const HullArgs &a) {
    if (r == 1 || r < a.fin_from || a.fin_cap <= 0) return false;
    const int p = r & 1;
    const RoundState &rs = ctl->rs[p];
    const int S = rs.s[0] + rs.s[1];
    if (S <= 0) return false;
    if (fin_each(ctl, r, a)) return true;
    return r >= 2 && ctl->maxseg[p] <= kFinUnit && (int64_t)rs.n[0] + rs.n[1] <= (int64_t)a.fin_pts;
}


// the 8-bit field c of a packed counter
__device__ __forceinline__ uint32_t field8(uint32_t v, uint32_t c) { return (v >> (8u * c)) & 0xffu; }

// a copy of a wave-uniform value in a vector register (so that a per-lane
// select between two such values needs no scalar operand)
__device__ __forceinline__ int32_t vcopy(int32_t s) {
    int32_t v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// one DPP step of a 64-bit reduction: lanes whose source is outside their
// row, or whose row is masked off, receive the identity (lo, hi)
template <int Ctrl, int RowMask>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v, uint32_t idl, uint32_t idh) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)idl, (int)(uint32_t)v, Ctrl, RowMask, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)idh, (int)(uint32_t)(v >> 32), Ctrl, RowMask, 0xf, false);
    return ((uint64_t)hi << 32) | lo;
}

// maximum / minimum over the wave (row shifts and row broadcasts, no LDS;
// complete in lane 63, returned as a uniform value)
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
    uint64_t o;
    o = dpp_u64<0x111, 0xf>(v, 0u, 0u); v = o > v ? o : v;
    o = dpp_u64<0x112, 0xf>(v, 0u, 0u); v = o > v ? o : v;
    o = dpp_u64<0x114, 0xf>(v, 0u, 0u); v = o > v ? o : v;
    o = dpp_u64<0x118, 0xf>(v, 0u, 0u); v = o > v ? o : v;
    o = dpp_u64<0x142, 0xa>(v, 0u, 0u); v = o > v ? o : v;
    o = dpp_u64<0x143, 0xc>(v, 0u, 0u); v = o > v ? o : v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, kWave - 1);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), kWave - 1);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
    const uint32_t ff = 0xffffffffu;
    uint64_t o;
    o = dpp_u64<0x111, 0xf>(v, ff, ff); v = o < v ? o : v;
    o = dpp_u64<0x112, 0xf>(v, ff, ff); v = o < v ? o : v;
    o = dpp_u64<0x114, 0xf>(v, ff, ff); v = o < v ? o : v;
    o = dpp_u64<0x118, 0xf>(v, ff, ff); v = o < v ? o : v;
    o = dpp_u64<0x142, 0xa>(v, ff, ff); v = o < v ? o : v;
    o = dpp_u64<0x143, 0xc>(v, ff, ff); v = o < v ? o : v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, kWave - 1);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), kWave - 1);
    return ((uint64_t)hi << 32) | lo;
}

// The wave's best point of each class so far in the run: distance W, tie key
// T (its low 32 bits are the index), and (FP32 filter) the estimate below
// which a point cannot reach W.  Offered the lanes' candidates of class k
// (cand: exact distance d > 0 and tie key tk).
// bit i set when item i's two-bit class field (bits 2i, 2i + 1) is 2 or 3
__device__ __forceinline__ uint32_t stb_dropped_mask(uint32_t stb) {
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) m |= ((stb >> (2 * i + 1)) & 1u) << i;
    return m;
}

struct WaveBest {
    uint64_t W[4], T[4];
    float tau[4];
    uint32_t C[4];
};

__device__ __forceinline__ void wave_offer(WaveBest &wb, int k, bool cand, uint64_t d, uint64_t tk, float B) {
    if (!__ballot(cand)) return;
    const uint64_t dm = wave_max_u64(cand ? d : 0ull);
    const uint64_t tm = wave_min_u64((cand && d == dm) ? tk : ~0ull);
    if (dm > wb.W[k] || (dm == wb.W[k] && tm < wb.T[k])) {
        wb.W[k] = dm;
        wb.T[k] = tm;
        // E < fl(fl(W) - 2B) implies d < W (the estimate's error is below
        // 4/5 of B, and fl(W) and the difference round by less than B/5)
        wb.tau[k] = __fsub_rn((float)dm, 2.f * B);
    }
}

// a tile's record with its segment's geometry (u, f, v) when one segment
// covers it
struct TileGeo {
    int32_t seg, single, start, end;
    int32_t ux, uy, fx, fy, vx, vy;
};

// the record of global tile t of round p (uniform), the geometry from the
// segment table (in the first split: u = v = the instance's minimum, f = its
// maximum)
__device__ __forceinline__ TileGeo tile_record(const Ws2 &ws, int p, int t, int nt0) {
    const int R = t < nt0 ? 0 : 1;
    const int32_t *src = reinterpret_cast<const int32_t *>(ws.tinfo(p, R) + (t - (R ? nt0 : 0)));
    TileGeo ti;
    ti.seg = scalar_load(src + 0);
    ti.single = scalar_load(src + 1);
    ti.start = scalar_load(src + 2);
    ti.end = scalar_load(src + 3);
    ti.ux = ti.uy = ti.fx = ti.fy = ti.vx = ti.vy = 0;
    if (ti.single) {
        const int32_t *g = reinterpret_cast<const int32_t *>(ws.geo(p, R) + ti.seg);
        ti.ux = scalar_load(g + 2); ti.uy = scalar_load(g + 3);
        ti.fx = scalar_load(g + 4); ti.fy = scalar_load(g + 5);
        ti.vx = scalar_load(g + 6); ti.vy = scalar_load(g + 7);
    }
    return ti;
}

// The one-segment tiles may emit their survivors in any order, so their
// waves work on contiguous quarters of the tile with 64-lane runs: lane l of
// wave w holds items v = lo + 512 w + 64 i + l (gathered loads and the
// per-item scatter are dense per instruction); the first split reads the
// caller's array as 4-point vectors, v = lo + 512 w + 256 (i / 4) + 4 l + i % 4.
__device__ __forceinline__ int fast_pos(int lo, int i) {
    return lo + (int)(threadIdx.x / kWave) * 512 + i * kWave + lane_id();
}
__device__ __forceinline__ int fast_pos_init(int lo, int i) {
    return lo + (int)(threadIdx.x / kWave) * 512 + (i >> 2) * 256 + lane_id() * 4 + (i & 3);
}

// A full tile's points, every lane's four-point vectors in range: no
// per-lane conditions, so that loads of the next tile issued before this
// one is classified need not wait for anything.
__device__ __forceinline__ void load_full_wave(const HullArgs &a, int lo, int32_t (&X)[kItems],
                                               int32_t (&Y)[kItems]) {
#pragma unroll
    for (int qq = 0; qq < kQ; ++qq) {
        const int v0 = fast_pos_init(lo, qq * 4);
        const i32x4u pa = *reinterpret_cast<const i32x4u *>(a.x + v0);
        const i32x4u pb = *reinterpret_cast<const i32x4u *>(a.y + v0);
        X[qq * 4 + 0] = pa.x; X[qq * 4 + 1] = pa.y; X[qq * 4 + 2] = pa.z; X[qq * 4 + 3] = pa.w;
        Y[qq * 4 + 0] = pb.x; Y[qq * 4 + 1] = pb.y; Y[qq * 4 + 2] = pb.z; Y[qq * 4 + 3] = pb.w;
    }
}

__device__ __forceinline__ uint32_t load_input_wave(const HullArgs &a, int lo, int hi,
                                                    int32_t (&X)[kItems], int32_t (&Y)[kItems]) {
    uint32_t vm = 0;
#pragma unroll
    for (int qq = 0; qq < kQ; ++qq) {
        const int v0 = fast_pos_init(lo, qq * 4);
        if (a.vec_ok && v0 + 3 < hi) {
            const i32x4u pa = *reinterpret_cast<const i32x4u *>(a.x + v0);
            const i32x4u pb = *reinterpret_cast<const i32x4u *>(a.y + v0);
            X[qq * 4 + 0] = pa.x; X[qq * 4 + 1] = pa.y; X[qq * 4 + 2] = pa.z; X[qq * 4 + 3] = pa.w;
            Y[qq * 4 + 0] = pb.x; Y[qq * 4 + 1] = pb.y; Y[qq * 4 + 2] = pb.z; Y[qq * 4 + 3] = pb.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int v = v0 + j;
                X[qq * 4 + j] = v < hi ? a.x[v] : 0;
                Y[qq * 4 + j] = v < hi ? a.y[v] : 0;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) vm |= (v0 + j < hi ? 1u : 0u) << (qq * 4 + j);
    }
    return vm;
}

// later rounds: the pieces [kA, kA + K) of the previous round that hold tile
// lt of region R (uniform values, read through the scalar cache); false if
// the piece table is malformed
__device__ __forceinline__ bool piece_range(const Ws2 &ws, int p, int R, int lt, int ntR, int npc,
                                            int &kA, int &K) {
    const int32_t *kf = ws.kf(p, R);
    kA = scalar_load(kf + lt);
    const int kB = (lt + 1 < ntR) ? scalar_load(kf + lt + 1) : npc - 1;
    K = kB - kA + 1;
    return kA >= 0 && K >= 1 && K <= kTile + 2 && kB < npc;
}

// gather the tile's virtual range [lo, hi) from its piece table in LDS (the
// virtual and physical starts of K pieces); returns the valid-item mask
__device__ __forceinline__ uint32_t gather_pieces(const Ws2 &ws, int p, int R, int K, int lo, int hi,
                                                  const int32_t *pvs, const int32_t *pps,
                                                  int32_t (&X)[kItems], int32_t (&Y)[kItems],
                                                  int32_t (&I)[kItems]) {
    // a uniform base (the plane) and a 32-bit offset per item (the planes
    // hold fewer than 2^31 points); the pieces of a tile need not be
    // physically in order (the round after the split writes side 1 of a
    // tile backward from the end of its slot)
    const int64_t cap = ws.cap_pts;
    const int32_t *sx = ws.px(p, R), *sy = ws.py(p, R), *si = ws.pi(p, R);
    uint32_t vm = 0;
    bool bad = false;
    // the piece of the lane's first item, then a forward walk with the next
    // piece's start and the current piece's offset kept in registers
    int j = 0;
    const int w0 = fast_pos(lo, 0);
    if (K > 1) j = slot_of(pvs, K, min(w0, hi - 1));
    int nextv = j + 1 < K ? pvs[j + 1] : INT32_MAX;
    int delta = pps[j] - pvs[j];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const int v = fast_pos(lo, i);
        X[i] = Y[i] = I[i] = 0;
        if (v >= hi) continue;
        while (v >= nextv) {
            ++j;
            nextv = j + 1 < K ? pvs[j + 1] : INT32_MAX;
            delta = pps[j] - pvs[j];
        }
        const int off = v + delta;  // physical position
        if (off < 0 || (int64_t)off >= cap) { bad = true; continue; }
        X[i] = sx[(uint32_t)off];
        Y[i] = sy[(uint32_t)off];
        I[i] = si[(uint32_t)off];
        vm |= 1u << i;
    }
    if (bad) atomicOr(&ws.ctl->error, kErrInternal);
    return vm;
}

// later rounds, without prefetch: the piece table to LDS, then the gather;
// returns the valid-item mask, or 0xffffffff if the table does not fit
__device__ __forceinline__ uint32_t load_pieces_wave(const Ws2 &ws, int p, int R, int lt, int ntR,
                                                     int npc, int lo, int hi, int32_t *pvs,
                                                     int32_t *pps, int32_t (&X)[kItems],
                                                     int32_t (&Y)[kItems], int32_t (&I)[kItems]) {
    const int tid = threadIdx.x;
    int kA, K;
    const bool ok = piece_range(ws, p, R, lt, ntR, npc, kA, K);
    __syncthreads();  // earlier readers of this table buffer are done
    if (ok) {
        const int32_t *pv = ws.pv(p, R) + kA;
        const int32_t *pp = ws.pp(p, R) + kA;
        for (int j = tid; j < K; j += kBlock) {
            pvs[j] = pv[j];
            pps[j] = pp[j];
        }
    }
    __syncthreads();
    if (!ok) {
        atomicOr(&ws.ctl->error, kErrInternal);
        return 0xffffffffu;
    }
    return gather_pieces(ws, p, R, K, lo, hi, pvs, pps, X, Y, I);
}

// The one-segment tiles of a round.  Every block takes a contiguous range of
// T tiles (the segment kernel finds the argmax record of a run at the run's
// first tile in each range, so it needs T).  The tiles are software
// pipelined: the next tile's record and piece table are read while this tile
// is classified, and its points are loaded before this tile's survivors are
// stored (a load issued after a burst of stores waits for them, since the
// wave's memory counter retires in order).
template <int MODE>
__device__ __forceinline__ void phase_round_fast(const Ws2 &ws, const HullArgs &a, int r, char *smem) {
    FastSmem *sm = reinterpret_cast<FastSmem *>(smem);
    uint32_t *stat = sm->stat;
    Control *ctl = ws.ctl;
    const int p = r & 1, q = p ^ 1;
    const RoundState *rs = &ctl->rs[p];
    const int n0 = rs->n[0], n1 = rs->n[1];
    const int S0 = rs->s[0];
    const int npc0 = rs->npc[0], npc1 = rs->npc[1];
    const int nt0 = (n0 + kTile - 1) / kTile, nt1 = (n1 + kTile - 1) / kTile;
    const int ntiles = nt0 + nt1;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
    // output planes of this parity: [child][x, y, index][cap]
    int32_t *const obase = ws.px(q, 0);
    const int64_t cap = ws.cap_pts;

    uint32_t ntests = 0, nfall = 0, ncand = 0;
    uint32_t acc0 = 0, acc1 = 0;  // survivors written by this block (thread 0)
    bool oob = false;
    // the multi-segment tiles of the next round are listed afresh by the
    // segment kernel that follows
    if (fin_mode(ctl, r, a)) return;  // the multi-segment kernel finishes the segments
    const int T = (ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
    if (blockIdx.x == 0 && tid == 0) {
        ctl->rs[q].nmulti = 0;
        ctl->tper[p] = T;
        ctl->maxseg[q] = 0;
    }
    const int tb = blockIdx.x * T, te = min(tb + T, ntiles);
    const float c2 = MODE ? coord_c2(ctl) : 0.f;
    // A run: consecutive one-segment tiles of one segment in this block.
    // Each wave keeps the best point of each child of the run as uniform
    // values; a lane's point is compared exactly only when it reaches it.
    WaveBest wb;
    auto wb_reset = [&]() {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            wb.W[k] = 0;
            wb.T[k] = ~0ull;
            wb.tau[k] = -INFINITY;
            wb.C[k] = 0;
        }
    };
    wb_reset();
    int cur = -1, run0 = 0, run_lo = 0, run_hi = 0, seg_st = 0, seg_en = 0;
    // the current tile's record and, when prefetched, its points
    TileGeo tc;
    tc.single = 0;
    if (tb < te) tc = tile_record(ws, p, tb, nt0);
    uint32_t vm = 0;
    bool have = false;
    // One tile; the points of the next one go to the other register set (the
    // loop below alternates the two sets, so no copy waits for the loads).
    // Returns true after the last tile.
    auto step = [&](int tile, int32_t(&X)[kItems], int32_t(&Y)[kItems], int32_t(&I)[kItems],
                    int32_t(&Xn)[kItems], int32_t(&Yn)[kItems], int32_t(&In)[kItems])
        __attribute__((always_inline)) -> bool {
        // tile >= te only closes the last run (a block past the last tile
        // has tb > te)
        const bool past = tile >= te;
        const int R = tile < nt0 ? 0 : 1;
        const int lt = tile - (R ? nt0 : 0);
        const int NR = R ? n1 : n0;
        const int lo = lt * kTile;
        const int hi = min(lo + kTile, NR);
        TileGeo ti = tc;
        if (past) ti.single = 0;
        const int gseg = (R ? S0 : 0) + ti.seg;
        if (cur >= 0 && (!ti.single || gseg != cur)) {
            // the run ends: merge the waves' bests, record it at its first tile
            if (lane == 0) {
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    RunBest rr;
                    rr.k1 = wb.W[c];
                    rr.k2 = wb.T[c];
                    rr.cnt = (int32_t)wb.C[c];
                    sm->wrb[wv][c] = rr;
                }
            }
            __syncthreads();
            if (tid < 2) {
                RunBest m = sm->wrb[0][tid];
#pragma unroll
                for (int w = 1; w < kNW; ++w) rb_merge(m, sm->wrb[w][tid]);
                Best b;
                b.key1 = m.k1;
                b.key2 = m.k2;
                b.cnt = m.cnt;
                b.idx = m.k1 ? (int32_t)(uint32_t)m.k2 : 0;
                b.x = b.y = 0;  // filled in by the segment kernel for the winner
                if (seg_st >= run_lo && seg_en <= run_hi) ws.adir[cur * 2 + tid] = b;
                ws.recF[run0 * 2 + tid] = b;
                ws.recL[run0 * 2 + tid] = b;
            }
            __syncthreads();
            wb_reset();
            cur = -1;
        }
        if (past) return true;
        // the next tile's record (scalar loads, consumed a tile later)
        const bool nxt = tile + 1 < te;
        TileGeo tn;
        tn.single = 0;
        if (nxt) tn = tile_record(ws, p, tile + 1, nt0);
        if (!ti.single) {  // uniform: the multi-segment kernel takes it
            tc = tn;
            have = false;
            return false;
        }
        if (cur < 0) {
            cur = gseg;
            run0 = tile;
            run_lo = lo;
            seg_st = ti.start;
            seg_en = ti.end;
        }
        run_hi = hi;
        const int buf = tile & 1;  // LDS buffers of piece tables and wave counts
        if (!have) {
            vm = load_pieces_wave(ws, p, R, lt, R ? nt1 : nt0, R ? npc1 : npc0, lo, hi, sm->pvs[buf],
                                  sm->pps[buf], X, Y, I);
            if (vm == 0xffffffffu) {
                tc = tn;
                return false;
            }
            // wait for these loads here: after the join, only the prefetched
            // loads are outstanding, behind this block's stores
#pragma unroll
            for (int i = 0; i < kItems; ++i) asm volatile("" ::"v"(X[i]), "v"(Y[i]), "v"(I[i]));
        }
        // the next tile's piece table: up to two entries per thread, read now
        // into registers and put into the other LDS buffer after classifying
        const int Rn = tile + 1 < nt0 ? 0 : 1;
        const int ltn = tile + 1 - (Rn ? nt0 : 0);
        int kAn = 0, Kn = 0;
        bool pre = nxt && tn.single;
        int32_t pv0 = 0, pp0 = 0, pv1 = 0, pp1 = 0;
        if (pre) {
            pre = piece_range(ws, p, Rn, ltn, Rn ? nt1 : nt0, Rn ? npc1 : npc0, kAn, Kn) &&
                  Kn <= 2 * kBlock;
            if (pre) {
                const int32_t *pv = ws.pv(p, Rn) + kAn, *pp = ws.pp(p, Rn) + kAn;
                if (tid < Kn) { pv0 = pv[tid]; pp0 = pp[tid]; }
                if (tid + kBlock < Kn) { pv1 = pv[tid + kBlock]; pp1 = pp[tid + kBlock]; }
            }
        }
        // per item two bits: 0, 1 = child, 2 = dropped (3 = undecided in FP32,
        // only until the exact pass below)
        uint32_t stb = 0;
        uint32_t total;       // the tile's survivors (packed child 0 | child 1 << 16)
        uint32_t bw0, bw1;    // this wave's first in-tile rank in each child
        {
            // one segment covers the tile: uniform geometry, every wave on its own
            const int ux = ti.ux, uy = ti.uy, fx = ti.fx, fy = ti.fy, vx = ti.vx, vy = ti.vy;
            const int e0x = fx - ux, e0y = fy - uy, e1x = vx - fx, e1y = vy - fy;
            // items that may be a child's farthest point: resolved once per
            // tile and child below
            uint32_t fl = 0;
            float B0 = 0.f, B1 = 0.f;
            if (MODE == 0) {
#pragma unroll
                for (int i = 0; i < kItems; ++i) {
                    const bool valid = (vm >> i) & 1u;
                    const int64_t d0 = cross_i64(X[i], Y[i], ux, uy, fx, fy);
                    const int64_t d1 = cross_i64(X[i], Y[i], fx, fy, vx, vy);
                    const bool o0 = valid && d0 > 0;
                    const bool o1 = valid && !o0 && d1 > 0;
                    stb |= (o0 ? 0u : (o1 ? 1u : 2u)) << (2 * i);
                    const uint64_t d = (uint64_t)(o0 ? d0 : d1);
                    const bool need = (o0 & (d >= wb.W[0])) | (o1 & (d >= wb.W[1]));
                    fl |= (need ? 1u : 0u) << i;
                }
            } else {
                // FP32 with one bound per child edge for every point (the
                // largest coordinate bounds the differences); undecided items
                // are redone in int64 and are argmax candidates; a decided
                // survivor is one when its estimate reaches its child's
                // threshold
                B0 = static_bound(e0x, e0y, c2);
                B1 = static_bound(e1x, e1y, c2);
                uint32_t und = 0, cand = 0;
#pragma unroll
                for (int i = 0; i < kItems; ++i) {
                    const bool valid = (vm >> i) & 1u;
                    const float e0 = cross_f32_nb(X[i], Y[i], ux, uy, e0x, e0y);
                    const float e1 = cross_f32_nb(X[i], Y[i], fx, fy, e1x, e1y);
                    uint32_t sti = e0 > B0 ? 0u : (!(e0 < -B0) ? 3u : (e1 > B1 ? 1u : (e1 < -B1 ? 2u : 3u)));
                    sti = valid ? sti : 2u;
                    stb |= sti << (2 * i);
                    und |= (sti == 3 ? 1u : 0u) << i;
                    const bool c = ((sti == 0) & (e0 >= wb.tau[0])) | ((sti == 1) & (e1 >= wb.tau[1]));
                    cand |= (c ? 1u : 0u) << i;
                }
                // exact pass over the undecided items (rare): both signs in int64
                if (__ballot(und != 0)) {
#pragma unroll
                    for (int i = 0; i < kItems; ++i) {
                        if (!((und >> i) & 1u)) continue;
                        const int32_t x = X[i], y = Y[i];
                        const float e0 = cross_f32_nb(x, y, ux, uy, e0x, e0y);
                        const bool o0 = cross_i64(x, y, ux, uy, fx, fy) > 0;
                        const bool o1 = !o0 && cross_i64(x, y, fx, fy, vx, vy) > 0;
                        nfall += ((e0 > B0 || e0 < -B0) ? 0u : 1u) + (o0 ? 0u : 1u);
                        stb ^= ((o0 ? 0u : (o1 ? 1u : 2u)) ^ 3u) << (2 * i);
                    }
                }
                // (undecided items may have been dropped by the exact pass)
                fl = (und | cand) & ~stb_dropped_mask(stb);
            }
            if (__ballot(fl != 0)) {
                // each lane's best flagged item of each child, then the wave's;
                // the edges are made opaque so that the distances are
                // recomputed here, not kept alive from the classification
                int gux = ux, guy = uy, gfx = fx, gfy = fy, g0x = e0x, g0y = e0y, g1x = e1x, g1y = e1y;
                asm volatile("" : "+v"(gux), "+v"(guy), "+v"(gfx), "+v"(gfy), "+v"(g0x), "+v"(g0y), "+v"(g1x),
                             "+v"(g1y));
                uint64_t bd[2] = {0, 0}, bt[2] = {~0ull, ~0ull};
#pragma unroll
                for (int i = 0; i < kItems; ++i) {
                    if (!((fl >> i) & 1u)) continue;
                    const bool c1 = ((stb >> (2 * i)) & 3u) == 1u;
                    const int px0 = c1 ? gfx : gux, py0 = c1 ? gfy : guy;
                    const int cx = c1 ? g1x : g0x, cy = c1 ? g1y : g0y;
                    const uint64_t d = (uint64_t)((int64_t)(X[i] - px0) * (int64_t)cy - (int64_t)(Y[i] - py0) * (int64_t)cx);
                    const uint64_t tk = tie_key(X[i], Y[i], I[i], cx, cy);
                    const uint64_t od = c1 ? bd[1] : bd[0], ot = c1 ? bt[1] : bt[0];
                    const bool better = d > od || (d == od && tk < ot);
                    bd[0] = (better && !c1) ? d : bd[0];
                    bt[0] = (better && !c1) ? tk : bt[0];
                    bd[1] = (better && c1) ? d : bd[1];
                    bt[1] = (better && c1) ? tk : bt[1];
                }
                if (MODE != 0) ncand += (uint32_t)__popc(fl);
                wave_offer(wb, 0, bd[0] != 0, bd[0], bt[0], B0);
                wave_offer(wb, 1, bd[1] != 0, bd[1], bt[1], B1);
            }
            // the lane's survivors per child: fields 00 and 01 of stb
            const uint32_t lc0 = (uint32_t)__popc(~(stb | (stb >> 1)) & 0x5555u);
            const uint32_t lc1 = (uint32_t)__popc(stb & ~(stb >> 1) & 0x5555u);
            if (MODE != 0) ntests += 2u * (uint32_t)__popc(vm) - lc0;
            const uint32_t wt = wave_sum(lc0 | (lc1 << 16));
            wb.C[0] += wt & 0xffffu;
            wb.C[1] += wt >> 16;
            if (lane == 0) sm->wcnt[buf][wv] = wt;
            if (pre) {
                int32_t *pvs = sm->pvs[buf ^ 1], *pps = sm->pps[buf ^ 1];
                if (tid < Kn) { pvs[tid] = pv0; pps[tid] = pp0; }
                if (tid + kBlock < Kn) { pvs[tid + kBlock] = pv1; pps[tid + kBlock] = pp1; }
            }
            __syncthreads();
            // any order inside the tile keeps the children contiguous: wave
            // order, then item, then lane (each store instruction is dense)
            uint32_t base = 0;
            total = 0;
#pragma unroll
            for (int w = 0; w < kNW; ++w) {
                const uint32_t c = sm->wcnt[buf][w];
                base += (w < wv) ? c : 0u;
                total += c;
            }
            bw0 = base & 0xffffu;
            bw1 = base >> 16;
        }
        // the next tile's points, before this tile's stores
        uint32_t vmn = 0;
        if (pre) {
            const int lon = ltn * kTile;
            const int hin = min(lon + kTile, Rn ? n1 : n0);
            vmn = gather_pieces(ws, p, Rn, Kn, lon, hin, sm->pvs[buf ^ 1], sm->pps[buf ^ 1], Xn, Yn, In);
        }
        // scatter: child c of this tile goes to region c at tile * kTile; a
        // survivor's rank is its wave's base plus the set lanes below it.
        // Every lane stores every item (the others into the last tile slot of
        // the planes, which no tile uses), so the number of stores after the
        // next tile's loads is fixed and waiting for those loads does not
        // wait for the stores.
        const int64_t pbase = (int64_t)tile * kTile;
        {
            const bool fits = pbase + kTile <= cap - kTile;  // else all to the sink
            oob |= !fits;
            int32_t *const sink = obase + (cap - kTile) + lane;
            int32_t *const ob = fits ? obase + pbase : sink;
            const int64_t creg = fits ? 3 * cap : 0;  // child 1's planes follow child 0's
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                const uint32_t sti = (stb >> (2 * i)) & 3u;
                const uint64_t m0 = __ballot(sti == 0), m1 = __ballot(sti == 1);
                const uint32_t e = sti == 0 ? bw0 + lanes_below(m0) : bw1 + lanes_below(m1);
                int32_t *d = (sti < 2 && fits) ? ob + (sti ? creg : (int64_t)0) + e : sink;
                d[0] = X[i];
                d[cap] = Y[i];
                d[2 * cap] = I[i];
                bw0 += (uint32_t)__popcll(m0);
                bw1 += (uint32_t)__popcll(m1);
            }
        }
        if (tid == 0) {
            ws.tcnt(p)[tile] = total;
            acc0 += total & 0xffffu;
            acc1 += total >> 16;
        }
        vm = vmn;
        have = pre;
        tc = tn;
        return false;
    };
    int32_t XA[kItems], YA[kItems], IA[kItems], XB[kItems], YB[kItems], IB[kItems];
    for (int tile = tb;; tile += 2) {
        if (step(tile, XA, YA, IA, XB, YB, IB)) break;
        if (step(tile + 1, XB, YB, IB, XA, YA, IA)) break;
    }
    if (oob) atomicOr(&ctl->error, kErrInternal);
    if (tid == 0 && (acc0 | acc1)) {
        atomicAdd(&ctl->nacc[p][0][blockIdx.x % kAccSlots], acc0);
        atomicAdd(&ctl->nacc[p][1][blockIdx.x % kAccSlots], acc1);
    }
    if (MODE != 0) {
        if (tid == 0) { stat[0] = 0; stat[1] = 0; stat[2] = 0; }
        __syncthreads();
        const uint32_t t = wave_sum(ntests), f = wave_sum(nfall), c = wave_sum(ncand);
        if (lane == 0) {
            atomicAdd(&stat[0], t);
            atomicAdd(&stat[1], f);
            atomicAdd(&stat[2], c);
        }
        __syncthreads();
        if (tid == 0 && stat[0]) {
            atomicAdd(&ctl->fstat[0][blockIdx.x % kAccSlots], (unsigned long long)stat[0]);
            atomicAdd(&ctl->fstat[1][blockIdx.x % kAccSlots], (unsigned long long)stat[1]);
            atomicAdd(&ctl->fstat[2][blockIdx.x % kAccSlots], (unsigned long long)stat[2]);
        }
    }
}

// ---------------------------------------------------------------------------
// the first split, read-only
// ---------------------------------------------------------------------------
// Algorithm 4's first split tests every point of an instance against the line
// through its extremes a (lexicographic minimum) and b (maximum):
// d = (p - a) x (b - a) > 0 puts the point in child 0 (outside a -> b), d < 0 in
// child 1 (outside b -> a), and d = 0 drops it.  This pass writes no point: it
// finds each child's farthest point (its apex) and size, and the round after
// it reads the caller's array again, taking each point's side from the same
// sign (the children are kept as the instance's input range).
struct SplitSmem {
    uint32_t stat[4];
    RunBest wrb[kNW][2];
};

// the run's argmax records of the split (2 children) or of the round after it
// (2 sides x 2 children): wave reduction, then one thread per record
template <int NREC>
__device__ __forceinline__ void close_run_records(const Ws2 &ws, RunBest (&rb)[NREC], RunBest (*wrb)[NREC],
                                                  int cur, int S0, int nt, int run0, bool whole) {
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
#pragma unroll
    for (int c = 0; c < NREC; ++c) wave_rb63(rb[c]);
    if (lane == kWave - 1) {
#pragma unroll
        for (int c = 0; c < NREC; ++c) wrb[wv][c] = rb[c];
    }
    __syncthreads();
    if (tid < NREC) {
        RunBest m = wrb[0][tid];
#pragma unroll
        for (int w = 1; w < kNW; ++w) rb_merge(m, wrb[w][tid]);
        Best b;
        b.key1 = m.k1;
        b.key2 = m.k2;
        b.cnt = m.cnt;
        b.idx = m.k1 ? (int32_t)(uint32_t)m.k2 : 0;
        b.x = b.y = 0;  // filled in by the segment kernel for the winner
        // record tid: side s = tid / 2 (region s of the segment tables, tiles
        // of region 1 after the nt of region 0), child c = tid % 2
        const int sd = tid >> 1, c = tid & 1;
        const int g = (sd ? S0 : 0) + cur, rt = (sd ? nt : 0) + run0;
        if (whole) ws.adir[g * 2 + c] = b;
        ws.recF[rt * 2 + c] = b;
        ws.recL[rt * 2 + c] = b;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NREC; ++c) rb[c] = rb_none();
}

// offer a candidate with its precomputed tie key
__device__ __forceinline__ void rb_offer_k(RunBest &b, bool take, uint64_t d, uint64_t k2) {
    const bool better = take && (d > b.k1 || (d == b.k1 && k2 < b.k2));
    b.k1 = better ? d : b.k1;
    b.k2 = better ? k2 : b.k2;
}

// the block's filter counters into the control block
__device__ __forceinline__ void flush_filter_stats(Control *ctl, uint32_t *stat, uint32_t ntests, uint32_t nfall,
                                                   uint32_t ncand) {
    const int tid = threadIdx.x, lane = lane_id();
    if (tid == 0) { stat[0] = 0; stat[1] = 0; stat[2] = 0; }
    __syncthreads();
    const uint32_t t = wave_sum(ntests), f = wave_sum(nfall), c = wave_sum(ncand);
    if (lane == 0) {
        atomicAdd(&stat[0], t);
        atomicAdd(&stat[1], f);
        atomicAdd(&stat[2], c);
    }
    __syncthreads();
    if (tid == 0 && stat[0]) {
        atomicAdd(&ctl->fstat[0][blockIdx.x % kAccSlots], (unsigned long long)stat[0]);
        atomicAdd(&ctl->fstat[1][blockIdx.x % kAccSlots], (unsigned long long)stat[1]);
        atomicAdd(&ctl->fstat[2][blockIdx.x % kAccSlots], (unsigned long long)stat[2]);
    }
}

template <int MODE>
__device__ __forceinline__ void phase_split(const Ws2 &ws, const HullArgs &a, char *smem) {
    SplitSmem *sm = reinterpret_cast<SplitSmem *>(smem);
    Control *ctl = ws.ctl;
    const int n = ctl->rs[0].n[0];
    const int ntiles = (n + kTile - 1) / kTile;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
    if (fin_mode(ctl, 0, a)) return;  // the multi-segment kernel finishes the segments
    const int T = (ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
    if (blockIdx.x == 0 && tid == 0) {
        ctl->rs[1].nmulti = 0;
        ctl->tper[0] = T;
        ctl->maxseg[1] = 0;
    }
    const int tb = blockIdx.x * T, te = min(tb + T, ntiles);
    const float c2 = MODE ? coord_c2(ctl) : 0.f;
    // each wave's best point of each child in the run (uniform values); a
    // lane's point is compared exactly only when it reaches it
    WaveBest wb;
    auto wb_reset = [&]() {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            wb.W[k] = 0;
            wb.T[k] = ~0ull;
            wb.tau[k] = -INFINITY;
            wb.C[k] = 0;
        }
    };
    wb_reset();
    int cur = -1, run0 = 0, run_lo = 0, run_hi = 0, seg_st = 0, seg_en = 0;
    uint32_t acc0 = 0, acc1 = 0, ntests = 0, nfall = 0, ncand = 0;

    auto close_run = [&]() __attribute__((always_inline)) {
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                RunBest r;
                r.k1 = wb.W[k];
                r.k2 = wb.T[k];
                r.cnt = (int32_t)wb.C[k];
                sm->wrb[wv][k] = r;
            }
        }
        __syncthreads();
        if (tid < 2) {
            RunBest m = sm->wrb[0][tid];
#pragma unroll
            for (int w = 1; w < kNW; ++w) rb_merge(m, sm->wrb[w][tid]);
            Best b;
            b.key1 = m.k1;
            b.key2 = m.k2;
            b.cnt = m.cnt;
            b.idx = m.k1 ? (int32_t)(uint32_t)m.k2 : 0;
            b.x = b.y = 0;  // filled in by the segment kernel for the winner
            if (seg_st >= run_lo && seg_en <= run_hi) ws.adir[cur * 2 + tid] = b;
            ws.recF[run0 * 2 + tid] = b;
            ws.recL[run0 * 2 + tid] = b;
        }
        __syncthreads();
        wb_reset();
        cur = -1;
    };
    // one tile whose points are in X, Y (valid mask vm)
    auto process = [&](int tile, const TileGeo &ti, const int32_t (&X)[kItems], const int32_t (&Y)[kItems],
                       uint32_t vm) __attribute__((always_inline)) {
        const int lo = tile * kTile, hi = min(lo + kTile, n);
        // this tile's loads end here on every path (also for a tile that is
        // skipped), so the loads issued for the next tile never count as
        // pending where its registers are written again
#pragma unroll
        for (int i = 0; i < kItems; ++i) asm volatile("" ::"v"(X[i]), "v"(Y[i]));
        if (cur >= 0 && (!ti.single || ti.seg != cur)) close_run();
        if (!ti.single) return;  // the multi-segment kernel takes it
        if (cur < 0) {
            cur = ti.seg;
            run0 = tile;
            run_lo = lo;
            seg_st = ti.start;
            seg_en = ti.end;
        }
        run_hi = hi;
        // the instance's extremes: u = v = a, f = b
        const int ax = ti.ux, ay = ti.uy, bx = ti.fx, by = ti.fy;
        const int ex = bx - ax, ey = by - ay;
        uint32_t m0 = 0, m1 = 0;  // the items of child 0 / child 1
        uint32_t fl = 0;          // items that may be a child's farthest point
        float B = 0.f;
        if (MODE == 0) {
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                const bool valid = (vm >> i) & 1u;
                const int64_t d = cross_i64(X[i], Y[i], ax, ay, bx, by);
                const bool o0 = valid && d > 0, o1 = valid && d < 0;
                m0 |= (o0 ? 1u : 0u) << i;
                m1 |= (o1 ? 1u : 0u) << i;
                const uint64_t dd = (uint64_t)(o0 ? d : -d);
                const bool need = (o0 & (dd >= wb.W[0])) | (o1 & (dd >= wb.W[1]));
                fl |= (need ? 1u : 0u) << i;
            }
        } else {
            // FP32 estimates with one bound for every point; a point is
            // compared exactly when its estimate reaches its child's
            // threshold (its exact distance may then reach the child's best)
            B = static_bound(ex, ey, c2);
            uint32_t und = 0, cand = 0;
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                const bool valid = (vm >> i) & 1u;
                const float e = cross_f32_nb(X[i], Y[i], ax, ay, ex, ey);
                const bool p0 = valid && e > B, n0 = valid && e < -B;
                cand |= (((p0 & (e >= wb.tau[0])) | (n0 & (-e >= wb.tau[1]))) ? 1u : 0u) << i;
                m0 |= (p0 ? 1u : 0u) << i;
                m1 |= (n0 ? 1u : 0u) << i;
                und |= (valid && !p0 && !n0 ? 1u : 0u) << i;
            }
            ntests += (uint32_t)__popc(vm);
            // undecided signs (rare): exact, and always argmax candidates
            if (__ballot(und != 0)) {
#pragma unroll
                for (int i = 0; i < kItems; ++i) {
                    if (!((und >> i) & 1u)) continue;
                    const int64_t d = cross_i64(X[i], Y[i], ax, ay, bx, by);
                    m0 |= (d > 0 ? 1u : 0u) << i;
                    m1 |= (d < 0 ? 1u : 0u) << i;
                }
                nfall += (uint32_t)__popc(und);
            }
            // (undecided items may have been dropped by the exact pass)
            fl = (und | cand) & (m0 | m1);
        }
        if (__ballot(fl != 0)) {
            // each lane's best flagged item of each child, then the wave's;
            // the edge is made opaque so that the distances are recomputed
            // here, not kept alive from the classification above
            int gax = ax, gay = ay, gex = ex, gey = ey;
            asm volatile("" : "+v"(gax), "+v"(gay), "+v"(gex), "+v"(gey));
            uint64_t bd[2] = {0, 0}, bt[2] = {~0ull, ~0ull};
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                if (!((fl >> i) & 1u)) continue;
                const bool c1 = (m1 >> i) & 1u;
                const int64_t d = (int64_t)(X[i] - gax) * (int64_t)gey - (int64_t)(Y[i] - gay) * (int64_t)gex;
                const uint64_t dd = (uint64_t)(c1 ? -d : d);
                const uint64_t tk = tie_key(X[i], Y[i], fast_pos_init(lo, i), c1 ? -gex : gex, c1 ? -gey : gey);
                const uint64_t od = c1 ? bd[1] : bd[0], ot = c1 ? bt[1] : bt[0];
                const bool better = dd > od || (dd == od && tk < ot);
                bd[0] = (better && !c1) ? dd : bd[0];
                bt[0] = (better && !c1) ? tk : bt[0];
                bd[1] = (better && c1) ? dd : bd[1];
                bt[1] = (better && c1) ? tk : bt[1];
            }
            if (MODE != 0) ncand += (uint32_t)__popc(fl);
            wave_offer(wb, 0, bd[0] != 0, bd[0], bt[0], B);
            wave_offer(wb, 1, bd[1] != 0, bd[1], bt[1], B);
        }
        const uint32_t lc0 = (uint32_t)__popc(m0), lc1 = (uint32_t)__popc(m1);
        acc0 += lc0;
        acc1 += lc1;
        const uint32_t w = wave_sum(lc0 | (lc1 << 16));
        wb.C[0] += w & 0xffffu;
        wb.C[1] += w >> 16;
    };
    // software pipelined over the full tiles: the next tile's record and
    // points are requested before this tile is classified, unconditionally
    // (the last iteration reloads its own tile; a tile of several instances
    // is loaded and skipped), so that the wait for this tile's points never
    // waits for them; the input's ragged last tile comes after the loop
    const int tfe = max(tb, min(te, n / kTile));
    constexpr uint32_t kAll = (1u << kItems) - 1u;
    int32_t XA[kItems], YA[kItems], XB[kItems], YB[kItems];
    TileGeo tc;
    tc.single = 0;
    if (tb < tfe) {
        tc = tile_record(ws, 0, tb, ntiles);
        load_full_wave(a, tb * kTile, XA, YA);
    }
    for (int tile = tb; tile < tfe; tile += 2) {
        const int t1 = min(tile + 1, tfe - 1);
        TileGeo tn = tile_record(ws, 0, t1, ntiles);
        load_full_wave(a, t1 * kTile, XB, YB);
        process(tile, tc, XA, YA, kAll);
        if (tile + 1 >= tfe) break;
        tc = tn;
        const int t2 = min(tile + 2, tfe - 1);
        tn = tile_record(ws, 0, t2, ntiles);
        load_full_wave(a, t2 * kTile, XA, YA);
        process(tile + 1, tc, XB, YB, kAll);
        tc = tn;
    }
    for (int tile = tfe; tile < te; ++tile) {
        const TileGeo tl = tile_record(ws, 0, tile, ntiles);
        int32_t X[kItems], Y[kItems];
        const uint32_t vm = tl.single ? load_input_wave(a, tile * kTile, min(tile * kTile + kTile, n), X, Y) : 0u;
        process(tile, tl, X, Y, vm);
    }
    if (cur >= 0) close_run();
    // survivors of the split (counted, not written) per child
    const uint32_t s0 = wave_sum(acc0), s1 = wave_sum(acc1);
    if (lane == 0 && (s0 | s1)) {
        const int sl = (blockIdx.x * kNW + wv) % kAccSlots;
        atomicAdd(&ctl->nacc[0][0][sl], s0);
        atomicAdd(&ctl->nacc[0][1][sl], s1);
    }
    if (MODE != 0) flush_filter_stats(ctl, sm->stat, ntests, nfall, ncand);
}

// ---------------------------------------------------------------------------
// the round after the read-only split
// ---------------------------------------------------------------------------
// Its segments are the split's children: child 0 of an instance (edge a -> b,
// apex f0) holds the instance's points with (p - a) x (b - a) > 0, child 1
// (edge b -> a, apex f1) those with a negative sign.  Both are kept as the
// instance's input range, child 0 in region 0 and child 1 in region 1 under
// the same segment index, so one pass over the caller's array serves both:
// each point takes its side from the sign, then is tested against its
// side's new edges u -> f and f -> v as in every round (Algorithm 1's
// classification).  The survivors of input tile t that go to child c of
// side 0 are written to region c from the start of slot t, those of side 1
// so that they end at the slot's end (a tile has at most kTile points on
// both sides together); for the piece table they are the pieces of tile t
// and of tile nt + t, the tiles of region 0 and region 1 of this round.
// the low bit of each item's three-bit field
constexpr uint32_t kLow3 = 0x249249u & ((1u << (3 * kItems)) - 1u);
static_assert(3 * kItems <= 24, "three-bit class fields");

struct Ro1Smem {
    uint32_t stat[4];
    RunBest wrb[kNW][4];
    uint32_t wcnt[kNW][4];                   // survivors of the tile per wave and class
    int32_t sx[kTile], sy[kTile], si[kTile];  // the tile's survivors, grouped by class
};

// a tile's record in this round with the geometry of both sides
struct TileGeo2 {
    int32_t seg, single, start, end;
    int32_t ax, ay, bx, by, f0x, f0y, f1x, f1y;
};

__device__ __forceinline__ TileGeo2 ro1_record(const Ws2 &ws, int lt) {
    const int32_t *src = reinterpret_cast<const int32_t *>(ws.tinfo(1, 0) + lt);
    TileGeo2 ti;
    ti.seg = scalar_load(src + 0);
    ti.single = scalar_load(src + 1);
    ti.start = scalar_load(src + 2);
    ti.end = scalar_load(src + 3);
    ti.ax = ti.ay = ti.bx = ti.by = ti.f0x = ti.f0y = ti.f1x = ti.f1y = 0;
    if (ti.single) {
        const int32_t *g0 = reinterpret_cast<const int32_t *>(ws.geo(1, 0) + ti.seg);
        const int32_t *g1 = reinterpret_cast<const int32_t *>(ws.geo(1, 1) + ti.seg);
        ti.ax = scalar_load(g0 + 2); ti.ay = scalar_load(g0 + 3);
        ti.f0x = scalar_load(g0 + 4); ti.f0y = scalar_load(g0 + 5);
        ti.bx = scalar_load(g0 + 6); ti.by = scalar_load(g0 + 7);
        ti.f1x = scalar_load(g1 + 4); ti.f1y = scalar_load(g1 + 5);
    }
    return ti;
}

// Items are classified into four classes, k = 2 side + child (0: side 0 /
// child 0, 1: side 0 / child 1, 2: side 1 / child 0, 3: side 1 / child 1),
// 4 = dropped; three bits per item in one register.  The survivors of a tile
// are staged in LDS grouped by class (each lane's items in item order at the
// lane's offset within its wave's share), then written out in order: class
// k goes to region (k & 1), side 0 from the start of the tile's slot, side 1
// so that it ends at the slot's end.  Each wave keeps the best point of
// every class of the run as uniform values; a lane's point is compared
// exactly only when it reaches its class's best (FP32 filter: when its
// estimate reaches the class's threshold), which soon becomes rare.
template <int MODE>
__device__ __forceinline__ void phase_round_ro1(const Ws2 &ws, const HullArgs &a, char *smem) {
    Ro1Smem *sm = reinterpret_cast<Ro1Smem *>(smem);
    Control *ctl = ws.ctl;
    const RoundState *rs = &ctl->rs[1];
    const int n = rs->n[0];  // = rs->n[1]: both regions are the input
    const int S0 = rs->s[0];
    const int nt = (n + kTile - 1) / kTile;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
    int32_t *const obase = ws.px(0, 0);  // output planes: [child][x, y, index][cap]
    const int64_t cap = ws.cap_pts;
    const int T = (nt + (int)gridDim.x - 1) / (int)gridDim.x;
    if (blockIdx.x == 0 && tid == 0) {
        ctl->rs[0].nmulti = 0;
        ctl->tper[1] = T;
        ctl->maxseg[0] = 0;
    }
    const int tb = blockIdx.x * T, te = min(tb + T, nt);
    const float c2 = MODE ? coord_c2(ctl) : 0.f;
    WaveBest wb;
    auto wb_reset = [&]() {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            wb.W[k] = 0;
            wb.T[k] = ~0ull;
            wb.tau[k] = -INFINITY;
            wb.C[k] = 0;
        }
    };
    wb_reset();
    int cur = -1, run0 = 0, run_lo = 0, run_hi = 0, seg_st = 0, seg_en = 0;
    uint32_t acc0 = 0, acc1 = 0, ntests = 0, nfall = 0, ncand = 0;
    bool oob = false;
    // FP32 form: the full tiles' points are requested a tile ahead,
    // unconditionally (the last one reloads its own tile; a skipped tile's
    // loads are consumed too), so that the wait for a tile's points covers
    // only them and the stores before them; the input's ragged last tile is
    // loaded when it comes.  (The exact form loads each tile when it comes:
    // with the prefetch it was slower, 1.76 against 1.70 ms on 4,096 disks.)
    const int tfe = MODE != 0 ? max(tb, min(te, n / kTile)) : tb;
    constexpr uint32_t kAll = (1u << kItems) - 1u;
    int32_t XN[kItems], YN[kItems];
    if (MODE != 0 && tb < tfe) load_full_wave(a, tb * kTile, XN, YN);

    for (int tile = tb; tile <= te; ++tile) {
        int32_t X[kItems], Y[kItems];
        const bool pf = MODE != 0 && tile < tfe;
        if (pf) {
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                X[i] = XN[i];
                Y[i] = YN[i];
                asm volatile("" ::"v"(X[i]), "v"(Y[i]));
            }
            load_full_wave(a, min(tile + 1, tfe - 1) * kTile, XN, YN);
        }
        TileGeo2 ti;
        ti.single = 0;
        if (tile < te) ti = ro1_record(ws, tile);
        if (cur >= 0 && (!ti.single || ti.seg != cur)) {
            // the run ends: the waves' bests merged into its records
            if (lane == 0) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    RunBest r;
                    r.k1 = wb.W[k];
                    r.k2 = wb.T[k];
                    r.cnt = (int32_t)wb.C[k];
                    sm->wrb[wv][k] = r;
                }
            }
            __syncthreads();
            if (tid < 4) {
                RunBest m = sm->wrb[0][tid];
#pragma unroll
                for (int w = 1; w < kNW; ++w) rb_merge(m, sm->wrb[w][tid]);
                Best b;
                b.key1 = m.k1;
                b.key2 = m.k2;
                b.cnt = m.cnt;
                b.idx = m.k1 ? (int32_t)(uint32_t)m.k2 : 0;
                b.x = b.y = 0;  // filled in by the segment kernel for the winner
                const int sd = tid >> 1, c = tid & 1;
                const int g = (sd ? S0 : 0) + cur, rt = (sd ? nt : 0) + run0;
                if (seg_st >= run_lo && seg_en <= run_hi) ws.adir[g * 2 + c] = b;
                ws.recF[rt * 2 + c] = b;
                ws.recL[rt * 2 + c] = b;
            }
            __syncthreads();
            wb_reset();
            cur = -1;
        }
        if (!ti.single) continue;  // past the last tile, or the multi-segment kernel takes it
        const int lo = tile * kTile, hi = min(lo + kTile, n);
        if (cur < 0) {
            cur = ti.seg;
            run0 = tile;
            run_lo = lo;
            seg_st = ti.start;
            seg_en = ti.end;
        }
        run_hi = hi;
        const uint32_t vm = pf ? kAll : load_input_wave(a, lo, hi, X, Y);
        // Relative to a (q = p - a): the side is the sign of q x (b - a); side
        // 0's children are q x E00 and q x E01 - K01, side 1's q x E10 - K10
        // and q x E11, with E00 = f0 - a, E01 = b - f0, E10 = f1 - b,
        // E11 = a - f1, K01 = E00 x E01, K10 = (b - a) x E10 (the cross
        // products of Algorithm 1's tests, regrouped)
        const int ax = ti.ax, ay = ti.ay, bx = ti.bx, by = ti.by;
        const int esx = bx - ax, esy = by - ay;
        const int e00x = ti.f0x - ax, e00y = ti.f0y - ay, e01x = bx - ti.f0x, e01y = by - ti.f0y;
        const int e10x = ti.f1x - bx, e10y = ti.f1y - by, e11x = ax - ti.f1x, e11y = ay - ti.f1y;
        uint32_t cl = 0;  // class of item i in bits 3i .. 3i + 2
        uint32_t fl = 0;  // FP32 filter: argmax candidates (bit 3i)
        float Bk[4] = {0.f, 0.f, 0.f, 0.f};
        if (MODE == 0) {
            const int64_t nk01 = -((int64_t)e00x * e01y - (int64_t)e00y * e01x);
            const int64_t nk10 = -((int64_t)esx * e10y - (int64_t)esy * e10x);
            // the per-side values as vector-register copies
            const int32_t v00x = vcopy(e00x), v00y = vcopy(e00y), v10x = vcopy(e10x), v10y = vcopy(e10y);
            const int32_t v01x = vcopy(e01x), v01y = vcopy(e01y), v11x = vcopy(e11x), v11y = vcopy(e11y);
            const int32_t k01l = vcopy((int32_t)(uint32_t)nk01), k01h = vcopy((int32_t)(uint32_t)(nk01 >> 32));
            const int32_t k10l = vcopy((int32_t)(uint32_t)nk10), k10h = vcopy((int32_t)(uint32_t)(nk10 >> 32));
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                const bool valid = (vm >> i) & 1u;
                const int32_t qx = X[i] - ax, nqy = ay - Y[i];
                const int64_t ds = (int64_t)((uint64_t)((int64_t)qx * esy) + (uint64_t)((int64_t)nqy * esx));
                const bool s1 = ds < 0, live = valid && ds != 0;
                const int32_t a0x = s1 ? v10x : v00x, a0y = s1 ? v10y : v00y;
                const int32_t a1x = s1 ? v11x : v01x, a1y = s1 ? v11y : v01y;
                const int64_t nk0 = (int64_t)(((uint64_t)(uint32_t)(s1 ? k10h : 0) << 32) | (uint32_t)(s1 ? k10l : 0));
                const int64_t nk1 = (int64_t)(((uint64_t)(uint32_t)(s1 ? 0 : k01h) << 32) | (uint32_t)(s1 ? 0 : k01l));
                const int64_t d0 = (int64_t)((uint64_t)((int64_t)qx * a0y) + (uint64_t)((int64_t)nqy * a0x) + (uint64_t)nk0);
                const int64_t d1 = (int64_t)((uint64_t)((int64_t)qx * a1y) + (uint64_t)((int64_t)nqy * a1x) + (uint64_t)nk1);
                const bool o0 = live && d0 > 0, o1 = live && !o0 && d1 > 0;
                const uint32_t k = (o0 || o1) ? (s1 ? 2u : 0u) + (o1 ? 1u : 0u) : 4u;
                cl |= k << (3 * i);
                const uint64_t d = (uint64_t)(o0 ? d0 : d1);
                // (bitwise: no short-circuit branches)
                const bool need = ((k == 0) & (d >= wb.W[0])) | ((k == 1) & (d >= wb.W[1])) |
                                  ((k == 2) & (d >= wb.W[2])) | ((k == 3) & (d >= wb.W[3]));
                // offered at once: the wave's bests rise item by item, and
                // with four classes that keeps the offers fewer than
                // flagging them for a pass per tile
                if (__ballot(need)) {
                    const uint64_t tk = tie_key(X[i], Y[i], fast_pos_init(lo, i), o0 ? a0x : a1x, o0 ? a0y : a1y);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) wave_offer(wb, kk, need && k == (uint32_t)kk, d, tk, 0.f);
                }
            }
        } else {
            const float Bs = static_bound(esx, esy, c2);
            Bk[0] = static_bound(e00x, e00y, c2);
            Bk[1] = static_bound(e01x, e01y, c2);
            Bk[2] = static_bound(e10x, e10y, c2);
            Bk[3] = static_bound(e11x, e11y, c2);
            const float fesx = (float)esx, fesy = (float)esy;
            // per-side values as vector-register copies: the child edges, the
            // offsets of u and f from a, the bounds
            const int32_t v00x = vcopy(e00x), v00y = vcopy(e00y), v10x = vcopy(e10x), v10y = vcopy(e10y);
            const int32_t v01x = vcopy(e01x), v01y = vcopy(e01y), v11x = vcopy(e11x), v11y = vcopy(e11y);
            const int32_t vesx = vcopy(esx), vesy = vcopy(esy);
            const int32_t vf0x = vcopy(e00x), vf0y = vcopy(e00y);
            const int32_t vf1x = vcopy(ti.f1x - ax), vf1y = vcopy(ti.f1y - ay);
            const float vb00 = __int_as_float(vcopy(__float_as_int(Bk[0]))), vb10 = __int_as_float(vcopy(__float_as_int(Bk[2])));
            const float vb01 = __int_as_float(vcopy(__float_as_int(Bk[1]))), vb11 = __int_as_float(vcopy(__float_as_int(Bk[3])));
            uint32_t und = 0, cand = 0;  // undecided items; estimates at their class's threshold
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                const bool valid = (vm >> i) & 1u;
                const int32_t qx = X[i] - ax, qy = Y[i] - ay;
                const float es = __fsub_rn(__fmul_rn((float)qx, fesy), __fmul_rn((float)qy, fesx));
                const bool s1 = es < -Bs, sure = s1 || es > Bs;
                // u - a: 0 or b - a; f - a: f0 - a or f1 - a
                const int32_t d0x = qx - (s1 ? vesx : 0), d0y = qy - (s1 ? vesy : 0);
                const int32_t d1x = qx - (s1 ? vf1x : vf0x), d1y = qy - (s1 ? vf1y : vf0y);
                const int32_t a0x = s1 ? v10x : v00x, a0y = s1 ? v10y : v00y;
                const int32_t a1x = s1 ? v11x : v01x, a1y = s1 ? v11y : v01y;
                const float B0 = s1 ? vb10 : vb00, B1 = s1 ? vb11 : vb01;
                const float e0 = __fsub_rn(__fmul_rn((float)d0x, (float)a0y), __fmul_rn((float)d0y, (float)a0x));
                const float e1 = __fsub_rn(__fmul_rn((float)d1x, (float)a1y), __fmul_rn((float)d1y, (float)a1x));
                // 0, 1: child; 2: dropped; 3: undecided
                uint32_t st = e0 > B0 ? 0u : (!(e0 < -B0) ? 3u : (e1 > B1 ? 1u : (e1 < -B1 ? 2u : 3u)));
                st = !valid ? 2u : (!sure ? 3u : st);
                const uint32_t k = st < 2 ? (s1 ? 2u : 0u) + st : 4u;
                cl |= k << (3 * i);
                und |= (st == 3 ? 1u : 0u) << i;
                const float e = st == 0 ? e0 : e1;
                const bool c = ((k == 0) & (e >= wb.tau[0])) | ((k == 1) & (e >= wb.tau[1])) |
                               ((k == 2) & (e >= wb.tau[2])) | ((k == 3) & (e >= wb.tau[3]));
                cand |= (c ? 1u : 0u) << i;
                ntests += valid ? (sure ? (e0 > B0 ? 2u : 3u) : 1u) : 0u;
            }
            // undecided items (rare): the whole classification in int64
            if (__ballot(und != 0)) {
#pragma unroll
                for (int i = 0; i < kItems; ++i) {
                    if (!((und >> i) & 1u)) continue;
                    const int32_t x = X[i], y = Y[i];
                    const int64_t ds = cross_i64(x, y, ax, ay, bx, by);
                    const bool s1 = ds < 0;
                    const bool o0 = ds != 0 && cross_i64(x, y, s1 ? bx : ax, s1 ? by : ay, s1 ? ti.f1x : ti.f0x,
                                                         s1 ? ti.f1y : ti.f0y) > 0;
                    const bool o1 = ds != 0 && !o0 &&
                                    cross_i64(x, y, s1 ? ti.f1x : ti.f0x, s1 ? ti.f1y : ti.f0y, s1 ? ax : bx,
                                              s1 ? ay : by) > 0;
                    const uint32_t k = (o0 || o1) ? (s1 ? 2u : 0u) + (o1 ? 1u : 0u) : 4u;
                    cl = (cl & ~(7u << (3 * i))) | (k << (3 * i));
                }
                nfall += (uint32_t)__popc(und);
            }
            // candidates: estimates at or above their class's threshold, and
            // the items decided exactly
#pragma unroll
            for (int i = 0; i < kItems; ++i) fl |= (((und | cand) >> i) & 1u) << (3 * i);
        }
        if (MODE != 0 && __ballot(fl != 0)) {
            // each lane's best flagged item of each class (exact distances to
            // the child edge), then the wave's
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                // bit 3i: item i is flagged and of class kk
                const uint32_t x = cl ^ ((uint32_t)kk * kLow3);
                const uint32_t fc = fl & ~(x | (x >> 1) | (x >> 2)) & kLow3;
                if (!__ballot(fc != 0)) continue;
                if (MODE != 0) ncand += (uint32_t)__popc(fc);
                int px0 = kk == 0 ? ax : kk == 1 ? ti.f0x : kk == 2 ? bx : ti.f1x;
                int py0 = kk == 0 ? ay : kk == 1 ? ti.f0y : kk == 2 ? by : ti.f1y;
                int cx = kk == 0 ? e00x : kk == 1 ? e01x : kk == 2 ? e10x : e11x;
                int cy = kk == 0 ? e00y : kk == 1 ? e01y : kk == 2 ? e10y : e11y;
                // opaque: the distances are recomputed here, not kept alive
                // from the classification
                asm volatile("" : "+v"(px0), "+v"(py0), "+v"(cx), "+v"(cy));
                uint64_t bd = 0, bt = ~0ull;
#pragma unroll
                for (int i = 0; i < kItems; ++i) {
                    if (!((fc >> (3 * i)) & 1u)) continue;
                    const uint64_t d = (uint64_t)((int64_t)(X[i] - px0) * (int64_t)cy - (int64_t)(Y[i] - py0) * (int64_t)cx);
                    const uint64_t tk = tie_key(X[i], Y[i], fast_pos_init(lo, i), cx, cy);
                    const bool better = d > bd || (d == bd && tk < bt);
                    bd = better ? d : bd;
                    bt = better ? tk : bt;
                }
                wave_offer(wb, kk, bd != 0, bd, bt, Bk[kk]);
            }
        }
        // per-lane counts of the four classes (8-bit fields), their prefix in
        // the wave (16-bit fields, two classes per word)
        uint32_t cnt = 0;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t k = (cl >> (3 * i)) & 7u;
            cnt += k < 4 ? (1u << (8u * k)) : 0u;
        }
        const uint32_t c01 = field8(cnt, 0) | (field8(cnt, 1) << 16), c23 = field8(cnt, 2) | (field8(cnt, 3) << 16);
        const uint32_t i01 = wave_incl_sum(c01), i23 = wave_incl_sum(c23);
        const uint32_t w01 = wave_read(i01, kWave - 1), w23 = wave_read(i23, kWave - 1);
        wb.C[0] += w01 & 0xffffu;
        wb.C[1] += w01 >> 16;
        wb.C[2] += w23 & 0xffffu;
        wb.C[3] += w23 >> 16;
        if (lane == 0) {
            sm->wcnt[wv][0] = w01 & 0xffffu;
            sm->wcnt[wv][1] = w01 >> 16;
            sm->wcnt[wv][2] = w23 & 0xffffu;
            sm->wcnt[wv][3] = w23 >> 16;
        }
        __syncthreads();
        uint32_t tot[4], wbase[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            tot[k] = 0;
            wbase[k] = 0;
#pragma unroll
            for (int w = 0; w < kNW; ++w) {
                const uint32_t c = sm->wcnt[w][k];
                wbase[k] += (w < wv) ? c : 0u;
                tot[k] += c;
            }
        }
        const uint32_t cs1 = tot[0], cs2 = cs1 + tot[1], cs3 = cs2 + tot[2], S = cs3 + tot[3];
        // staging offsets of this lane's first item of each class
        const uint32_t e01 = i01 - c01, e23 = i23 - c23;
        const uint32_t lb0 = wbase[0] + (e01 & 0xffffu), lb1 = cs1 + wbase[1] + (e01 >> 16);
        const uint32_t lb2 = cs2 + wbase[2] + (e23 & 0xffffu), lb3 = cs3 + wbase[3] + (e23 >> 16);
        uint32_t run = 0;  // the lane's items staged so far per class (8-bit fields)
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t k = (cl >> (3 * i)) & 7u;
            if (k < 4) {
                const uint32_t pos = ((k & 2u) ? ((k & 1u) ? lb3 : lb2) : ((k & 1u) ? lb1 : lb0)) + field8(run, k);
                run += 1u << (8u * k);
                sm->sx[pos] = X[i];
                sm->sy[pos] = Y[i];
                sm->si[pos] = fast_pos_init(lo, i);
            }
        }
        __syncthreads();
        // write out: class k of output j by comparing with the class starts;
        // slot position j + D[k]
        const int64_t pbase = (int64_t)tile * kTile;
        const bool fits = pbase + kTile <= cap - kTile;
        oob |= !fits;
        int32_t *const P0 = obase + pbase;
        int32_t *const P1 = P0 + 3 * cap;
        const int32_t D0 = 0, D1 = -(int32_t)cs1;
        const int32_t D2 = kTile - (int32_t)tot[2] - (int32_t)cs2, D3 = kTile - (int32_t)tot[3] - (int32_t)cs3;
        if (fits) {
            for (uint32_t j = (uint32_t)tid; j < S; j += kBlock) {
                const bool g1 = j >= cs1, g2 = j >= cs2, g3 = j >= cs3;
                const int32_t D = g3 ? D3 : (g2 ? D2 : (g1 ? D1 : D0));
                const bool r1 = g3 || (g1 && !g2);  // classes 1 and 3 go to region 1
                int32_t *d = (r1 ? P1 : P0) + ((int32_t)j + D);
                d[0] = sm->sx[j];
                d[cap] = sm->sy[j];
                d[2 * cap] = sm->si[j];
            }
        }
        if (tid == 0) {
            ws.tcnt(1)[tile] = tot[0] | (tot[1] << 16);
            ws.tcnt(1)[nt + tile] = tot[2] | (tot[3] << 16);
            acc0 += tot[0] + tot[2];
            acc1 += tot[1] + tot[3];
        }
        __syncthreads();  // the staging buffer is reused by the next tile
    }
    if (oob) atomicOr(&ctl->error, kErrInternal);
    if (tid == 0 && (acc0 | acc1)) {
        atomicAdd(&ctl->nacc[1][0][blockIdx.x % kAccSlots], acc0);
        atomicAdd(&ctl->nacc[1][1][blockIdx.x % kAccSlots], acc1);
    }
    if (MODE != 0) flush_filter_stats(ctl, sm->stat, ntests, nfall, ncand);
}

// Tiles that hold several segments (listed by the segment kernel): the whole
// block in point order, per-segment reductions in LDS.
template <int MODE>
__device__ __forceinline__ void phase_round_multi(const Ws2 &ws, const HullArgs &a, int r, char *smem) {
    RoundSmem *sm = reinterpret_cast<RoundSmem *>(smem);
    uint32_t *stat = sm->stat;
    // the split and the round after it read the input (index = position); the
    // split writes no point, and in the round after it a segment keeps only
    // the points strictly outside its own edge u -> v (its side of the
    // split's line), and region 1 writes its survivors so that they end at
    // the end of their tile's slot
    const bool INIT = r <= 1, KEEP = r != 0, OWN = r == 1;
    Control *ctl = ws.ctl;
    const int p = r & 1, q = p ^ 1;
    const RoundState *rs = &ctl->rs[p];
    const int n0 = rs->n[0], n1 = rs->n[1];
    const int S0 = rs->s[0], S1 = rs->s[1];
    const int nt0 = (n0 + kTile - 1) / kTile, nt1 = (n1 + kTile - 1) / kTile;
    const int ntiles = nt0 + nt1;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
    int32_t *ox0 = ws.px(q, 0), *oy0 = ws.py(q, 0), *oi0 = ws.pi(q, 0);
    int32_t *ox1 = ws.px(q, 1), *oy1 = ws.py(q, 1), *oi1 = ws.pi(q, 1);
    const int64_t cap = ws.cap_pts;
    (void)S0; (void)S1; (void)lane; (void)wv;

    uint32_t ntests = 0, nfall = 0, ncand = 0;
    uint32_t acc0 = 0, acc1 = 0;  // survivors written by this block (thread 0)
    bool oob = false;
    const int nm = min(rs->nmulti, ws.tcap);
    const int32_t *ml = ws.ml(p);
    for (int j = blockIdx.x; j < nm; j += gridDim.x) {
        const int tile = ml[j];
        if (tile < 0 || tile >= ntiles) {
            oob = true;
            continue;
        }
        const int R = tile < nt0 ? 0 : 1;
        const int lt = tile - (R ? nt0 : 0);
        const int NR = R ? n1 : n0;
        const int SR = R ? S1 : S0;
        const int gbase = R ? S0 : 0;
        const int lo = lt * kTile;
        const int hi = min(lo + kTile, NR);
        (void)SR;
        const TileInfo ti = ws.tinfo(p, R)[lt];
        const int s0 = ti.seg;
        int32_t X[kItems], Y[kItems], I[kItems];
        if (INIT) {
            load_input(a, lo, hi, X, Y, I);
        } else if (!load_pieces(ws, p, R, lt, R ? nt1 : nt0, rs->npc[R], lo, hi, sm->pvs, sm->pps,
                                X, Y, I)) {
            __syncthreads();
            continue;
        }
        uint32_t stbits = 0xaaaaaaaau;  // 2 bits per point: 0, 1 = child, 2 = dropped
        uint32_t rr[kQ];                // packed in-tile ranks of each row's first survivor
        uint32_t total;                 // the tile's survivors (packed)
        {
            // several segments: starts into LDS, per-slot reductions (point order)
            const SegGeo *geo = ws.geo(p, R);
            if (tid == 0) sm->s_m = 0;
            __syncthreads();
            for (int b = 0; b <= kTile; b += kBlock) {
                const int j = b + tid;
                bool in = false;
                if (j <= kTile) {
                    const int si = s0 + j;
                    const int st = si < SR ? geo[si].start : NR;
                    sm->sstart[j] = st;
                    in = st < hi;
                }
                const int cnt = __syncthreads_count(in);
                if (tid == 0) sm->s_m += cnt;
                if (cnt < kBlock) break;
            }
            __syncthreads();
            const int m = sm->s_m;
            uint32_t slotpk[kItems / 2];
#pragma unroll
            for (int i = 0; i < kItems; i += 2) {
                const int va = item_pos(lo, i);
                const int sa = (va >= hi) ? 0 : slot_of(sm->sstart, m, va);
                const int sb = (va + 1 >= hi) ? 0 : slot_of(sm->sstart, m, va + 1);
                slotpk[i >> 1] = (uint32_t)sa | ((uint32_t)sb << 16);
            }
            for (int w0 = 0; w0 < m; w0 += kSlots) {
                const int wn = min(kSlots, m - w0);
                for (int j = tid; j < wn; j += kBlock) {
                    const SegGeo g = geo[s0 + w0 + j];
                    sm->lgeo[j][0] = g.ux; sm->lgeo[j][1] = g.uy;
                    sm->lgeo[j][2] = g.fx; sm->lgeo[j][3] = g.fy;
                    sm->lgeo[j][4] = g.vx; sm->lgeo[j][5] = g.vy;
                }
                for (int j = tid; j < 2 * kSlots; j += kBlock) {
                    (&sm->k1[0][0])[j] = 0;
                    (&sm->k2[0][0])[j] = ~0ull;
                    (&sm->lm[0][0])[j] = 0;
                    (&sm->scnt[0][0])[j] = 0;
                }
                __syncthreads();
                // classify; the best distance (exact) or lower bound (filter) per
                // slot.  The filter keeps each survivor's upper bound key, the
                // value the argmax steps below compare with the slot's best
                // lower bound.
                uint32_t ckey[kItems];
                uint64_t dd[kItems];  // exact distance to the child's edge (candidates)
#pragma unroll
                for (int i = 0; i < kItems; ++i) {
                    ckey[i] = 0;
                    dd[i] = 0;
                    const int v = item_pos(lo, i);
                    const int sl = (int)((slotpk[i >> 1] >> ((i & 1) * 16)) & 0xffffu);
                    if (v >= hi || sl < w0 || sl >= w0 + wn) continue;
                    const int ls = sl - w0;
                    const int ux = sm->lgeo[ls][0], uy = sm->lgeo[ls][1];
                    const int fx = sm->lgeo[ls][2], fy = sm->lgeo[ls][3];
                    const int vx = sm->lgeo[ls][4], vy = sm->lgeo[ls][5];
                    uint32_t st = 2;
                    if (OWN) {
                        // the split's side: strictly outside the segment's own edge
                        bool own;
                        if (MODE == 0) {
                            own = cross_i64(X[i], Y[i], ux, uy, vx, vy) > 0;
                        } else {
                            float Bo;
                            const float eo = cross_f32(X[i], Y[i], ux, uy, vx, vy, Bo);
                            ntests++;
                            if (eo > Bo) own = true;
                            else if (eo < -Bo) own = false;
                            else { nfall++; own = cross_i64(X[i], Y[i], ux, uy, vx, vy) > 0; }
                        }
                        if (!own) continue;
                    }
                    if (MODE == 0) {
                        const int64_t d0 = cross_i64(X[i], Y[i], ux, uy, fx, fy);
                        if (d0 > 0) {
                            st = 0;
                            dd[i] = (uint64_t)d0;
                            atomicMax(&sm->k1[0][ls], (uint64_t)d0);
                        } else {
                            const int64_t d1 = cross_i64(X[i], Y[i], fx, fy, vx, vy);
                            if (d1 > 0) {
                                st = 1;
                                dd[i] = (uint64_t)d1;
                                atomicMax(&sm->k1[1][ls], (uint64_t)d1);
                            }
                        }
                    } else {
                        float B0;
                        const float e0 = cross_f32(X[i], Y[i], ux, uy, fx, fy, B0);
                        ntests++;
                        bool out0;
                        if (e0 > B0) out0 = true;
                        else if (e0 < -B0) out0 = false;
                        else { nfall++; out0 = cross_i64(X[i], Y[i], ux, uy, fx, fy) > 0; }
                        if (out0) {
                            st = 0;
                            atomicMax(&sm->lm[0][ls], fkey(__fsub_rn(e0, 2.f * B0)));
                            ckey[i] = fkey(__fadd_rn(e0, 2.f * B0));
                        } else {
                            float B1;
                            const float e1 = cross_f32(X[i], Y[i], fx, fy, vx, vy, B1);
                            ntests++;
                            bool out1;
                            if (e1 > B1) out1 = true;
                            else if (e1 < -B1) out1 = false;
                            else { nfall++; out1 = cross_i64(X[i], Y[i], fx, fy, vx, vy) > 0; }
                            if (out1) {
                                st = 1;
                                atomicMax(&sm->lm[1][ls], fkey(__fsub_rn(e1, 2.f * B1)));
                                ckey[i] = fkey(__fadd_rn(e1, 2.f * B1));
                            }
                        }
                    }
                    if (st < 2) atomicAdd(&sm->scnt[st][ls], 1u);
                    stbits ^= (st ^ 2u) << (2 * i);
                }
                __syncthreads();
                if (MODE != 0) {
                    // candidates of the argmax get exact distances
#pragma unroll
                    for (int i = 0; i < kItems; ++i) {
                        const int v = item_pos(lo, i);
                        const int sl = (int)((slotpk[i >> 1] >> ((i & 1) * 16)) & 0xffffu);
                        const uint32_t st = (stbits >> (2 * i)) & 3u;
                        if (v >= hi || st > 1 || sl < w0 || sl >= w0 + wn) continue;
                        const int ls = sl - w0;
                        if (ckey[i] < sm->lm[st][ls]) continue;
                        ncand++;
                        dd[i] = (uint64_t)child_d(X[i], Y[i], st, sm->lgeo[ls]);
                        atomicMax(&sm->k1[st][ls], dd[i]);
                    }
                    __syncthreads();
                }
                // tie-break among the farthest points, then the winner
#pragma unroll
                for (int i = 0; i < kItems; ++i) {
                    const int v = item_pos(lo, i);
                    const int sl = (int)((slotpk[i >> 1] >> ((i & 1) * 16)) & 0xffffu);
                    const uint32_t st = (stbits >> (2 * i)) & 3u;
                    if (v >= hi || st > 1 || sl < w0 || sl >= w0 + wn) continue;
                    const int ls = sl - w0;
                    if (MODE != 0 && ckey[i] < sm->lm[st][ls]) continue;
                    if (dd[i] != sm->k1[st][ls]) continue;
                    const int ex = st == 0 ? sm->lgeo[ls][2] - sm->lgeo[ls][0] : sm->lgeo[ls][4] - sm->lgeo[ls][2];
                    const int ey = st == 0 ? sm->lgeo[ls][3] - sm->lgeo[ls][1] : sm->lgeo[ls][5] - sm->lgeo[ls][3];
                    atomicMin(&sm->k2[st][ls], tie_key(X[i], Y[i], I[i], ex, ey));
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < kItems; ++i) {
                    const int v = item_pos(lo, i);
                    const int sl = (int)((slotpk[i >> 1] >> ((i & 1) * 16)) & 0xffffu);
                    const uint32_t st = (stbits >> (2 * i)) & 3u;
                    if (v >= hi || st > 1 || sl < w0 || sl >= w0 + wn) continue;
                    const int ls = sl - w0;
                    if (MODE != 0 && ckey[i] < sm->lm[st][ls]) continue;
                    if (dd[i] != sm->k1[st][ls]) continue;
                    const int ex = st == 0 ? sm->lgeo[ls][2] - sm->lgeo[ls][0] : sm->lgeo[ls][4] - sm->lgeo[ls][2];
                    const int ey = st == 0 ? sm->lgeo[ls][3] - sm->lgeo[ls][1] : sm->lgeo[ls][5] - sm->lgeo[ls][3];
                    if (tie_key(X[i], Y[i], I[i], ex, ey) == sm->k2[st][ls]) {
                        sm->res[st][ls][0] = X[i]; sm->res[st][ls][1] = Y[i]; sm->res[st][ls][2] = I[i];
                    }
                }
                __syncthreads();
                // whole segments directly, the tile's first and last as partials
                for (int j = tid; j < wn; j += kBlock) {
                    const int sl = w0 + j;
                    const int g = gbase + s0 + sl;
                    const bool inside = sm->sstart[sl] >= lo && sm->sstart[sl + 1] <= hi;
                    for (int c = 0; c < 2; ++c) {
                        Best b;
                        b.key1 = sm->k1[c][j];
                        b.key2 = sm->k2[c][j];
                        b.x = b.key1 ? sm->res[c][j][0] : 0;
                        b.y = b.key1 ? sm->res[c][j][1] : 0;
                        b.idx = b.key1 ? sm->res[c][j][2] : 0;
                        b.cnt = (int32_t)sm->scnt[c][j];
                        if (inside) ws.adir[g * 2 + c] = b;
                        if (sl == 0) ws.recF[tile * 2 + c] = b;
                        if (sl == m - 1) ws.recL[tile * 2 + c] = b;
                    }
                }
                __syncthreads();
            }
            // point order keeps every segment's children contiguous
            uint32_t cnt[kQ], rowbase[kQ];
            total = tile_ranks(stbits, cnt, rowbase, sm->scan);
#pragma unroll
            for (int qq = 0; qq < kQ; ++qq) rr[qq] = rowbase[qq] + cnt[qq];
        }
        // scatter: child c of this tile goes to region c at tile * kTile; in the
        // round after the split, region 1's tiles (side 1 of input tile lt)
        // end at the end of slot lt
        const int64_t pbase = (int64_t)(OWN ? lt : tile) * kTile;
        const int64_t pb0 = pbase + ((OWN && R) ? kTile - (int64_t)(total & 0xffffu) : 0);
        const int64_t pb1 = pbase + ((OWN && R) ? kTile - (int64_t)(total >> 16) : 0);
#pragma unroll
        for (int qq = 0; qq < kQ && KEEP; ++qq) {
            uint32_t q_ = rr[qq];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = qq * 4 + j;
                const uint32_t st = (stbits >> (2 * i)) & 3u;
                if (st == 0) {
                    const int64_t e = pb0 + (q_ & 0xffffu);
                    if (e < cap) { ox0[e] = X[i]; oy0[e] = Y[i]; oi0[e] = I[i]; } else oob = true;
                    q_ += 1u;
                } else if (st == 1) {
                    const int64_t e = pb1 + (q_ >> 16);
                    if (e < cap) { ox1[e] = X[i]; oy1[e] = Y[i]; oi1[e] = I[i]; } else oob = true;
                    q_ += 0x10000u;
                }
            }
        }
        if (tid == 0) {
            if (KEEP) ws.tcnt(p)[tile] = total;
            acc0 += total & 0xffffu;
            acc1 += total >> 16;
        }
        __syncthreads();  // LDS is reused by the next tile
    }
    if (oob) atomicOr(&ctl->error, kErrInternal);
    if (tid == 0 && (acc0 | acc1)) {
        atomicAdd(&ctl->nacc[p][0][blockIdx.x % kAccSlots], acc0);
        atomicAdd(&ctl->nacc[p][1][blockIdx.x % kAccSlots], acc1);
    }
    if (MODE != 0) {
        if (tid == 0) { stat[0] = 0; stat[1] = 0; stat[2] = 0; }
        __syncthreads();
        const uint32_t t = wave_sum(ntests), f = wave_sum(nfall), c = wave_sum(ncand);
        if (lane == 0) {
            atomicAdd(&stat[0], t);
            atomicAdd(&stat[1], f);
            atomicAdd(&stat[2], c);
        }
        __syncthreads();
        if (tid == 0 && stat[0]) {
            atomicAdd(&ctl->fstat[0][blockIdx.x % kAccSlots], (unsigned long long)stat[0]);
            atomicAdd(&ctl->fstat[1][blockIdx.x % kAccSlots], (unsigned long long)stat[1]);
            atomicAdd(&ctl->fstat[2][blockIdx.x % kAccSlots], (unsigned long long)stat[2]);
        }
    }
}


// ---------------------------------------------------------------------------
// finishing: once no segment has more than kFinCap points, one block takes
// each segment and completes its recursion in LDS, level by level (the same
// rounds, with the same classification and the same argmax rule, but with no
// launches in between).  Every apex gets a hull id from a counter and is
// linked between its edge's ends, as the segment kernel does.
// ---------------------------------------------------------------------------
static_assert(kFinCap == QH_FINISH_CAP && kFinCap % kBlock == 0, "finishing capacity");
constexpr int kFinPer = kFinCap / kBlock;          // points per thread
constexpr int kFinPieces = 2 * (kTile + 2) + 8;    // pieces of the two tiles a segment may meet
constexpr int kFinChunk = (kFinCap + kBlock - 1) / kBlock;  // sub-segments per thread in the scan

struct FinSmem {
    int32_t px0[kFinCap], py0[kFinCap], pi0[kFinCap];   // point buffer 0
    union {
        struct {
            int32_t pv[kFinPieces], pp[kFinPieces];     // piece tables (loading only)
        } ld;
        struct {
            int32_t px1[kFinCap], py1[kFinCap], pi1[kFinCap];  // point buffer 1
            uint16_t sid[2][kFinCap];                   // sub-segment of every point
            int32_t sst[kFinCap + 4];                   // segment starts (set-up), then
                                                        // each vertex slot's successor
            uint32_t suv[kFinCap];                      // its ends: vertex slots u | v << 16
            uint64_t kmax[kFinCap];                     // argmax: distance, then tie key
            uint64_t kmin[kFinCap];
            uint32_t cnt[kFinCap];                      // child sizes c0 | c1 << 16
            int32_t sin[kFinCap];                       // its instance
            int32_t vx[kFinCap + 4], vy[kFinCap + 4];   // vertices: coordinates,
            int32_t vi[kFinCap + 4], vg[kFinCap + 4];   // input index, hull id
        } w;
    };
    uint32_t scan[kNW];
    int32_t s_base, s_ns, s_m;
};

// segments s0 .. s0 + M - 1 of round p in region R (consecutive, so their
// points are one range; M = 1 in the first split, where the points are the
// instance's input range): their points, edges u -> v and apexes f.  The
// levels treat the segments as the sub-segments of one
__device__ void finish_unit(const Ws2 &ws, const HullArgs &a, int p, int R, int s0, int M, bool init,
                            int nt0, int nt1, int hbase, FinSmem *sm) {
    Control *ctl = ws.ctl;
    const int tid = threadIdx.x;
    const SegGeo G0 = ws.geo(p, R)[s0];
    const SegGeo GL = ws.geo(p, R)[s0 + M - 1];
    const int start = G0.start, len = GL.start + GL.len - G0.start;
    // vertex slots: u and v of segment j at 2j and 2j + 1, then the apexes
    // of each level in order (at most one per point)
    if (M < 1 || M > kBlock || (init && M != 1) || len < 1 || len > kFinCap || 2 * M + len > kFinCap + 4) {
        if (tid == 0) atomicOr(&ctl->error, kErrInternal);  // the caller's bounds: never
        return;
    }
    SegGeo G;
    SegTop Tp;
    if (tid < M) {
        G = ws.geo(p, R)[s0 + tid];
        Tp = ws.top(p, R)[s0 + tid];
    }
    // the points into buffer 0
    if (init) {
        for (int j = tid; j < len; j += kBlock) {
            const int v = start + j;
            sm->px0[j] = a.x[v];
            sm->py0[j] = a.y[v];
            sm->pi0[j] = v;
        }
    } else {
        const int NR = R ? ctl->rs[p].n[1] : ctl->rs[p].n[0];
        const int ntR = R ? nt1 : nt0;
        const int npc = ctl->rs[p].npc[R];
        const int lt0 = start / kTile, lt1 = (start + len - 1) / kTile;
        const int32_t *kf = ws.kf(p, R);
        const int kA = kf[lt0];
        const int kB = (lt1 + 1 < ntR) ? kf[lt1 + 1] : npc - 1;
        const int K = kB - kA + 1;
        const bool ok = start + len <= NR && kA >= 0 && K >= 1 && K <= kFinPieces && kB < npc;
        if (ok) {
            for (int j = tid; j < K; j += kBlock) {
                sm->ld.pv[j] = ws.pv(p, R)[kA + j];
                sm->ld.pp[j] = ws.pp(p, R)[kA + j];
            }
        }
        __syncthreads();
        if (!ok) {
            if (tid == 0) atomicOr(&ctl->error, kErrInternal);
            return;
        }
        const int32_t *sx = ws.px(p, R), *sy = ws.py(p, R), *si = ws.pi(p, R);
        const int64_t cap = ws.cap_pts;
        int32_t bx[kFinPer], by[kFinPer], bi[kFinPer];
        bool bad = false;
#pragma unroll
        for (int k = 0; k < kFinPer; ++k) {
            const int j = tid + k * kBlock;
            bx[k] = by[k] = bi[k] = 0;
            if (j >= len) continue;
            const int v = start + j;
            const int sl = slot_of(sm->ld.pv, K, v);
            const int64_t ph = (int64_t)sm->ld.pp[sl] + (v - sm->ld.pv[sl]);
            if (ph < 0 || ph >= cap) { bad = true; continue; }
            bx[k] = sx[ph];
            by[k] = sy[ph];
            bi[k] = si[ph];
        }
        __syncthreads();  // the piece tables share LDS with the buffers below
#pragma unroll
        for (int k = 0; k < kFinPer; ++k) {
            const int j = tid + k * kBlock;
            if (j < len) { sm->px0[j] = bx[k]; sm->py0[j] = by[k]; sm->pi0[j] = bi[k]; }
        }
        if (bad) atomicOr(&ctl->error, kErrInternal);
    }
    // first split of a one-point instance: u = f
    const bool same = M == 1 && G0.fx == G0.ux && G0.fy == G0.uy;
    const bool defer = !same;
    if (tid < M) {
        const int u = 2 * tid, v = u + 1, f = 2 * M + tid;
        sm->w.vx[u] = G.ux; sm->w.vy[u] = G.uy; sm->w.vg[u] = Tp.uc;
        sm->w.vx[v] = G.vx; sm->w.vy[v] = G.vy; sm->w.vg[v] = Tp.vc;
        sm->w.vx[f] = G.fx; sm->w.vy[f] = G.fy; sm->w.vi[f] = Tp.fidx;
        sm->w.sst[tid] = G.start - start;
        sm->w.suv[tid] = (uint32_t)u | ((uint32_t)v << 16);
        sm->w.sin[tid] = Tp.inst;
        if (G.len < 1) atomicOr(&ctl->error, kErrInternal);
    }
    __syncthreads();
    // each point's segment: the last one starting at or before it
    for (int j = tid; j < len; j += kBlock) {
        int lo = 0, hi = M - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sm->w.sst[mid] <= j) lo = mid; else hi = mid - 1;
        }
        sm->w.sid[0][j] = (uint16_t)lo;
    }
    __syncthreads();
    int b = 0, m = len, ns = M, nv = 2 * M;
    for (int level = 0; ns > 0; ++level) {
        const int32_t *X = b ? sm->w.px1 : sm->px0;
        const int32_t *Y = b ? sm->w.py1 : sm->py0;
        const int32_t *I = b ? sm->w.pi1 : sm->pi0;
        const uint16_t *SID = sm->w.sid[b];
        int32_t px[kFinPer], py[kFinPer], pi[kFinPer], ps[kFinPer];
#pragma unroll
        for (int k = 0; k < kFinPer; ++k) {
            const int j = tid + k * kBlock;
            const bool in = j < m;
            px[k] = in ? X[j] : 0;
            py[k] = in ? Y[j] : 0;
            pi[k] = in ? I[j] : 0;
            ps[k] = in ? (int)SID[j] : -1;
        }
        // A. the apex of every sub-segment: farthest from u -> v, ties by the
        // tie key (the first level's apex is the segment's own)
        if (level > 0) {
            for (int t = tid; t < ns; t += kBlock) {
                sm->w.kmax[t] = 0;
                sm->w.kmin[t] = ~0ull;
            }
            __syncthreads();
            uint64_t d[kFinPer];
#pragma unroll
            for (int k = 0; k < kFinPer; ++k) {
                d[k] = 0;
                if (ps[k] < 0) continue;
                const uint32_t uv = sm->w.suv[ps[k]];
                const int u = (int)(uv & 0xffffu), v = (int)(uv >> 16);
                const int64_t dd = cross_i64(px[k], py[k], sm->w.vx[u], sm->w.vy[u], sm->w.vx[v], sm->w.vy[v]);
                if (dd <= 0) { atomicOr(&ctl->error, kErrInternal); continue; }
                d[k] = (uint64_t)dd;
                atomicMax(&sm->w.kmax[ps[k]], d[k]);
            }
            __syncthreads();
            uint64_t tk[kFinPer];
#pragma unroll
            for (int k = 0; k < kFinPer; ++k) {
                tk[k] = ~0ull;
                if (ps[k] < 0 || d[k] != sm->w.kmax[ps[k]]) continue;
                const uint32_t uv = sm->w.suv[ps[k]];
                const int u = (int)(uv & 0xffffu), v = (int)(uv >> 16);
                tk[k] = tie_key(px[k], py[k], pi[k], sm->w.vx[v] - sm->w.vx[u], sm->w.vy[v] - sm->w.vy[u]);
                atomicMin(&sm->w.kmin[ps[k]], tk[k]);
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kFinPer; ++k) {
                if (ps[k] < 0 || tk[k] != sm->w.kmin[ps[k]]) continue;
                const int at = nv + ps[k];
                sm->w.vx[at] = px[k];
                sm->w.vy[at] = py[k];
                sm->w.vi[at] = pi[k];
            }
        }
        // B. the apexes join the hull between their edge's ends: as links
        // between vertex slots, given hull ids when the levels end (one
        // claim on the global id counter per call, not one per level), or,
        // for the one-point instance of a first split, at once
        if (defer) {
            for (int t = tid; t < ns; t += kBlock) {
                const uint32_t uv = sm->w.suv[t];
                const int u = (int)(uv & 0xffffu), v = (int)(uv >> 16);
                const int at = nv + t;
                sm->w.sst[at] = v;
                sm->w.sst[u] = at;
                sm->w.vg[at] = sm->w.sin[t];  // the instance, until the ids are known
                sm->w.cnt[t] = 0;
            }
        }
        const bool link = !(level == 0 && same);
        if (!defer && tid == 0) sm->s_base = link ? (int)atomicAdd(&ctl->fin_ids, (unsigned)ns) : 0;
        __syncthreads();
        for (int t = tid; t < ns && !defer; t += kBlock) {
            const uint32_t uv = sm->w.suv[t];
            const int u = (int)(uv & 0xffffu), v = (int)(uv >> 16);
            const int at = nv + t;
            if (!link) {
                sm->w.vg[at] = sm->w.vg[u];
                ws.nxt[sm->w.vg[u]] = sm->w.vg[u];  // a one-point hull
            } else {
                const int gid = hbase + sm->s_base + t;
                sm->w.vg[at] = gid;
                if (gid < ws.hcap) {
                    ws.V[gid] = sm->w.vi[at];
                    ws.hinst[gid] = sm->w.sin[t];
                    ws.nxt[gid] = sm->w.vg[v];
                    ws.nxt[sm->w.vg[u]] = gid;
                } else {
                    atomicOr(&ctl->error, kErrHullCap);
                }
            }
            sm->w.cnt[t] = 0;
        }
        __syncthreads();
        // C. the children: outside u -> f, else outside f -> v, else dropped
        uint32_t ch[kFinPer], rk[kFinPer];
#pragma unroll
        for (int k = 0; k < kFinPer; ++k) {
            ch[k] = 2;
            rk[k] = 0;
            if (ps[k] < 0) continue;
            const uint32_t uv = sm->w.suv[ps[k]];
            const int u = (int)(uv & 0xffffu), v = (int)(uv >> 16), f = nv + ps[k];
            const int fx = sm->w.vx[f], fy = sm->w.vy[f];
            if (cross_i64(px[k], py[k], sm->w.vx[u], sm->w.vy[u], fx, fy) > 0) ch[k] = 0;
            else if (cross_i64(px[k], py[k], fx, fy, sm->w.vx[v], sm->w.vy[v]) > 0) ch[k] = 1;
            if (ch[k] < 2) {
                const uint32_t o = atomicAdd(&sm->w.cnt[ps[k]], ch[k] ? 0x10000u : 1u);
                rk[k] = ch[k] ? (o >> 16) : (o & 0xffffu);
            }
        }
        __syncthreads();
        // D. the next level's sub-segments: child 0 then child 1 of each, in
        // order (a scan over contiguous chunks of sub-segments)
        const int c0s = tid * kFinChunk, c1s = min(c0s + kFinChunk, ns);
        uint32_t cc[kFinChunk], uvs[kFinChunk];
        int32_t ins[kFinChunk];
        uint32_t loc = 0;  // new sub-segments | their points << 16
#pragma unroll
        for (int k = 0; k < kFinChunk; ++k) {
            const int t = c0s + k;
            cc[k] = t < c1s ? sm->w.cnt[t] : 0u;
            uvs[k] = t < c1s ? sm->w.suv[t] : 0u;
            ins[k] = t < c1s ? sm->w.sin[t] : 0;
            const uint32_t a0 = cc[k] & 0xffffu, a1 = cc[k] >> 16;
            loc += (a0 > 0 ? 1u : 0u) + (a1 > 0 ? 1u : 0u) + ((a0 + a1) << 16);
        }
        uint32_t sv[1] = {loc}, tot[1];
        block_excl_scan<kBlock, 1>(sv, tot, sm->scan);
        uint32_t nid = sv[0] & 0xffffu, npt = sv[0] >> 16;
#pragma unroll
        for (int k = 0; k < kFinChunk; ++k) {
            const int t = c0s + k;
            if (t >= c1s) continue;
            const uint32_t a0 = cc[k] & 0xffffu, a1 = cc[k] >> 16;
            const uint32_t u = uvs[k] & 0xffffu, v = uvs[k] >> 16, f = (uint32_t)(nv + t);
            uint32_t id0 = 0xffffu, id1 = 0xffffu;
            const uint32_t st0 = npt, st1 = npt + a0;
            if (a0 > 0) {
                id0 = nid;
                sm->w.suv[nid] = u | (f << 16); sm->w.sin[nid] = ins[k];
                ++nid;
            }
            if (a1 > 0) {
                id1 = nid;
                sm->w.suv[nid] = f | (v << 16); sm->w.sin[nid] = ins[k];
                ++nid;
            }
            npt += a0 + a1;
            // where each child's points go (read by the scatter below)
            sm->w.kmax[t] = (uint64_t)st0 | ((uint64_t)st1 << 32);
            sm->w.kmin[t] = (uint64_t)id0 | ((uint64_t)id1 << 32);
        }
        __syncthreads();
        // E. the points into the other buffer
        int32_t *Xo = b ? sm->px0 : sm->w.px1;
        int32_t *Yo = b ? sm->py0 : sm->w.py1;
        int32_t *Io = b ? sm->pi0 : sm->w.pi1;
        uint16_t *SIDo = sm->w.sid[b ^ 1];
#pragma unroll
        for (int k = 0; k < kFinPer; ++k) {
            if (ch[k] > 1) continue;
            const int pos = (int)((sm->w.kmax[ps[k]] >> (32 * ch[k])) & 0xffffffffu) + (int)rk[k];
            const int id = (int)((sm->w.kmin[ps[k]] >> (32 * ch[k])) & 0xffffffffu);
            if (pos >= kFinCap || id >= kFinCap) { atomicOr(&ctl->error, kErrInternal); continue; }
            Xo[pos] = px[k];
            Yo[pos] = py[k];
            Io[pos] = pi[k];
            SIDo[pos] = (uint16_t)id;
        }
        nv += ns;
        ns = (int)(tot[0] & 0xffffu);
        m = (int)(tot[0] >> 16);
        b ^= 1;
        if (nv + ns > kFinCap + 3) {  // more apexes than points: never
            if (tid == 0) atomicOr(&ctl->error, kErrInternal);
            ns = 0;
        }
        __syncthreads();
    }
    if (!defer) return;
    // the hull ids of the apexes (slots 2M .. nv - 1, in slot order) and the
    // links: every apex and every segment's u (its new successor); the v
    // ends keep theirs
    const int na = nv - 2 * M;
    if (tid == 0) sm->s_base = na > 0 ? (int)atomicAdd(&ctl->fin_ids, (unsigned)na) : 0;
    __syncthreads();
    const int gb = hbase + sm->s_base;
    for (int sl = tid; sl < nv; sl += kBlock) {
        if (sl < 2 * M && (sl & 1)) continue;
        const int nx = sm->w.sst[sl];
        const int gn = nx < 2 * M ? sm->w.vg[nx] : gb + (nx - 2 * M);
        const int gid = sl < 2 * M ? sm->w.vg[sl] : gb + (sl - 2 * M);
        if (sl < 2 * M && gn < ws.hcap) {
            ws.nxt[gid] = gn;
        } else if (sl >= 2 * M && gid < ws.hcap && gn < ws.hcap) {
            ws.V[gid] = sm->w.vi[sl];
            ws.hinst[gid] = sm->w.vg[sl];
            ws.nxt[gid] = gn;
        } else {
            atomicOr(&ctl->error, kErrHullCap);
        }
    }
}

// every segment of round p, one per block
__device__ void phase_finish(const Ws2 &ws, const HullArgs &a, int r, FinSmem *sm) {
    Control *ctl = ws.ctl;
    const int p = r & 1;
    if (ctl->error) return;
    const RoundState *rs = &ctl->rs[p];
    const int S0 = rs->s[0], S1 = rs->s[1];
    const int nt0 = (rs->n[0] + kTile - 1) / kTile, nt1 = (rs->n[1] + kTile - 1) / kTile;
    const int hbase = rs->hbase;
    if (fin_each(ctl, r, a)) {
        for (int g = blockIdx.x; g < S0 + S1; g += gridDim.x) {
            const int R = g < S0 ? 0 : 1;
            finish_unit(ws, a, p, R, R ? g - S0 : g, 1, r == 0, nt0, nt1, hbase, sm);
            __syncthreads();
        }
        return;
    }
    // many small segments: each block takes a range of the segments (in
    // table order, region 0 then 1) and finishes them in runs: the next
    // segments of a region (at most kBlock) that hold at most kFinUnit points
    // together, always at least one (no segment is larger)
    const int tid = threadIdx.x;
    const int S = S0 + S1;
    const int Q = (S + (int)gridDim.x - 1) / (int)gridDim.x;
    const int glo = min(S, (int)blockIdx.x * Q), ghi = min(S, glo + Q);
    for (int R = 0; R < 2; ++R) {
        const int off = R ? S0 : 0, SR = R ? S1 : S0;
        int s = max(glo - off, 0);
        const int se = min(ghi - off, SR);
        while (s < se) {
            const int st = ws.geo(p, R)[s].start;
            const int cand = min(kBlock, se - s);
            bool fits = false;
            if (tid < cand) {
                const SegGeo G = ws.geo(p, R)[s + tid];
                fits = G.start + G.len - st <= kFinUnit;
            }
            // the segments are consecutive, so their ends rise: the ones that
            // fit are a prefix
            const int M = __syncthreads_count(fits);
            if (M < 1) {
                if (tid == 0) atomicOr(&ctl->error, kErrInternal);
                return;
            }
            finish_unit(ws, a, p, R, s, M, false, nt0, nt1, hbase, sm);
            __syncthreads();
            s += M;
        }
    }
}

// Merge the record slots of one segment, both children, with one wave (the
// result is valid in its last lane).
// In the round after the split (sub = the region's tile offset) the blocks'
// tile ranges start at multiples of T in each region's own tile numbers.
__device__ __forceinline__ void wave_merge_seg(const Ws2 &ws, int p, int R, int nt0, int T, int t0,
                                               int t1, int sub, Best &m0, Best &m1) {
    const TileInfo *ti = ws.tinfo(p, R);
    const int off = R ? nt0 : 0;
    const bool s0 = ti[t0 - off].single != 0, s1 = ti[t1 - off].single != 0;
    Best acc0 = best_none(), acc1 = best_none();
    const int ns = seg_slots(T, t0 - sub, t1 - sub);
    // four slots per lane requested at a time, then merged (order-free)
    for (int k0 = lane_id(); k0 < ns; k0 += 4 * kWave) {
        Best c0[4], c1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            c0[u] = best_none();
            c1[u] = best_none();
            bool last;
            const int k = k0 + u * kWave;
            const int t = k < ns ? seg_slot(T, t0 - sub, t1 - sub, s0, s1, k, last) : -1;
            if (t >= 0) {
                const Best *rec = last ? ws.recL : ws.recF;
                c0[u] = rec[(t + sub) * 2 + 0];
                c1[u] = rec[(t + sub) * 2 + 1];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            rec_merge(acc0, c0[u]);
            rec_merge(acc1, c1[u]);
        }
    }
    wave_rec63(acc0);
    wave_rec63(acc1);
    m0 = acc0;
    m1 = acc1;
}
// ---------------------------------------------------------------------------
// segments: hull insertion, multi-tile argmax, next segment table
// ---------------------------------------------------------------------------
__device__ __forceinline__ void phase_segments(const Ws2 &ws, const HullArgs &a, int r, char *smem) {
    Control *ctl = ws.ctl;
    SegSmem *sm = reinterpret_cast<SegSmem *>(smem);
    const int p = r & 1, q = p ^ 1;
    RoundState *rs = &ctl->rs[p];
    RoundState *rn = &ctl->rs[q];
    const int S0 = rs->s[0], S1 = rs->s[1];
    const int Stot = S0 + S1;
    const int hbase = rs->hbase;
    const int nt0 = (rs->n[0] + kTile - 1) / kTile;
    const int nt1 = (rs->n[1] + kTile - 1) / kTile;
    // survivors of this round per region (summed by the round kernel's blocks)
    const int An0 = (int)wave_sum(ctl->nacc[p][0][lane_id()]), An1 = (int)wave_sum(ctl->nacc[p][1][lane_id()]);
    // The split (r = 0) keeps no point: its children are the instances'
    // input ranges (both regions of the next round are the input), and every
    // child is made, even an empty one, so that every input tile has its
    // record.  The round after it (r = 1) reads its tiles per region in the
    // input's tile numbers.
    const bool ro0 = r == 0, ro1 = r == 1;
    const int nin0 = rs->n[0] + rs->n[1];
    const int Nn0 = ro0 ? nin0 : An0, Nn1 = ro0 ? nin0 : An1;
    const int nsegt = (Stot + kSegBlock - 1) / kSegBlock;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;

    if (fin_mode(ctl, r, a)) {
        // the segments were finished by the finishing kernel: no next round
        if (blockIdx.x == 0 && tid == 0) {
            RoundState z = {};
            z.hbase = hbase + (int32_t)ctl->fin_ids;
            *rn = z;
            ctl->fin_round = r;
            ctl->fin_runs = fin_each(ctl, r, a) ? 0 : 1;
        }
        if (blockIdx.x == 0 && tid < kAccSlots) {
            ctl->nacc[q][0][tid] = 0;
            ctl->nacc[q][1][tid] = 0;
        }
        return;
    }
    if (blockIdx.x == 0 && tid == 0) {
        rn->seg_ctr = 0;
        rn->piece_ctr = 0;
        rn->n[0] = Nn0;
        rn->n[1] = Nn1;
        const unsigned long long nin = (unsigned long long)(rs->n[0] + rs->n[1]);
        if (nin) {
            if (ro0) {
                ctl->first_in += nin;
                ctl->first_out += (unsigned long long)(An0 + An1);
            } else if (ro1) {
                ctl->second_in += (unsigned long long)rs->n[0];  // both regions are the input
                ctl->second_out += (unsigned long long)(An0 + An1);
            } else {
                ctl->points_in += nin;
                ctl->points_out += (unsigned long long)(An0 + An1);
            }
            ctl->rounds_with_work += 1ull;
        }
    }
    if (blockIdx.x == 0 && tid < kAccSlots) {
        ctl->nacc[q][0][tid] = 0;
        ctl->nacc[q][1][tid] = 0;
    }
    for (int i = blockIdx.x * kSegBlock + tid; i < 2 * nsegt + 4 && i < ws.s4cap; i += gridDim.x * kSegBlock) {
        ws.st4(q)[i] = 0;
        ws.st4b(q)[i] = 0;
    }
    for (int i = blockIdx.x * kSegBlock + tid; i < ws.s5cap; i += gridDim.x * kSegBlock) {
        ws.st5(q)[i] = 0;
        ws.st5b(q)[i] = 0;
    }
    if (Stot == 0 || ctl->error) {
        if (blockIdx.x == 0 && tid == 0) {
            rn->s[0] = 0; rn->s[1] = 0; rn->hbase = hbase;
            rn->npc[0] = 0; rn->npc[1] = 0;
        }
        return;
    }

    while (true) {
        if (tid == 0) {
            sm->s_tile = (int32_t)atomicAdd(&rs->seg_ctr, 1u);
            sm->qn_apex = 0;
            sm->qn_map = 0;
        }
        __syncthreads();
        const int tile = __builtin_amdgcn_readfirstlane(sm->s_tile);
        if (tile >= nsegt) break;
        const int g = tile * kSegBlock + tid;
        const bool valid = g < Stot;
        const int R = g < S0 ? 0 : 1;
        const int s = g - (R ? S0 : 0);
        SegGeo G = {};
        SegTop Tp = {};
        if (valid) {
            G = ws.geo(p, R)[s];
            Tp = ws.top(p, R)[s];
        }

        // the children's argmax and counts: merged over the records of the
        // tiles the segment spans
        Best b0 = best_none(), b1 = best_none();
        const int t0 = (R ? nt0 : 0) + G.start / kTile;
        const int t1 = (R ? nt0 : 0) + (G.start + G.len - 1) / kTile;
        const int T = max(1, ctl->tper[p]);
        const int sub = (ro1 && R) ? nt0 : 0;  // see wave_merge_seg
        if (valid) {
            if (t0 == t1) {
                b0 = ws.adir[g * 2 + 0];
                b1 = ws.adir[g * 2 + 1];
            } else if (seg_slots(T, t0 - sub, t1 - sub) <= 12) {
                const int ns = seg_slots(T, t0 - sub, t1 - sub);
                const TileInfo *ti = ws.tinfo(p, R);
                const int off = R ? nt0 : 0;
                const bool s0 = ti[t0 - off].single != 0, s1 = ti[t1 - off].single != 0;
                // four slots' records requested at a time, then merged (the
                // merge is order-free), so a thread waits ns / 4 times, not ns
                for (int k0 = 0; k0 < ns; k0 += 4) {
                    Best c0[4], c1[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        c0[u] = best_none();
                        c1[u] = best_none();
                        bool last;
                        const int t = k0 + u < ns ? seg_slot(T, t0 - sub, t1 - sub, s0, s1, k0 + u, last) : -1;
                        if (t >= 0) {
                            const Best *rec = last ? ws.recL : ws.recF;
                            c0[u] = rec[(t + sub) * 2 + 0];
                            c1[u] = rec[(t + sub) * 2 + 1];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        rec_merge(b0, c0[u]);
                        rec_merge(b1, c1[u]);
                    }
                }
            } else {
                const int qi = atomicAdd(&sm->qn_apex, 1);
                sm->q_apex[qi] = (int16_t)tid;
                sm->o_t0[tid] = t0;
                sm->o_t1[tid] = t1;
            }
        }
        __syncthreads();
        // segments over many slots: one wave each, the block's waves side by side
        const int nqa = sm->qn_apex;
        for (int qi = wv; qi < nqa; qi += kSegBlock / kWave) {
            const int own = sm->q_apex[qi];
            const int a0 = sm->o_t0[own], a1 = sm->o_t1[own];
            const int Ro = own + tile * kSegBlock < S0 ? 0 : 1;
            Best m0, m1;
            wave_merge_seg(ws, p, Ro, nt0, T, a0, a1, (ro1 && Ro) ? nt0 : 0, m0, m1);
            if (lane == kWave - 1) {
                sm->qres[own * 2 + 0] = m0;
                sm->qres[own * 2 + 1] = m1;
            }
        }
        __syncthreads();
        if (valid && t0 != t1 && seg_slots(T, t0 - sub, t1 - sub) > 12) {
            b0 = sm->qres[tid * 2 + 0];
            b1 = sm->qres[tid * 2 + 1];
        }
        const int c0 = valid ? b0.cnt : 0, c1 = valid ? b1.cnt : 0;
        // the winners' coordinates (the one-segment records carry the index only)
        if (valid && b0.key1) { b0.x = a.x[b0.idx]; b0.y = a.y[b0.idx]; }
        if (valid && b1.key1) { b1.x = a.x[b1.idx]; b1.y = a.y[b1.idx]; }

        // the apex f of this segment joins the hull between u and v
        int fc = 0;
        if (valid && Tp.fidx < 0) {
            // an empty child of the split: no apex, its hull id stays unused
            if (hbase + g < ws.hcap) ws.nxt[hbase + g] = -1;
        } else if (valid) {
            const bool same = (G.fx == G.ux) && (G.fy == G.uy);
            fc = same ? Tp.uc : hbase + g;
            if (!same) {
                if (fc < ws.hcap) {
                    ws.V[fc] = Tp.fidx;
                    ws.hinst[fc] = Tp.inst;
                    ws.nxt[fc] = Tp.vc;
                } else {
                    atomicOr(&ctl->error, kErrHullCap);
                }
            }
            ws.nxt[Tp.uc] = fc;
        }

        // ids of the non-empty children, and their start offsets (children of
        // earlier segments come first, in both regions of the next round)
        const bool has0 = valid && (ro0 || c0 > 0), has1 = valid && (ro0 || c1 > 0);
        const int len0 = ro0 ? G.len : c0, len1 = ro0 ? G.len : c1;  // the children's ranges
        uint32_t v[2] = {has0 ? 1u : 0u, has1 ? 1u : 0u}, tot[2];
        block_excl_scan<kSegBlock, 2>(v, tot, sm->scan);
        if (wv == 0) {
            const uint64_t ex = lookback_excl(ws.st4(p), tile, pack2(tot[0], tot[1]), &ctl->error);
            if (lane == 0) sm->s_ex = ex;
        }
        uint32_t w[2] = {(uint32_t)len0, (uint32_t)len1}, wt[2];
        block_excl_scan<kSegBlock, 2>(w, wt, sm->scan2);
        if (wv == 0) {
            const uint64_t ex = lookback_excl(ws.st4b(p), tile, pack2(wt[0], wt[1]), &ctl->error);
            if (lane == 0) sm->s_ex2 = ex;
        }
        __syncthreads();
        const int id0 = (int)(unpackA(sm->s_ex) + v[0]);
        const int id1 = (int)(unpackB(sm->s_ex) + v[1]);
        const int st0 = (int)(unpackA(sm->s_ex2) + w[0]);
        const int st1 = (int)(unpackB(sm->s_ex2) + w[1]);
        const bool ok0 = has0 && id0 < ws.scap, ok1 = has1 && id1 < ws.scap;
        if ((has0 && !ok0) || (has1 && !ok1)) atomicOr(&ctl->error, kErrSegCap);
        {
            // the largest segment of the next round
            uint32_t mc = (uint32_t)max(ok0 ? c0 : 0, ok1 ? c1 : 0);
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) mc = max(mc, (uint32_t)__shfl_xor((int)mc, o));
            if (lane == 0 && mc) atomicMax(&ctl->maxseg[q], (int32_t)mc);
        }

        // child segments of the next round
        if (ok0) {
            SegGeo cg;
            cg.start = st0; cg.len = len0;
            cg.ux = G.ux; cg.uy = G.uy;
            cg.fx = b0.x; cg.fy = b0.y;
            cg.vx = G.fx; cg.vy = G.fy;
            ws.geo(q, 0)[id0] = cg;
            SegTop ct;
            ct.fidx = c0 > 0 ? b0.idx : -1; ct.uc = Tp.uc; ct.vc = fc; ct.inst = Tp.inst;
            ws.top(q, 0)[id0] = ct;
        }
        if (ok1) {
            SegGeo cg;
            cg.start = st1; cg.len = len1;
            cg.ux = G.fx; cg.uy = G.fy;
            cg.fx = b1.x; cg.fy = b1.y;
            cg.vx = G.vx; cg.vy = G.vy;
            ws.geo(q, 1)[id1] = cg;
            SegTop ct;
            ct.fidx = c1 > 0 ? b1.idx : -1; ct.uc = fc; ct.vc = Tp.vc; ct.inst = Tp.inst;
            ws.top(q, 1)[id1] = ct;
        }
        // the child's last tile holds further segments unless the child runs
        // to the tile's end: list it for the multi-segment round kernel
        {
            const int ntn0 = (Nn0 + kTile - 1) / kTile;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const bool ok = c == 0 ? ok0 : ok1;
                const int st = c == 0 ? st0 : st1;
                const int ln = c == 0 ? len0 : len1;
                const int ka = (st + kTile - 1) / kTile, kb = (st + ln + kTile - 1) / kTile;
                const int Nc = c == 0 ? Nn0 : Nn1;
                const bool multi = ok && kb > ka && (st + ln) < min(kb * kTile, Nc);
                ml_append(ws, q, rn, multi, (c ? ntn0 : 0) + kb - 1);
            }
        }
        // tile records of the next round: tiles whose first point lies in a
        // child; a child over many tiles is written by the whole block
        for (int c = 0; c < 2; ++c) {
            const bool ok = c == 0 ? ok0 : ok1;
            if (!ok) continue;
            const int id = c == 0 ? id0 : id1;
            const int st = c == 0 ? st0 : st1;
            const int ln = c == 0 ? len0 : len1;
            const int ka = (st + kTile - 1) / kTile;
            const int kb = (st + ln + kTile - 1) / kTile;
            if (kb - ka <= 4) {
                TileInfo ti;
                ti.seg = id;
                ti.start = st;
                ti.end = st + ln;
                for (int kk = ka; kk < kb; ++kk) {
                    ti.single = ti.end >= min((kk + 1) * kTile, c == 0 ? Nn0 : Nn1) ? 1 : 0;
                    ws.tinfo(q, c)[kk] = ti;
                }
            } else {
                const int qi = atomicAdd(&sm->qn_map, 1);
                sm->q_map[qi] = (int16_t)(tid * 2 + c);
                sm->o_ka[tid * 2 + c] = ka;
                sm->o_kb[tid * 2 + c] = kb;
                sm->o_id[tid * 2 + c] = id;
                sm->o_st[tid * 2 + c] = st;
                sm->o_en[tid * 2 + c] = st + ln;
            }
        }
        __syncthreads();
        const int nqm = sm->qn_map;
        for (int qi = 0; qi < nqm; ++qi) {
            const int o = sm->q_map[qi];
            const int c = o & 1;
            const int ka = sm->o_ka[o], kb = sm->o_kb[o], id = sm->o_id[o];
            // the child's extent from LDS: no wait on a global load per child
            TileInfo ti;
            ti.seg = id;
            ti.start = sm->o_st[o];
            ti.end = sm->o_en[o];
            for (int kk = ka + tid; kk < kb; kk += kSegBlock) {
                ti.single = ti.end >= min((kk + 1) * kTile, c == 0 ? Nn0 : Nn1) ? 1 : 0;
                ws.tinfo(q, c)[kk] = ti;
            }
        }
        if (tile == nsegt - 1 && tid == 0) {
            const int n0n = (int)(unpackA(sm->s_ex) + tot[0]);
            const int n1n = (int)(unpackB(sm->s_ex) + tot[1]);
            const bool capbad = hbase + Stot > ws.hcap || n0n > ws.scap || n1n > ws.scap;
            if (capbad) atomicOr(&ctl->error, kErrHullCap);
            rn->s[0] = capbad ? 0 : n0n;
            rn->s[1] = capbad ? 0 : n1n;
            rn->hbase = hbase + Stot;
            atomicMax(&ctl->max_segments, n0n + n1n);
            ctl->rounds_done += 1;
        }
        __syncthreads();
    }

    // The next round's piece table: the survivors tile t of this round wrote
    // to region c (at t * kTile) are the next input's virtual range that
    // starts at the exclusive sum of the earlier tiles' counts.  Non-empty
    // pieces are listed in order with their virtual and physical starts, and
    // every next-round tile gets the piece holding its first point.
    __syncthreads();  // every thread has read the last segment-tile claim
    if (ro0) {
        // the next round reads the input: no piece table
        if (blockIdx.x == 0 && tid == 0) { rn->npc[0] = 0; rn->npc[1] = 0; }
        return;
    }
    const int NT = nt0 + nt1;
    constexpr int kPer = kSegBlock * kPieceItems;
    const int npt = (NT + kPer - 1) / kPer;
    while (true) {
        if (tid == 0) sm->s_tile = (int32_t)atomicAdd(&rs->piece_ctr, 1u);
        __syncthreads();
        const int pt = __builtin_amdgcn_readfirstlane(sm->s_tile);
        if (pt >= npt) break;
        const int t0 = pt * kPer + tid * kPieceItems;
        uint32_t cp[kPieceItems];
        uint32_t v[4] = {0u, 0u, 0u, 0u}, tot[4];
#pragma unroll
        for (int i = 0; i < kPieceItems; ++i) {
            const int t = t0 + i;
            cp[i] = t < NT ? ws.tcnt(p)[t] : 0u;
            const uint32_t a0 = cp[i] & 0xffffu, a1 = cp[i] >> 16;
            v[0] += a0;
            v[1] += a1;
            v[2] += a0 ? 1u : 0u;
            v[3] += a1 ? 1u : 0u;
        }
        block_excl_scan<kSegBlock, 4>(v, tot, sm->pscan);
        if (wv == 0) {
            const uint64_t ex = lookback_excl(ws.st5(p), pt, pack2(tot[0], tot[1]), &ctl->error);
            if (lane == 0) sm->s_ex = ex;
        } else if (wv == 1) {
            const uint64_t ex = lookback_excl(ws.st5b(p), pt, pack2(tot[2], tot[3]), &ctl->error);
            if (lane == 0) sm->s_ex2 = ex;
        }
        __syncthreads();
        int32_t V[2] = {(int32_t)(unpackA(sm->s_ex) + v[0]), (int32_t)(unpackB(sm->s_ex) + v[1])};
        int32_t K[2] = {(int32_t)(unpackA(sm->s_ex2) + v[2]), (int32_t)(unpackB(sm->s_ex2) + v[3])};
        const int Nn[2] = {Nn0, Nn1};
        bool bad = false;
#pragma unroll
        for (int i = 0; i < kPieceItems; ++i) {
            const int t = t0 + i;
            if (t >= NT) break;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int32_t cnt = (int32_t)(c == 0 ? (cp[i] & 0xffffu) : (cp[i] >> 16));
                if (cnt == 0) continue;
                if (K[c] >= ws.tcap || V[c] + cnt > Nn[c]) {
                    bad = true;
                    continue;
                }
                ws.pv(q, c)[K[c]] = V[c];
                // (after the split, region 1's tiles end at the end of the
                // slot of input tile t - nt0)
                ws.pp(q, c)[K[c]] = (ro1 && t >= nt0) ? (t - nt0) * kTile + kTile - cnt : t * kTile;
                // next-round tiles whose first point lies in this piece
                for (int tt = (V[c] + kTile - 1) / kTile; tt * kTile < V[c] + cnt && tt < ws.tcap; ++tt)
                    ws.kf(q, c)[tt] = K[c];
                K[c] += 1;
                V[c] += cnt;
            }
        }
        if (bad) atomicOr(&ctl->error, kErrInternal);
        if (pt == npt - 1 && tid == kSegBlock - 1) {
            // the last thread of the last block: totals, sentinels
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (V[c] != Nn[c] || K[c] > ws.tcap) {
                    atomicOr(&ctl->error, kErrInternal);
                    continue;
                }
                ws.pv(q, c)[K[c]] = V[c];
                ws.pp(q, c)[K[c]] = 0;
                rn->npc[c] = K[c];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// output: rank the hull cycles (pointer jumping), CCW index lists
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rank_init_one(const Ws2 &ws, int x, int32_t &su, int32_t &di) {
    const int nx = ws.nxt[x];
    if (nx < 0) { su = x; di = 0; return; }
    const bool term = (nx == ws.hinst[x]);   // next is the instance's first vertex
    su = term ? x : nx;
    di = term ? 0 : 1;
}

// ---------------------------------------------------------------------------
// output kernels
// ---------------------------------------------------------------------------
// small hulls: pointer jumping in one block's LDS (a block of the device's
// largest size, so each jump is a few LDS loads per thread)
constexpr int kRankBlock = 1024;
__global__ __launch_bounds__(kRankBlock) void k_rank_small(Ws2 ws, int32_t H, int32_t steps) {
    __shared__ RankSmem sm;
    for (int x = threadIdx.x; x < H; x += kRankBlock) rank_init_one(ws, x, sm.su[x], sm.di[x]);
    __syncthreads();
    constexpr int PER = kRankSmallCap / kRankBlock;
    for (int itr = 0; itr < steps; ++itr) {
        int ns[PER], nd[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int x = threadIdx.x + j * kRankBlock;
            if (x < H) {
                const int s = sm.su[x];
                nd[j] = sm.di[x] + sm.di[s];
                ns[j] = sm.su[s];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int x = threadIdx.x + j * kRankBlock;
            if (x < H) { sm.su[x] = ns[j]; sm.di[x] = nd[j]; }
        }
        __syncthreads();
    }
    for (int x = threadIdx.x; x < H; x += kRankBlock) ws.dist(0)[x] = sm.di[x];
}

__global__ void k_rank_init(Ws2 ws, int32_t H) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < H) rank_init_one(ws, x, ws.succ(0)[x], ws.dist(0)[x]);
}

__global__ void k_rank_step(Ws2 ws, int32_t H, int32_t src) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= H) return;
    const int s = ws.succ(src)[x];
    ws.dist(src ^ 1)[x] = ws.dist(src)[x] + ws.dist(src)[s];
    ws.succ(src ^ 1)[x] = ws.succ(src)[s];
}

// hull sizes per instance and their exclusive scan (one block)
__global__ __launch_bounds__(kBlock) void k_hull_offsets(Ws2 ws, HullArgs a, int32_t src) {
    __shared__ ScanSmem sm;
    Control *ctl = ws.ctl;
    if (threadIdx.x == 0) sm.carry = 0;
    __syncthreads();
    for (int base = 0; base < a.k; base += kBlock) {
        const int i = base + (int)threadIdx.x;
        uint32_t h = 0;
        if (i < a.k && ws.nxt[i] >= 0) h = (uint32_t)ws.dist(src)[i] + 1u;
        uint32_t v[1] = {h}, tot[1];
        block_excl_scan<kBlock, 1>(v, tot, sm.scratch);
        if (i < a.k) a.hull_offsets[i] = (int64_t)(sm.carry + v[0]);
        __syncthreads();
        if (threadIdx.x == 0) sm.carry += tot[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.hull_offsets[a.k] = (int64_t)sm.carry;
        ctl->h_total = (long long)sm.carry;
    }
}

__global__ void k_emit(Ws2 ws, HullArgs a, int32_t H, int32_t src) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= H || ws.nxt[x] < 0) return;
    const int i = ws.hinst[x];
    const int64_t base = a.hull_offsets[i];
    const int64_t h = a.hull_offsets[i + 1] - base;
    const int64_t pos = base + (h - 1 - ws.dist(src)[x]);
    if (pos < base || pos >= base + h || pos >= a.n) {
        atomicOr(&ws.ctl->error, kErrInternal);
        return;
    }
    a.hull_idx[pos] = (int32_t)(ws.V[x] - a.offsets[i]);
}

// ---------------------------------------------------------------------------
// the other kernels: one phase each
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_instances(Ws2 ws, HullArgs a) {
    __shared__ ScanSmem sm;
    phase_instances(ws, a, reinterpret_cast<char *>(&sm));
}

__global__ __launch_bounds__(kBlock) void k_setup(Ws2 ws, HullArgs a) { phase_setup(ws, a); }

__global__ __launch_bounds__(kBlock) void k_extremes(Ws2 ws, HullArgs a) {
    __shared__ ExtSmem sm;
    phase_extremes(ws, a, reinterpret_cast<char *>(&sm));
}

__global__ __launch_bounds__(kBlock) void k_extremes_final(Ws2 ws, HullArgs a) {
    __shared__ SegSmem sm;
    phase_extremes_final(ws, a, reinterpret_cast<char *>(&sm));
}

// (the exact form fits in 128 registers: four waves per SIMD)
template <int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MODE == 0 ? 4 : 3)))
void k_round(Ws2 ws, HullArgs a, int32_t r) {
    __shared__ FastSmem sm;
    if (ws.ctl->setup_error) return;
    phase_round_fast<MODE>(ws, a, r, reinterpret_cast<char *>(&sm));
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_split(Ws2 ws, HullArgs a) {
    __shared__ SplitSmem sm;
    if (ws.ctl->setup_error) return;
    phase_split<MODE>(ws, a, reinterpret_cast<char *>(&sm));
}

template <int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MODE == 0 ? 4 : 1)))
void k_round_ro1(Ws2 ws, HullArgs a) {
    __shared__ Ro1Smem sm;
    if (ws.ctl->setup_error) return;
    phase_round_ro1<MODE>(ws, a, reinterpret_cast<char *>(&sm));
}

// The multi-segment kernel needs about 37 KB of LDS, the finishing pass
// about 73 KB; in one kernel the larger size would hold the multi-segment
// kernel to two workgroups per CU in every round.  So the finishing pass is
// a kernel of its own, launched from round fin_from on (the round the
// context's last call finished in; 0 on a first call) and leaving at once
// unless the round finishes; rounds before fin_from do not finish.
// (the filter form held to 128 registers: four waves per SIMD, as the exact)
template <int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MODE == 0 ? 1 : 4)))
void k_round_multi(Ws2 ws, HullArgs a, int32_t r) {
    __shared__ RoundSmem sm;
    if (ws.ctl->setup_error) return;
    if (fin_mode(ws.ctl, r, a)) return;  // the finishing kernel takes the round
    phase_round_multi<MODE>(ws, a, r, reinterpret_cast<char *>(&sm));
}

__global__ __launch_bounds__(kBlock) void k_finish(Ws2 ws, HullArgs a, int32_t r) {
    __shared__ FinSmem sm;
    if (ws.ctl->setup_error) return;
    if (!fin_mode(ws.ctl, r, a)) return;
    phase_finish(ws, a, r, &sm);
}

__global__ __launch_bounds__(kSegBlock) void k_segments(Ws2 ws, HullArgs a, int32_t r) {
    __shared__ SegSmem sm;
    phase_segments(ws, a, r, reinterpret_cast<char *>(&sm));
}

// ---------------------------------------------------------------------------
// host-side launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_setup(const Ws2 &ws, const HullArgs &a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_instances, dim3(1), dim3(kBlock), 0, st, ws, a);
    hipLaunchKernelGGL(k_setup, dim3(grid), dim3(kBlock), 0, st, ws, a);
    return hipGetLastError();
}

hipError_t launch_extremes(const Ws2 &ws, const HullArgs &a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_extremes, dim3(grid), dim3(kBlock), 0, st, ws, a);
    hipLaunchKernelGGL(k_extremes_final, dim3(std::max(1, std::min(a.k, grid))), dim3(kBlock), 0, st, ws, a);
    return hipGetLastError();
}

hipError_t launch_round(const Ws2 &ws, const HullArgs &a, int mode, int32_t r, int grid,
                        int grid_multi, int grid_fin, hipStream_t st) {
    // round 0: the read-only split; round 1: one pass over the input for both
    // of the split's children; later rounds: the survivors through the pieces
    const int gs = a.grid_split > 0 ? a.grid_split : grid, g1 = a.grid_ro1 > 0 ? a.grid_ro1 : grid;
    if (mode == 0) {
        if (r == 0) hipLaunchKernelGGL(k_split<0>, dim3(gs), dim3(kBlock), 0, st, ws, a);
        else if (r == 1) hipLaunchKernelGGL(k_round_ro1<0>, dim3(g1), dim3(kBlock), 0, st, ws, a);
        else hipLaunchKernelGGL(k_round<0>, dim3(grid), dim3(kBlock), 0, st, ws, a, r);
        hipLaunchKernelGGL(k_round_multi<0>, dim3(grid_multi), dim3(kBlock), 0, st, ws, a, r);
    } else {
        if (r == 0) hipLaunchKernelGGL(k_split<1>, dim3(gs), dim3(kBlock), 0, st, ws, a);
        else if (r == 1) hipLaunchKernelGGL(k_round_ro1<1>, dim3(g1), dim3(kBlock), 0, st, ws, a);
        else hipLaunchKernelGGL(k_round<1>, dim3(grid), dim3(kBlock), 0, st, ws, a, r);
        hipLaunchKernelGGL(k_round_multi<1>, dim3(grid_multi), dim3(kBlock), 0, st, ws, a, r);
    }
    if (a.fin_cap > 0 && r >= a.fin_from)
        hipLaunchKernelGGL(k_finish, dim3(std::max(1, grid_fin)), dim3(kBlock), 0, st, ws, a, r);
    return hipGetLastError();
}

hipError_t launch_segments(const Ws2 &ws, const HullArgs &a, int32_t r, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_segments, dim3(grid), dim3(kSegBlock), 0, st, ws, a, r);
    return hipGetLastError();
}

hipError_t launch_output(const Ws2 &ws, const HullArgs &a, int32_t H, hipStream_t st) {
    int steps = 0;
    while ((1ll << steps) < (int64_t)H + 1) ++steps;
    int src = 0;
    if (H > 0) {
        if (H <= kRankSmallCap) {
            hipLaunchKernelGGL(k_rank_small, dim3(1), dim3(kRankBlock), 0, st, ws, H, steps);
        } else {
            const int grid = (H + 255) / 256;
            hipLaunchKernelGGL(k_rank_init, dim3(grid), dim3(256), 0, st, ws, H);
            for (int it = 0; it < steps; ++it) {
                hipLaunchKernelGGL(k_rank_step, dim3(grid), dim3(256), 0, st, ws, H, src);
                src ^= 1;
            }
        }
    }
    hipLaunchKernelGGL(k_hull_offsets, dim3(1), dim3(kBlock), 0, st, ws, a, src);
    if (H > 0)
        hipLaunchKernelGGL(k_emit, dim3((H + 255) / 256), dim3(256), 0, st, ws, a, H, src);
    return hipGetLastError();
}

__global__ void k_fill_offsets(int64_t *off, int64_t n) {
    if (threadIdx.x == 0) { off[0] = 0; off[1] = n; }
}

hipError_t fill_single_offsets(int64_t *off, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_offsets, dim3(1), dim3(64), 0, st, off, n);
    return hipGetLastError();
}

hipError_t extremes_grid(int cus, int *grid) {
    int per = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void *>(&k_extremes),
                                                                kBlock, 0);
    if (e != hipSuccess) return e;
    *grid = std::max(1, per) * cus;
    return hipSuccess;
}

hipError_t round_grids(int mode, int cus, int (&grids)[3]) {
    const void *f[3] = {mode == 0 ? reinterpret_cast<const void *>(&k_split<0>)
                                  : reinterpret_cast<const void *>(&k_split<1>),
                        mode == 0 ? reinterpret_cast<const void *>(&k_round_ro1<0>)
                                  : reinterpret_cast<const void *>(&k_round_ro1<1>),
                        mode == 0 ? reinterpret_cast<const void *>(&k_round<0>)
                                  : reinterpret_cast<const void *>(&k_round<1>)};
    for (int j = 0; j < 3; ++j) {
        int pj = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&pj, f[j], kBlock, 0);
        if (e != hipSuccess) return e;
        grids[j] = std::max(1, pj) * cus;
    }
    return hipSuccess;
}

}  // namespace qh
