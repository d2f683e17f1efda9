// qh2d_kernels.hip -- the 2D segmented Quickhull round on gfx950.
//
// One round of the permute-and-segment Quickhull (Tzeng & Owens, Section 3.1,
// Algorithm 4's recursive step) is two launches:
//
//   k_round     one pass over the survivors: every point is tested against
//               the two new edges u->f and f->v of its segment (the triangle
//               test and the "which edge" state of Algorithm 4), points
//               inside the triangle are dropped (compact, Section 4.2), the
//               others are written to the two child segments (a 2-state
//               flagPermute, Section 4.1) with a single-pass decoupled
//               look-back scan, and the farthest point of every child
//               segment (the next apex) is found on the way;
//   k_segments  one thread per segment: inserts the apex into the hull,
//               finishes the argmax of segments that span several tiles and
//               writes the child segment table of the next round.
//
// Layout: survivors are structure-of-arrays int32 x[], y[], idx[] in two
// regions per round (state-0 children and state-1 children), each region
// filled front to back; a segment is a range [start, start+len) of one region.
// Tiles of 4096 points are claimed from an atomic counter, which makes the
// look-back safe without any assumption on the dispatch order.
#include "qh2d.h"

namespace qh {

// FP32 filter constant: |fl(a b - c d) - (a b - c d)| <= 4.0000004 eps
// (|fl(a b)| + |fl(c d)|) for a, b, c, d rounded from int32 (eps = 2^-24);
// 5 eps also covers the rounding of the bound itself.
constexpr float kErrC = 5.0f / 16777216.0f;

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

// largest i in [0, m) with s[i] <= v  (s[0] <= v, s nondecreasing)
__device__ __forceinline__ int slot_of(const int32_t *s, int m, int32_t v) {
    int a = 0, b = m;
    while (b - a > 1) {
        const int c = (a + b) >> 1;
        if (s[c] <= v) a = c; else b = c;
    }
    return a;
}

__device__ __forceinline__ void store_best(Best *dst, const Best &b) { *dst = b; }

__device__ __forceinline__ void best_merge(Best &acc, const Best &b) {
    if (best_better(b, acc)) acc = b;
}

// ---------------------------------------------------------------------------
// Set-up: compact the non-empty instances into the first segment table
// (one block).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_instances(Ws2 ws, const int64_t *offsets, int64_t n_total,
                                                    int32_t k) {
    Control *ctl = ws.ctl;
    __shared__ uint32_t scratch[32];
    __shared__ uint32_t carry;
    __shared__ int32_t bad;
    if (threadIdx.x == 0) { carry = 0; bad = 0; }
    __syncthreads();
    for (int base = 0; base < k; base += 1024) {
        const int i = base + (int)threadIdx.x;
        int64_t lo = 0, hi = 0;
        bool ne = false;
        if (i < k) {
            lo = offsets[i];
            hi = offsets[i + 1];
            if (lo < 0 || hi < lo || hi > n_total || (i == 0 && lo != 0) ||
                (i == k - 1 && hi != n_total))
                atomicOr(&bad, 1);
            ne = hi > lo;
        }
        uint32_t v[1] = {ne ? 1u : 0u}, tot[1];
        block_excl_scan<1024, 1>(v, tot, scratch);
        const uint32_t j = carry + v[0];
        if (i < k) {
            ws.inst_rank[i] = ne ? (int32_t)j : -1;
            ws.nxt[i] = -1;
            ws.nxt[k + i] = -1;
            if (ne) {
                SegGeo g;
                g.start = (int32_t)lo;
                g.len = (int32_t)(hi - lo);
                g.ux = g.uy = g.fx = g.fy = g.vx = g.vy = 0;
                ws.geo[0][0][j] = g;
                SegTop t;
                t.fidx = 0;
                t.uc = i;
                t.vc = i;
                t.inst = i;
                ws.top[0][0][j] = t;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) carry += tot[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        RoundState z = {};
        ctl->rs[1] = z;
        RoundState r0 = {};
        r0.n[0] = (int32_t)n_total;
        r0.n[1] = 0;
        r0.s[0] = (int32_t)carry;
        r0.s[1] = 0;
        r0.hbase = k;
        ctl->rs[0] = r0;
        ctl->error = bad ? kErrOffsets : 0;
        ctl->rounds_done = 0;
        ctl->max_segments = (int32_t)carry;
        ctl->points_in = ctl->points_out = ctl->first_in = 0;
        ctl->filter_tests = ctl->filter_fallbacks = ctl->candidates = 0;
        ctl->round_launches_work = 0;
    }
}

// Set-up: tile map of the original array (tile -> instance segment), and a
// clean look-back status for both parities.
__global__ void k_setup(Ws2 ws, const int64_t *offsets, int32_t k, int32_t ntiles) {
    const int stride = gridDim.x * blockDim.x;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int i = tid; i < ws.tcap + 4; i += stride) {
        ws.st2[0][i] = 0;
        ws.st2[1][i] = 0;
    }
    for (int i = tid; i < ws.s4cap; i += stride) {
        ws.st4[0][i] = 0;
        ws.st4[1][i] = 0;
    }
    if (ws.ctl->error) return;
    for (int t = tid; t < ntiles; t += stride) {
        const int64_t v = (int64_t)t * kTile;
        // largest i with offsets[i] <= v: that instance holds v and is non-empty
        int a = 0, b = k;
        while (b - a > 1) {
            const int c = (a + b) >> 1;
            if (offsets[c] <= v) a = c; else b = c;
        }
        ws.tmap[0][0][t] = ws.inst_rank[a];
    }
}

// ---------------------------------------------------------------------------
// K0: lexicographic extremes of every instance and the coordinate range check
// (first split of Algorithm 4: the extrema along x, ties by y then index).
// ---------------------------------------------------------------------------
template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_extremes(Ws2 ws, const int32_t *in_x, const int32_t *in_y,
                                                    int32_t n, int32_t vec_ok) {
    constexpr int T = BLOCK * ITEMS;
    constexpr int Q = ITEMS / 4;
    Control *ctl = ws.ctl;
    if (ctl->error) return;
    const int S = ctl->rs[0].s[0];
    const int ntiles = (n + T - 1) / T;
    const int tid = threadIdx.x;

    __shared__ int32_t sstart[T + 1];
    __shared__ uint64_t kmin1[kSlots], kmin2[kSlots], kmax1[kSlots], kmax2[kSlots];
    __shared__ int32_t rmin[kSlots][3], rmax[kSlots][3];
    __shared__ int32_t s_tile, s_m, s_bad;

    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int lo = tile * T;
        const int hi = min(lo + T, n);
        int32_t X[ITEMS], Y[ITEMS];
#pragma unroll
        for (int qq = 0; qq < Q; ++qq) {
            const int v0 = lo + qq * BLOCK * 4 + tid * 4;
            if (vec_ok && v0 + 3 < hi) {
                const int4 a = *reinterpret_cast<const int4 *>(in_x + v0);
                const int4 b = *reinterpret_cast<const int4 *>(in_y + v0);
                X[qq * 4 + 0] = a.x; X[qq * 4 + 1] = a.y; X[qq * 4 + 2] = a.z; X[qq * 4 + 3] = a.w;
                Y[qq * 4 + 0] = b.x; Y[qq * 4 + 1] = b.y; Y[qq * 4 + 2] = b.z; Y[qq * 4 + 3] = b.w;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int v = v0 + j;
                    X[qq * 4 + j] = v < hi ? in_x[v] : 0;
                    Y[qq * 4 + j] = v < hi ? in_y[v] : 0;
                }
            }
        }
        // instances overlapping the tile
        const int s0 = ws.tmap[0][0][tile];
        if (tid == 0) { s_m = 0; s_bad = 0; }
        __syncthreads();
        for (int b = 0; b <= T; b += BLOCK) {
            const int j = b + tid;
            bool in = false;
            if (j <= T) {
                const int si = s0 + j;
                const int st = si < S ? ws.geo[0][0][si].start : n;
                sstart[j] = st;
                in = st < hi;
            }
            const int cnt = __syncthreads_count(in);
            if (tid == 0) s_m += cnt;
            if (cnt < BLOCK) break;
        }
        __syncthreads();
        const int m = s_m;
        // range check
        bool bad = false;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int v = lo + (i >> 2) * BLOCK * 4 + tid * 4 + (i & 3);
            if (v < hi) {
                bad |= (X[i] > kCoordMax2D) | (X[i] < -kCoordMax2D) | (Y[i] > kCoordMax2D) |
                       (Y[i] < -kCoordMax2D);
            }
        }
        if (__syncthreads_or(bad) && tid == 0) atomicOr(&ctl->error, kErrRange);

        for (int w0 = 0; w0 < m; w0 += kSlots) {
            const int wn = min(kSlots, m - w0);
            for (int j = tid; j < kSlots; j += BLOCK) {
                kmin1[j] = 0; kmin2[j] = ~0ull; kmax1[j] = 0; kmax2[j] = ~0ull;
            }
            __syncthreads();
            // phase 1: best coordinate key per slot (min as max of complement)
            int cur = -1;
            uint64_t bmin = 0, bmax = 0;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int v = lo + (i >> 2) * BLOCK * 4 + tid * 4 + (i & 3);
                if (v >= hi) continue;
                const int sl = (m == 1) ? 0 : slot_of(sstart, m, v);
                if (sl < w0 || sl >= w0 + wn) continue;
                if (sl != cur) {
                    if (cur >= 0) {
                        atomicMax(&kmin1[cur - w0], bmin);
                        atomicMax(&kmax1[cur - w0], bmax);
                    }
                    cur = sl;
                    bmin = 0;
                    bmax = 0;
                }
                const uint64_t ck = coord_key(X[i], Y[i]);
                bmin = max(bmin, ~ck);
                bmax = max(bmax, ck);
            }
            if (cur >= 0) {
                atomicMax(&kmin1[cur - w0], bmin);
                atomicMax(&kmax1[cur - w0], bmax);
            }
            __syncthreads();
            // phase 2: lowest index among the points with that key
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int v = lo + (i >> 2) * BLOCK * 4 + tid * 4 + (i & 3);
                if (v >= hi) continue;
                const int sl = (m == 1) ? 0 : slot_of(sstart, m, v);
                if (sl < w0 || sl >= w0 + wn) continue;
                const uint64_t ck = coord_key(X[i], Y[i]);
                if (~ck == kmin1[sl - w0]) atomicMin(&kmin2[sl - w0], (uint64_t)(uint32_t)v);
                if (ck == kmax1[sl - w0]) atomicMin(&kmax2[sl - w0], (uint64_t)(uint32_t)v);
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int v = lo + (i >> 2) * BLOCK * 4 + tid * 4 + (i & 3);
                if (v >= hi) continue;
                const int sl = (m == 1) ? 0 : slot_of(sstart, m, v);
                if (sl < w0 || sl >= w0 + wn) continue;
                if ((uint64_t)(uint32_t)v == kmin2[sl - w0]) {
                    rmin[sl - w0][0] = X[i]; rmin[sl - w0][1] = Y[i]; rmin[sl - w0][2] = v;
                }
                if ((uint64_t)(uint32_t)v == kmax2[sl - w0]) {
                    rmax[sl - w0][0] = X[i]; rmax[sl - w0][1] = Y[i]; rmax[sl - w0][2] = v;
                }
            }
            __syncthreads();
            for (int j = tid; j < wn; j += BLOCK) {
                const int sl = w0 + j;
                Best bmn, bmx;
                bmn.key1 = kmin1[j]; bmn.key2 = kmin2[j];
                bmn.x = rmin[j][0]; bmn.y = rmin[j][1]; bmn.idx = rmin[j][2]; bmn.pad = 0;
                bmx.key1 = kmax1[j]; bmx.key2 = kmax2[j];
                bmx.x = rmax[j][0]; bmx.y = rmax[j][1]; bmx.idx = rmax[j][2]; bmx.pad = 0;
                const bool inside = sstart[sl] >= lo && sstart[sl + 1] <= hi;
                if (inside) {
                    ws.dir0[(s0 + sl) * 2 + 0] = bmn;
                    ws.dir0[(s0 + sl) * 2 + 1] = bmx;
                }
                if (sl == 0) {
                    ws.recF0[tile * 2 + 0] = bmn;
                    ws.recF0[tile * 2 + 1] = bmx;
                }
                if (sl == m - 1) {
                    ws.recL0[tile * 2 + 0] = bmn;
                    ws.recL0[tile * 2 + 1] = bmx;
                }
            }
            __syncthreads();
        }
    }
}

// K0f: one block per instance segment: finish the extremes over the tiles it
// spans and write the first-split segment (edge a -> a with apex b, so the
// round kernel splits the points by the line ab).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_extremes_final(Ws2 ws) {
    Control *ctl = ws.ctl;
    if (ctl->error) return;
    const int S = ctl->rs[0].s[0];
    const int s = blockIdx.x;
    if (s >= S) return;
    __shared__ Best red[2][BLOCK];
    SegGeo g = ws.geo[0][0][s];
    const SegTop tp = ws.top[0][0][s];
    const int t0 = g.start / kTile;
    const int t1 = (g.start + g.len - 1) / kTile;
    Best b[2];
    if (t0 == t1) {
        b[0] = ws.dir0[s * 2 + 0];
        b[1] = ws.dir0[s * 2 + 1];
    } else {
        for (int c = 0; c < 2; ++c) {
            Best acc;
            acc.key1 = 0; acc.key2 = ~0ull; acc.x = acc.y = acc.idx = acc.pad = 0;
            for (int t = t0 + (int)threadIdx.x; t <= t1; t += BLOCK)
                best_merge(acc, t == t0 ? ws.recL0[t * 2 + c] : ws.recF0[t * 2 + c]);
            red[c][threadIdx.x] = acc;
        }
        __syncthreads();
        for (int w = BLOCK / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                for (int c = 0; c < 2; ++c) {
                    Best o = red[c][threadIdx.x + w];
                    if (best_better(o, red[c][threadIdx.x])) red[c][threadIdx.x] = o;
                }
            }
            __syncthreads();
        }
        b[0] = red[0][0];
        b[1] = red[1][0];
    }
    if (threadIdx.x != 0) return;
    g.ux = b[0].x; g.uy = b[0].y;
    g.vx = b[0].x; g.vy = b[0].y;
    g.fx = b[1].x; g.fy = b[1].y;
    ws.geo[0][0][s] = g;
    SegTop t = tp;
    t.fidx = b[1].idx;
    ws.top[0][0][s] = t;
    ws.V[tp.uc] = b[0].idx;
    ws.hinst[tp.uc] = tp.inst;
}

// ---------------------------------------------------------------------------
// The fused round kernel.
// ---------------------------------------------------------------------------
template <bool INIT, int MODE, int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_round(Ws2 ws, int32_t r, const int32_t *in_x,
                                                 const int32_t *in_y, int32_t vec_ok) {
    constexpr int T = BLOCK * ITEMS;
    constexpr int Q = ITEMS / 4;
    constexpr int NW = BLOCK / kWave;
    static_assert(T == kTile, "tile size");
    Control *ctl = ws.ctl;
    if (ctl->error) return;
    const int p = r & 1, q = p ^ 1;
    RoundState *rs = &ctl->rs[p];
    RoundState *rn = &ctl->rs[q];
    const int n0 = rs->n[0], n1 = rs->n[1];
    const int S0 = rs->s[0];
    const int S1 = rs->s[1];
    const int nt0 = (n0 + T - 1) / T, nt1 = (n1 + T - 1) / T;
    const int ntiles = nt0 + nt1;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wv = tid / kWave;

    // house-keeping for the next round
    if (blockIdx.x == 0 && tid == 0) rn->tile_ctr = 0;
    for (int i = blockIdx.x * BLOCK + tid; i < ntiles + 2 && i < ws.tcap + 4; i += gridDim.x * BLOCK)
        ws.st2[q][i] = 0;
    if (ntiles == 0) {
        if (blockIdx.x == 0 && tid == 0) { rn->n[0] = 0; rn->n[1] = 0; }
        return;
    }

    __shared__ int32_t sstart[T + 1];
    __shared__ int32_t lgeo[kSlots][6];
    __shared__ uint64_t k1[2][kSlots];
    __shared__ uint64_t k2[2][kSlots];
    __shared__ uint32_t lm[2][kSlots];
    __shared__ int32_t res[2][kSlots][3];
    __shared__ uint32_t scan_scr[Q * NW];
    __shared__ int32_t s_tile, s_m;
    __shared__ uint64_t s_ex;

    while (true) {
        if (tid == 0) s_tile = (int32_t)atomicAdd(&rs->tile_ctr, 1u);
        __syncthreads();
        const int tile = s_tile;
        if (tile >= ntiles) break;
        const int R = tile < nt0 ? 0 : 1;
        const int lt = tile - (R ? nt0 : 0);
        const int NR = R ? n1 : n0;
        const int SR = R ? S1 : S0;
        const int gbase = R ? S0 : 0;
        const int lo = lt * T;
        const int hi = min(lo + T, NR);
        const SegGeo *geo = ws.geo[p][R];

        // 1. the tile's points (structure of arrays, 16-byte loads)
        int32_t X[ITEMS], Y[ITEMS], I[ITEMS];
#pragma unroll
        for (int qq = 0; qq < Q; ++qq) {
            const int v0 = lo + qq * BLOCK * 4 + tid * 4;
            if (INIT) {
                if (vec_ok && v0 + 3 < hi) {
                    const int4 a = *reinterpret_cast<const int4 *>(in_x + v0);
                    const int4 b = *reinterpret_cast<const int4 *>(in_y + v0);
                    X[qq * 4 + 0] = a.x; X[qq * 4 + 1] = a.y; X[qq * 4 + 2] = a.z; X[qq * 4 + 3] = a.w;
                    Y[qq * 4 + 0] = b.x; Y[qq * 4 + 1] = b.y; Y[qq * 4 + 2] = b.z; Y[qq * 4 + 3] = b.w;
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int v = v0 + j;
                        X[qq * 4 + j] = v < hi ? in_x[v] : 0;
                        Y[qq * 4 + j] = v < hi ? in_y[v] : 0;
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) I[qq * 4 + j] = v0 + j;
            } else {
                const int4 a = *reinterpret_cast<const int4 *>(ws.px[p][R] + v0);
                const int4 b = *reinterpret_cast<const int4 *>(ws.py[p][R] + v0);
                const int4 c = *reinterpret_cast<const int4 *>(ws.pi[p][R] + v0);
                X[qq * 4 + 0] = a.x; X[qq * 4 + 1] = a.y; X[qq * 4 + 2] = a.z; X[qq * 4 + 3] = a.w;
                Y[qq * 4 + 0] = b.x; Y[qq * 4 + 1] = b.y; Y[qq * 4 + 2] = b.z; Y[qq * 4 + 3] = b.w;
                I[qq * 4 + 0] = c.x; I[qq * 4 + 1] = c.y; I[qq * 4 + 2] = c.z; I[qq * 4 + 3] = c.w;
            }
        }

        // 2. the segments overlapping the tile: starts into LDS
        const int s0 = ws.tmap[p][R][lt];
        if (tid == 0) s_m = 0;
        __syncthreads();
        for (int b = 0; b <= T; b += BLOCK) {
            const int j = b + tid;
            bool in = false;
            if (j <= T) {
                const int si = s0 + j;
                const int st = si < SR ? geo[si].start : NR;
                sstart[j] = st;
                in = st < hi;
            }
            const int cnt = __syncthreads_count(in);
            if (tid == 0) s_m += cnt;
            if (cnt < BLOCK) break;
        }
        __syncthreads();
        const int m = s_m;

        // slot of every point (16 bits each)
        uint32_t slotpk[ITEMS / 2];
#pragma unroll
        for (int i = 0; i < ITEMS; i += 2) {
            const int va = lo + (i >> 2) * BLOCK * 4 + tid * 4 + (i & 3);
            const int sa = (m == 1 || va >= hi) ? 0 : slot_of(sstart, m, va);
            const int sb = (m == 1 || va + 1 >= hi) ? 0 : slot_of(sstart, m, va + 1);
            slotpk[i >> 1] = (uint32_t)sa | ((uint32_t)sb << 16);
        }
        auto SLOT = [&](int i) -> int { return (int)((slotpk[i >> 1] >> ((i & 1) * 16)) & 0xffffu); };
        auto VOF = [&](int i) -> int { return lo + (i >> 2) * BLOCK * 4 + tid * 4 + (i & 3); };

        uint32_t stbits = 0;        // 2 bits per point: 0, 1 = child, 2 = dropped
        uint64_t D[ITEMS];          // exact distance to the child edge (argmax key)
        float U[ITEMS];             // FP32 filter: upper bound of that distance
        uint32_t ntests = 0, nfall = 0, ncand = 0;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) { D[i] = 0; U[i] = 0.f; }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) stbits |= 2u << (2 * i);

        for (int w0 = 0; w0 < m; w0 += kSlots) {
            const int wn = min(kSlots, m - w0);
            for (int j = tid; j < wn; j += BLOCK) {
                const SegGeo g = geo[s0 + w0 + j];
                lgeo[j][0] = g.ux; lgeo[j][1] = g.uy;
                lgeo[j][2] = g.fx; lgeo[j][3] = g.fy;
                lgeo[j][4] = g.vx; lgeo[j][5] = g.vy;
            }
            for (int j = tid; j < 2 * kSlots; j += BLOCK) {
                (&k1[0][0])[j] = 0;
                (&k2[0][0])[j] = ~0ull;
                (&lm[0][0])[j] = 0;
            }
            __syncthreads();

            // 3. classify against u->f and f->v; running max per (slot, child)
            int cur = -1;
            uint64_t rb0 = 0, rb1 = 0;     // exact: max distance
            uint32_t rl0 = 0, rl1 = 0;     // filter: max lower bound (ordered key)
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int v = VOF(i);
                const int sl = SLOT(i);
                if (v >= hi || sl < w0 || sl >= w0 + wn) continue;
                const int ls = sl - w0;
                const int ux = lgeo[ls][0], uy = lgeo[ls][1];
                const int fx = lgeo[ls][2], fy = lgeo[ls][3];
                const int vx = lgeo[ls][4], vy = lgeo[ls][5];
                uint32_t st = 2;
                if (MODE == 0) {
                    const int64_t d0 = cross_i64(X[i], Y[i], ux, uy, fx, fy);
                    if (d0 > 0) {
                        st = 0;
                        D[i] = (uint64_t)d0;
                    } else {
                        const int64_t d1 = cross_i64(X[i], Y[i], fx, fy, vx, vy);
                        if (d1 > 0) {
                            st = 1;
                            D[i] = (uint64_t)d1;
                        }
                    }
                } else {
                    float B0, B1;
                    const float e0 = cross_f32(X[i], Y[i], ux, uy, fx, fy, B0);
                    ntests++;
                    bool out0;
                    if (e0 > B0) out0 = true;
                    else if (e0 < -B0) out0 = false;
                    else { nfall++; out0 = cross_i64(X[i], Y[i], ux, uy, fx, fy) > 0; }
                    if (out0) {
                        st = 0;
                        U[i] = __fadd_rn(e0, 2.f * B0);
                        const float L = __fsub_rn(e0, 2.f * B0);
                        if (sl != cur) {
                            if (cur >= 0) {
                                if (rl0) atomicMax(&lm[0][cur - w0], rl0);
                                if (rl1) atomicMax(&lm[1][cur - w0], rl1);
                            }
                            cur = sl; rl0 = 0; rl1 = 0;
                        }
                        rl0 = max(rl0, fkey(L));
                    } else {
                        const float e1 = cross_f32(X[i], Y[i], fx, fy, vx, vy, B1);
                        ntests++;
                        bool out1;
                        if (e1 > B1) out1 = true;
                        else if (e1 < -B1) out1 = false;
                        else { nfall++; out1 = cross_i64(X[i], Y[i], fx, fy, vx, vy) > 0; }
                        if (out1) {
                            st = 1;
                            U[i] = __fadd_rn(e1, 2.f * B1);
                            const float L = __fsub_rn(e1, 2.f * B1);
                            if (sl != cur) {
                                if (cur >= 0) {
                                    if (rl0) atomicMax(&lm[0][cur - w0], rl0);
                                    if (rl1) atomicMax(&lm[1][cur - w0], rl1);
                                }
                                cur = sl; rl0 = 0; rl1 = 0;
                            }
                            rl1 = max(rl1, fkey(L));
                        }
                    }
                }
                stbits = (stbits & ~(3u << (2 * i))) | (st << (2 * i));
                if (MODE == 0 && st < 2) {
                    if (sl != cur) {
                        if (cur >= 0) {
                            if (rb0) atomicMax(&k1[0][cur - w0], rb0);
                            if (rb1) atomicMax(&k1[1][cur - w0], rb1);
                        }
                        cur = sl; rb0 = 0; rb1 = 0;
                    }
                    if (st == 0) rb0 = max(rb0, D[i]); else rb1 = max(rb1, D[i]);
                }
            }
            if (cur >= 0) {
                if (MODE == 0) {
                    if (rb0) atomicMax(&k1[0][cur - w0], rb0);
                    if (rb1) atomicMax(&k1[1][cur - w0], rb1);
                } else {
                    if (rl0) atomicMax(&lm[0][cur - w0], rl0);
                    if (rl1) atomicMax(&lm[1][cur - w0], rl1);
                }
            }
            __syncthreads();

            if (MODE != 0) {
                // 3b. filter: points whose upper bound reaches the best lower
                // bound are the only possible argmax; they get exact keys
                cur = -1;
                uint64_t cb0 = 0, cb1 = 0;
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const int v = VOF(i);
                    const int sl = SLOT(i);
                    const uint32_t st = (stbits >> (2 * i)) & 3u;
                    if (v >= hi || st > 1 || sl < w0 || sl >= w0 + wn) continue;
                    const int ls = sl - w0;
                    if (fkey(U[i]) < lm[st][ls]) continue;
                    ncand++;
                    int64_t d;
                    if (st == 0) d = cross_i64(X[i], Y[i], lgeo[ls][0], lgeo[ls][1], lgeo[ls][2], lgeo[ls][3]);
                    else d = cross_i64(X[i], Y[i], lgeo[ls][2], lgeo[ls][3], lgeo[ls][4], lgeo[ls][5]);
                    D[i] = (uint64_t)d;
                    if (sl != cur) {
                        if (cur >= 0) {
                            if (cb0) atomicMax(&k1[0][cur - w0], cb0);
                            if (cb1) atomicMax(&k1[1][cur - w0], cb1);
                        }
                        cur = sl; cb0 = 0; cb1 = 0;
                    }
                    if (st == 0) cb0 = max(cb0, D[i]); else cb1 = max(cb1, D[i]);
                }
                if (cur >= 0) {
                    if (cb0) atomicMax(&k1[0][cur - w0], cb0);
                    if (cb1) atomicMax(&k1[1][cur - w0], cb1);
                }
                __syncthreads();
            }

            // 4. tie-break among the farthest points, then the winner
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int v = VOF(i);
                const int sl = SLOT(i);
                const uint32_t st = (stbits >> (2 * i)) & 3u;
                if (v >= hi || st > 1 || sl < w0 || sl >= w0 + wn) continue;
                const int ls = sl - w0;
                if (D[i] != k1[st][ls]) continue;
                const int ex = st == 0 ? lgeo[ls][2] - lgeo[ls][0] : lgeo[ls][4] - lgeo[ls][2];
                const int ey = st == 0 ? lgeo[ls][3] - lgeo[ls][1] : lgeo[ls][5] - lgeo[ls][3];
                atomicMin(&k2[st][ls], tie_key(X[i], Y[i], I[i], ex, ey));
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const int v = VOF(i);
                const int sl = SLOT(i);
                const uint32_t st = (stbits >> (2 * i)) & 3u;
                if (v >= hi || st > 1 || sl < w0 || sl >= w0 + wn) continue;
                const int ls = sl - w0;
                if (D[i] != k1[st][ls]) continue;
                const int ex = st == 0 ? lgeo[ls][2] - lgeo[ls][0] : lgeo[ls][4] - lgeo[ls][2];
                const int ey = st == 0 ? lgeo[ls][3] - lgeo[ls][1] : lgeo[ls][5] - lgeo[ls][3];
                if (tie_key(X[i], Y[i], I[i], ex, ey) == k2[st][ls]) {
                    res[st][ls][0] = X[i]; res[st][ls][1] = Y[i]; res[st][ls][2] = I[i];
                }
            }
            __syncthreads();

            // 5. per-slot results: whole segments directly, the first and the
            // last segment of the tile as partial records
            for (int j = tid; j < wn; j += BLOCK) {
                const int sl = w0 + j;
                const int g = gbase + s0 + sl;
                const bool inside = sstart[sl] >= lo && sstart[sl + 1] <= hi;
                for (int c = 0; c < 2; ++c) {
                    Best b;
                    b.key1 = k1[c][j];
                    b.key2 = k2[c][j];
                    b.x = b.key1 ? res[c][j][0] : 0;
                    b.y = b.key1 ? res[c][j][1] : 0;
                    b.idx = b.key1 ? res[c][j][2] : 0;
                    b.pad = 0;
                    if (inside) ws.adir[g * 2 + c] = b;
                    if (sl == 0) ws.recF[tile * 2 + c] = b;
                    if (sl == m - 1) ws.recL[tile * 2 + c] = b;
                }
            }
            __syncthreads();
        }

        // 6. ranks of the survivors inside the tile (point order), per child
        uint32_t cnt[Q], tot[Q];
#pragma unroll
        for (int qq = 0; qq < Q; ++qq) {
            uint32_t c = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t st = (stbits >> (2 * (qq * 4 + j))) & 3u;
                c += st == 0 ? 1u : (st == 1 ? 0x10000u : 0u);
            }
            cnt[qq] = c;
        }
        block_excl_scan<BLOCK, Q>(cnt, tot, scan_scr);
        uint32_t rowbase[Q];
        uint32_t acc = 0;
#pragma unroll
        for (int qq = 0; qq < Q; ++qq) { rowbase[qq] = acc; acc += tot[qq]; }
        const uint32_t c0 = acc & 0xffffu, c1 = acc >> 16;

        // 7. decoupled look-back: global offsets of this tile's survivors
        if (wv == 0) {
            const uint64_t ex = lookback_excl(ws.st2[p], tile, pack2(c0, c1), &ctl->error);
            if (lane == 0) s_ex = ex;
        }
        __syncthreads();
        const uint32_t E0 = unpackA(s_ex), E1 = unpackB(s_ex);

        // 8. scatter the survivors into the two child regions; segment
        // boundaries record their global offsets
        int32_t *ox0 = ws.px[q][0], *oy0 = ws.py[q][0], *oi0 = ws.pi[q][0];
        int32_t *ox1 = ws.px[q][1], *oy1 = ws.py[q][1], *oi1 = ws.pi[q][1];
#pragma unroll
        for (int qq = 0; qq < Q; ++qq) {
            uint32_t run = rowbase[qq] + cnt[qq];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = qq * 4 + j;
                const int v = VOF(i);
                const uint32_t st = (stbits >> (2 * i)) & 3u;
                const uint32_t e0 = E0 + (run & 0xffffu);
                const uint32_t e1 = E1 + (run >> 16);
                if (v < hi) {
                    const int sl = SLOT(i);
                    const int g = gbase + s0 + sl;
                    if (v == sstart[sl]) ws.pst[g] = make_int2((int)e0, (int)e1);
                    if (st == 0) {
                        if (e0 < (uint32_t)ws.cap_pts) {
                            ox0[e0] = X[i]; oy0[e0] = Y[i]; oi0[e0] = I[i];
                        } else {
                            atomicOr(&ctl->error, kErrInternal);
                        }
                    } else if (st == 1) {
                        if (e1 < (uint32_t)ws.cap_pts) {
                            ox1[e1] = X[i]; oy1[e1] = Y[i]; oi1[e1] = I[i];
                        } else {
                            atomicOr(&ctl->error, kErrInternal);
                        }
                    }
                    const uint32_t run2 = run + (st == 0 ? 1u : (st == 1 ? 0x10000u : 0u));
                    if (v == sstart[sl + 1] - 1)
                        ws.pen[g] = make_int2((int)(E0 + (run2 & 0xffffu)), (int)(E1 + (run2 >> 16)));
                    run = run2;
                }
            }
        }
        if (MODE != 0) {
            const uint32_t a = wave_sum(ntests), b = wave_sum(nfall), c = wave_sum(ncand);
            if (lane == 0) {
                atomicAdd(&ctl->filter_tests, (unsigned long long)a);
                atomicAdd(&ctl->filter_fallbacks, (unsigned long long)b);
                atomicAdd(&ctl->candidates, (unsigned long long)c);
            }
            ntests = nfall = ncand = 0;
        }
        if (tile == ntiles - 1 && tid == 0) {
            rn->n[0] = (int32_t)(E0 + c0);
            rn->n[1] = (int32_t)(E1 + c1);
            atomicAdd(&ctl->points_in, (unsigned long long)(n0 + n1));
            atomicAdd(&ctl->points_out, (unsigned long long)(E0 + c0 + E1 + c1));
            if (INIT) atomicAdd(&ctl->first_in, (unsigned long long)(n0 + n1));
            atomicAdd(&ctl->round_launches_work, 1ull);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// The segment kernel: hull insertion, argmax finish, next segment table.
// ---------------------------------------------------------------------------
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_segments(Ws2 ws, int32_t r) {
    constexpr int NW = BLOCK / kWave;
    Control *ctl = ws.ctl;
    if (ctl->error) return;
    const int p = r & 1, q = p ^ 1;
    RoundState *rs = &ctl->rs[p];
    RoundState *rn = &ctl->rs[q];
    const int S0 = rs->s[0], S1 = rs->s[1];
    const int Stot = S0 + S1;
    const int hbase = rs->hbase;
    const int nt0 = (rs->n[0] + kTile - 1) / kTile;
    const int nsegt = (Stot + BLOCK - 1) / BLOCK;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wv = tid / kWave;

    if (blockIdx.x == 0 && tid == 0) rn->seg_ctr = 0;
    for (int i = blockIdx.x * BLOCK + tid; i < 2 * nsegt + 4 && i < ws.s4cap; i += gridDim.x * BLOCK)
        ws.st4[q][i] = 0;
    if (Stot == 0) {
        if (blockIdx.x == 0 && tid == 0) {
            rn->s[0] = 0; rn->s[1] = 0; rn->hbase = hbase;
        }
        return;
    }

    __shared__ uint32_t scan_scr[2 * NW];
    __shared__ int32_t s_tile;
    __shared__ uint64_t s_ex;
    __shared__ int32_t qn_apex, qn_map;
    __shared__ int16_t q_apex[BLOCK], q_map[2 * BLOCK];
    __shared__ int32_t o_t0[BLOCK], o_t1[BLOCK];
    __shared__ int32_t o_mst[2 * BLOCK], o_mlen[2 * BLOCK], o_mid[2 * BLOCK];
    __shared__ Best red[2][BLOCK];
    __shared__ Best o_best[2][BLOCK];

    while (true) {
        if (tid == 0) {
            s_tile = (int32_t)atomicAdd(&rs->seg_ctr, 1u);
            qn_apex = 0;
            qn_map = 0;
        }
        __syncthreads();
        const int tile = s_tile;
        if (tile >= nsegt) break;
        const int g = tile * BLOCK + tid;
        const bool valid = g < Stot;
        const int R = g < S0 ? 0 : 1;
        const int s = g - (R ? S0 : 0);
        SegGeo G = {};
        SegTop Tp = {};
        int2 ps = make_int2(0, 0), pe = make_int2(0, 0);
        int c0 = 0, c1 = 0;
        int fc = 0;
        if (valid) {
            G = ws.geo[p][R][s];
            Tp = ws.top[p][R][s];
            ps = ws.pst[g];
            pe = ws.pen[g];
            c0 = pe.x - ps.x;
            c1 = pe.y - ps.y;
            // the apex f of this segment joins the hull between u and v
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
        const bool has0 = valid && c0 > 0, has1 = valid && c1 > 0;
        uint32_t v[2] = {has0 ? 1u : 0u, has1 ? 1u : 0u}, tot[2];
        block_excl_scan<BLOCK, 2>(v, tot, scan_scr);
        if (wv == 0) {
            const uint64_t ex = lookback_excl(ws.st4[p], tile, pack2(tot[0], tot[1]), &ctl->error);
            if (lane == 0) s_ex = ex;
        }
        __syncthreads();
        const int id0 = (int)(unpackA(s_ex) + v[0]);
        const int id1 = (int)(unpackB(s_ex) + v[1]);
        if ((has0 && id0 >= ws.scap) || (has1 && id1 >= ws.scap)) atomicOr(&ctl->error, kErrSegCap);

        // apexes of the two children
        Best b0, b1;
        b0.key1 = 0; b0.key2 = ~0ull; b0.x = b0.y = b0.idx = b0.pad = 0;
        b1 = b0;
        const int t0 = (R ? nt0 : 0) + G.start / kTile;
        const int t1 = (R ? nt0 : 0) + (G.start + G.len - 1) / kTile;
        if (valid && (has0 || has1)) {
            if (t0 == t1) {
                b0 = ws.adir[g * 2 + 0];
                b1 = ws.adir[g * 2 + 1];
            } else if (t1 - t0 <= 8) {
                b0 = ws.recL[t0 * 2 + 0];
                b1 = ws.recL[t0 * 2 + 1];
                for (int t = t0 + 1; t <= t1; ++t) {
                    best_merge(b0, ws.recF[t * 2 + 0]);
                    best_merge(b1, ws.recF[t * 2 + 1]);
                }
            } else {
                const int qi = atomicAdd(&qn_apex, 1);
                q_apex[qi] = (int16_t)tid;
                o_t0[tid] = t0;
                o_t1[tid] = t1;
            }
        }
        __syncthreads();
        const int nqa = qn_apex;
        for (int qi = 0; qi < nqa; ++qi) {
            const int own = q_apex[qi];
            const int a0 = o_t0[own], a1 = o_t1[own];
            for (int c = 0; c < 2; ++c) {
                Best acc;
                acc.key1 = 0; acc.key2 = ~0ull; acc.x = acc.y = acc.idx = acc.pad = 0;
                for (int t = a0 + tid; t <= a1; t += BLOCK)
                    best_merge(acc, t == a0 ? ws.recL[t * 2 + c] : ws.recF[t * 2 + c]);
                red[c][tid] = acc;
            }
            __syncthreads();
            for (int w = BLOCK / 2; w > 0; w >>= 1) {
                if (tid < w) {
                    for (int c = 0; c < 2; ++c) {
                        const Best o = red[c][tid + w];
                        if (best_better(o, red[c][tid])) red[c][tid] = o;
                    }
                }
                __syncthreads();
            }
            if (tid == 0) {
                o_best[0][own] = red[0][0];
                o_best[1][own] = red[1][0];
            }
            __syncthreads();
        }
        if (valid && (has0 || has1) && t1 - t0 > 8) {
            b0 = o_best[0][tid];
            b1 = o_best[1][tid];
        }

        // child segments of the next round
        if (has0 && id0 < ws.scap) {
            SegGeo cg;
            cg.start = ps.x; cg.len = c0;
            cg.ux = G.ux; cg.uy = G.uy;
            cg.fx = b0.x; cg.fy = b0.y;
            cg.vx = G.fx; cg.vy = G.fy;
            ws.geo[q][0][id0] = cg;
            SegTop ct;
            ct.fidx = b0.idx; ct.uc = Tp.uc; ct.vc = fc; ct.inst = Tp.inst;
            ws.top[q][0][id0] = ct;
        }
        if (has1 && id1 < ws.scap) {
            SegGeo cg;
            cg.start = ps.y; cg.len = c1;
            cg.ux = G.fx; cg.uy = G.fy;
            cg.fx = b1.x; cg.fy = b1.y;
            cg.vx = G.vx; cg.vy = G.vy;
            ws.geo[q][1][id1] = cg;
            SegTop ct;
            ct.fidx = b1.idx; ct.uc = fc; ct.vc = Tp.vc; ct.inst = Tp.inst;
            ws.top[q][1][id1] = ct;
        }
        // tile maps of the next round: tiles whose first point lies in a child
        for (int c = 0; c < 2; ++c) {
            const bool h = c == 0 ? has0 : has1;
            const int id = c == 0 ? id0 : id1;
            if (!h || id >= ws.scap) continue;
            const int st = c == 0 ? ps.x : ps.y;
            const int ln = c == 0 ? c0 : c1;
            const int ka = (st + kTile - 1) / kTile;
            const int kb = (st + ln + kTile - 1) / kTile;
            if (kb - ka <= 8) {
                for (int kk = ka; kk < kb; ++kk) ws.tmap[q][c][kk] = id;
            } else {
                const int qi = atomicAdd(&qn_map, 1);
                q_map[qi] = (int16_t)(tid * 2 + c);
                o_mst[tid * 2 + c] = ka;
                o_mlen[tid * 2 + c] = kb;
                o_mid[tid * 2 + c] = id;
            }
        }
        __syncthreads();
        const int nqm = qn_map;
        for (int qi = 0; qi < nqm; ++qi) {
            const int o = q_map[qi];
            const int c = o & 1;
            const int ka = o_mst[o], kb = o_mlen[o], id = o_mid[o];
            for (int kk = ka + tid; kk < kb; kk += BLOCK) ws.tmap[q][c][kk] = id;
        }
        if (tile == nsegt - 1 && tid == 0) {
            const int n0n = (int)(unpackA(s_ex) + tot[0]);
            const int n1n = (int)(unpackB(s_ex) + tot[1]);
            rn->s[0] = n0n;
            rn->s[1] = n1n;
            rn->hbase = hbase + Stot;
            if (hbase + Stot > ws.hcap) atomicOr(&ctl->error, kErrHullCap);
            atomicMax(&ctl->max_segments, n0n + n1n);
            atomicAdd(&ctl->rounds_done, 1);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Output: rank the hull cycles (pointer jumping) and write CCW index lists.
// ---------------------------------------------------------------------------
__global__ void k_rank_init(Ws2 ws, int32_t H) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= H) return;
    const int nx = ws.nxt[x];
    if (nx < 0) { ws.succ[0][x] = x; ws.dist[0][x] = 0; return; }
    const bool term = (nx == ws.hinst[x]);   // next is the instance's first vertex
    ws.succ[0][x] = term ? x : nx;
    ws.dist[0][x] = term ? 0 : 1;
}

__global__ void k_rank_step(Ws2 ws, int32_t H, int32_t src) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= H) return;
    const int s = ws.succ[src][x];
    ws.dist[src ^ 1][x] = ws.dist[src][x] + ws.dist[src][s];
    ws.succ[src ^ 1][x] = ws.succ[src][s];
}

// small hulls: all pointer jumping in LDS by one block
template <int BLOCK, int CAP>
__global__ __launch_bounds__(BLOCK) void k_rank_small(Ws2 ws, int32_t H, int32_t steps) {
    __shared__ int32_t su[CAP], di[CAP];
    for (int x = threadIdx.x; x < H; x += BLOCK) {
        const int nx = ws.nxt[x];
        if (nx < 0) { su[x] = x; di[x] = 0; continue; }
        const bool term = (nx == ws.hinst[x]);
        su[x] = term ? x : nx;
        di[x] = term ? 0 : 1;
    }
    __syncthreads();
    constexpr int PER = CAP / BLOCK;
    for (int it = 0; it < steps; ++it) {
        int ns[PER], nd[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int x = threadIdx.x + j * BLOCK;
            if (x < H) {
                const int s = su[x];
                nd[j] = di[x] + di[s];
                ns[j] = su[s];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int x = threadIdx.x + j * BLOCK;
            if (x < H) { su[x] = ns[j]; di[x] = nd[j]; }
        }
        __syncthreads();
    }
    for (int x = threadIdx.x; x < H; x += BLOCK) ws.dist[0][x] = di[x];
}

// hull sizes per instance and their exclusive scan (one block)
__global__ __launch_bounds__(1024) void k_hull_offsets(Ws2 ws, int32_t k, int32_t src,
                                                       int64_t *hull_offsets) {
    __shared__ uint32_t scratch[32];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < k; base += 1024) {
        const int i = base + (int)threadIdx.x;
        uint32_t h = 0;
        if (i < k && ws.nxt[i] >= 0) h = (uint32_t)ws.dist[src][i] + 1u;
        uint32_t v[1] = {h}, tot[1];
        block_excl_scan<1024, 1>(v, tot, scratch);
        if (i < k) hull_offsets[i] = (int64_t)(carry + v[0]);
        __syncthreads();
        if (threadIdx.x == 0) carry += tot[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) hull_offsets[k] = (int64_t)carry;
}

__global__ void k_emit(Ws2 ws, int32_t H, int32_t src, const int64_t *offsets,
                       const int64_t *hull_offsets, int32_t *hull_idx, int64_t n_total) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= H) return;
    if (ws.nxt[x] < 0) return;
    const int i = ws.hinst[x];
    const int64_t base = hull_offsets[i];
    const int64_t h = hull_offsets[i + 1] - base;
    const int64_t pos = base + (h - 1 - ws.dist[src][x]);
    if (pos < base || pos >= base + h || pos >= n_total) {
        atomicOr(&ws.ctl->error, kErrInternal);
        return;
    }
    hull_idx[pos] = (int32_t)(ws.V[x] - offsets[i]);
}

// ---------------------------------------------------------------------------
// host-side launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_instances(const Ws2 &ws, const int64_t *offsets, int64_t n_total, int32_t k,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_instances, dim3(1), dim3(1024), 0, st, ws, offsets, n_total, k);
    return hipGetLastError();
}

hipError_t launch_setup(const Ws2 &ws, const int64_t *offsets, int32_t k, int32_t ntiles,
                        int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_setup, dim3(grid), dim3(256), 0, st, ws, offsets, k, ntiles);
    return hipGetLastError();
}

hipError_t launch_extremes(const Ws2 &ws, const int32_t *x, const int32_t *y, int32_t n,
                           int32_t vec_ok, int grid, int32_t nseg_max, hipStream_t st) {
    hipLaunchKernelGGL((k_extremes<kBlock, kItems>), dim3(grid), dim3(kBlock), 0, st, ws, x, y, n,
                       vec_ok);
    hipLaunchKernelGGL((k_extremes_final<kBlock>), dim3(nseg_max), dim3(kBlock), 0, st, ws);
    return hipGetLastError();
}

hipError_t launch_round(const Ws2 &ws, int32_t r, bool init, int mode, const int32_t *x,
                        const int32_t *y, int32_t vec_ok, int grid, hipStream_t st) {
    if (init) {
        if (mode == 0)
            hipLaunchKernelGGL((k_round<true, 0, kBlock, kItems>), dim3(grid), dim3(kBlock), 0, st,
                               ws, r, x, y, vec_ok);
        else
            hipLaunchKernelGGL((k_round<true, 1, kBlock, kItems>), dim3(grid), dim3(kBlock), 0, st,
                               ws, r, x, y, vec_ok);
    } else {
        if (mode == 0)
            hipLaunchKernelGGL((k_round<false, 0, kBlock, kItems>), dim3(grid), dim3(kBlock), 0,
                               st, ws, r, x, y, vec_ok);
        else
            hipLaunchKernelGGL((k_round<false, 1, kBlock, kItems>), dim3(grid), dim3(kBlock), 0,
                               st, ws, r, x, y, vec_ok);
    }
    return hipGetLastError();
}

hipError_t launch_segments(const Ws2 &ws, int32_t r, int grid, hipStream_t st) {
    hipLaunchKernelGGL((k_segments<kSegBlock>), dim3(grid), dim3(kSegBlock), 0, st, ws, r);
    return hipGetLastError();
}

hipError_t launch_output(const Ws2 &ws, int32_t H, int32_t k, const int64_t *offsets,
                         int64_t *hull_offsets, int32_t *hull_idx, int64_t n_total, hipStream_t st) {
    int steps = 0;
    while ((1ll << steps) < (int64_t)H + 1) ++steps;
    int src = 0;
    if (H > 0) {
        if (H <= kRankSmallCap) {
            hipLaunchKernelGGL((k_rank_small<1024, kRankSmallCap>), dim3(1), dim3(1024), 0, st, ws,
                               H, steps);
        } else {
            const int grid = (H + 255) / 256;
            hipLaunchKernelGGL(k_rank_init, dim3(grid), dim3(256), 0, st, ws, H);
            for (int it = 0; it < steps; ++it) {
                hipLaunchKernelGGL(k_rank_step, dim3(grid), dim3(256), 0, st, ws, H, src);
                src ^= 1;
            }
        }
    }
    hipLaunchKernelGGL(k_hull_offsets, dim3(1), dim3(1024), 0, st, ws, k, src, hull_offsets);
    if (H > 0) {
        const int grid = (H + 255) / 256;
        hipLaunchKernelGGL(k_emit, dim3(grid), dim3(256), 0, st, ws, H, src, offsets, hull_offsets,
                           hull_idx, n_total);
    }
    return hipGetLastError();
}

__global__ void k_fill_offsets(int64_t *off, int64_t n) {
    if (threadIdx.x == 0) { off[0] = 0; off[1] = n; }
}

}  // namespace qh

hipError_t qh_fill_offsets(int64_t *off, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(qh::k_fill_offsets, dim3(1), dim3(64), 0, st, off, n);
    return hipGetLastError();
}
