// qh_select.hip -- order statistics of many segments in the permute-and-
// segment framework (Tzeng & Owens, Section 6: k-median finding as a
// flagPermute followed by a compact that throws away the part of a segment
// that does not hold the wanted rank; Sections 4.1 and 4.2 for the two
// primitives).
//
// Every round, for every segment still open:
//   1. a pivot: the value at a pseudo-random position of the segment;
//   2. states: 0 below the pivot, 1 equal to it, 2 above, and the segment's
//      count of each (per-block run totals, one global add per run);
//   3. a 3-state flagPermute groups each segment by state, stably;
//   4. the wanted rank falls in one group: in the equal group the pivot is
//      the answer and the segment closes; otherwise that group is kept (the
//      rank shifted past the lower groups);
//   5. a compact keeps the kept groups; each becomes the segment's new range.
// The kept group never holds the pivot, so every round shrinks every open
// segment; with random pivots the expected work is linear.  The three
// states (rather than the two of the paper's sketch) make equal values
// finish at once instead of needing a tie rule.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <new>
#include <vector>

#include "../../include/qh.h"
#include "qh_device.h"

namespace qhfp {
size_t fp_scratch_bytes(int64_t n, int32_t k);
hipError_t fp_enqueue(const int32_t *f, const uint8_t *s, int32_t n, int32_t k, int32_t *p, uint8_t *s_new,
                      void *scratch, int32_t *err_dev, hipStream_t st);
size_t cp_scratch_bytes(int64_t n);
hipError_t cp_enqueue(const uint8_t *b, const uint8_t *s, int32_t n, int32_t *p, uint8_t *s_new, void *scratch,
                      int32_t *count_dev, hipStream_t st);
}  // namespace qhfp

namespace qhsel {

constexpr int kB = 256;

// SplitMix64's output function (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014) on a counter made of the
// segment and the round: the pivot position of a segment in a round.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// inclusive sum over the block (waves by DPP, then the wave totals)
__device__ __forceinline__ uint32_t block_incl_sum(uint32_t v, uint32_t *red) {
    const int w = threadIdx.x / qh::kWave;
    const uint32_t inc = qh::wave_incl_sum(v);
    if (qh::lane_id() == qh::kWave - 1) red[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int j = 0; j < w; ++j) before += red[j];
    __syncthreads();
    return before + inc;
}

// segment of every element, the initial head flags and values
__global__ void k_sel_init(const int32_t *vals, int32_t n, const int64_t *off, int32_t k, int32_t *v, int32_t *sid,
                           uint8_t *s) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t lo = 0, hi = k - 1;  // the last segment whose start is <= i
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    v[i] = vals[i];
    sid[i] = lo;
    s[i] = (off[lo] == i) ? 1 : 0;
}

// per open segment: its start, length and rank (set up from the offsets)
__global__ void k_sel_segs(const int64_t *off, const int64_t *rank, int32_t k, int32_t *start, int32_t *len,
                           int64_t *rk, int8_t *open) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= k) return;
    start[g] = (int32_t)off[g];
    len[g] = (int32_t)(off[g + 1] - off[g]);
    rk[g] = rank[g];
    open[g] = 1;
}

__global__ void k_sel_pivot(const int32_t *v, int32_t k, int32_t round, const int32_t *start, const int32_t *len,
                            const int8_t *open, int32_t *pivot, uint32_t *cnt) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= k) return;
    cnt[3 * g + 0] = cnt[3 * g + 1] = cnt[3 * g + 2] = 0;
    if (!open[g]) return;
    const uint64_t h = mix64(((uint64_t)(uint32_t)g << 32) | (uint32_t)round);
    pivot[g] = v[start[g] + (int32_t)(h % (uint64_t)len[g])];
}

// states and per-segment counts: the elements of a block form runs of one
// segment (segments are contiguous); each run's counts go out in one add
__global__ __launch_bounds__(kB) void k_sel_state(const int32_t *v, const int32_t *sid, int32_t n,
                                                  const int32_t *pivot, int32_t *f, uint32_t *cnt) {
    __shared__ uint32_t lc[3][kB];
    __shared__ uint32_t red[kB / qh::kWave];
    const int32_t i = blockIdx.x * kB + threadIdx.x;
    const bool in = i < n;
    const int32_t g = in ? sid[i] : -1;
    int32_t st = 3;
    if (in) {
        const int32_t x = v[i], pv = pivot[g];
        st = x < pv ? 0 : (x == pv ? 1 : 2);
        f[i] = st;
    }
    // run index of this element inside the block
    const bool first = in && (threadIdx.x == 0 || sid[i - 1] != g);
    const uint32_t run = block_incl_sum(first ? 1u : 0u, red) - 1u;
    lc[0][threadIdx.x] = lc[1][threadIdx.x] = lc[2][threadIdx.x] = 0;
    __syncthreads();
    if (in) atomicAdd(&lc[st][run], 1u);
    __syncthreads();
    if (first) {
        for (int c = 0; c < 3; ++c)
            if (lc[c][run]) atomicAdd(&cnt[3 * g + c], lc[c][run]);
    }
}

__global__ void k_sel_scatter(const int32_t *p, int32_t n, const int32_t *v, const int32_t *sid, const int32_t *f,
                              int32_t *v2, int32_t *sid2, int32_t *f2) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t d = p[i];
    v2[d] = v[i];
    sid2[d] = sid[i];
    f2[d] = f[i];
}

// the group holding each open segment's rank: 1 closes the segment
__global__ void k_sel_decide(int32_t k, const uint32_t *cnt, const int32_t *pivot, int64_t *rk, int32_t *len,
                             int8_t *open, int8_t *keep, int32_t *out) {
    const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= k) return;
    keep[g] = -1;
    if (!open[g]) return;
    const int64_t c0 = cnt[3 * g + 0], c1 = cnt[3 * g + 1], c2 = cnt[3 * g + 2];
    const int64_t r = rk[g];
    if (r < c0) {
        keep[g] = 0;
        len[g] = (int32_t)c0;
    } else if (r < c0 + c1) {
        out[g] = pivot[g];
        open[g] = 0;
    } else {
        keep[g] = 2;
        rk[g] = r - c0 - c1;
        len[g] = (int32_t)c2;
    }
}

__global__ void k_sel_keep(const int32_t *sid, const int32_t *f, int32_t n, const int8_t *keep, uint8_t *b) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    b[i] = (f[i] == keep[sid[i]]) ? 1 : 0;
}

// the kept elements to the front; a segment's new start is its first kept one
__global__ void k_sel_pack(const uint8_t *b, const int32_t *p, int32_t n, const int32_t *v2, const int32_t *sid2,
                           const uint8_t *s_cmp, int32_t *v, int32_t *sid, int32_t *start) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !b[i]) return;
    const int32_t d = p[i];
    v[d] = v2[i];
    sid[d] = sid2[i];
    if (s_cmp[d]) start[sid2[i]] = d;
}

}  // namespace qhsel

#define QS_TRY(expr)                      \
    do {                                  \
        if ((expr) != hipSuccess) {       \
            (void)hipGetLastError();      \
            rc = QH_EDEVICE;              \
            goto done;                    \
        }                                 \
    } while (0)

extern "C" qh_status qh_select(const int32_t *vals, int64_t n, const int64_t *offsets, int32_t k,
                               const int64_t *ranks, int32_t *out, void *stream) {
    using namespace qhsel;
    if (n < 0 || n > (int64_t)INT32_MAX / 4 || k < 1 || k > (1 << 24)) return QH_EINVAL;
    if (!offsets || !ranks || !out || (n > 0 && !vals)) return QH_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    // the bounds and ranks, checked on the host: every segment non-empty and
    // every rank inside its segment
    std::vector<int64_t> off((size_t)k + 1), rk((size_t)k);
    if (hipMemcpyAsync(off.data(), offsets, sizeof(int64_t) * off.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(rk.data(), ranks, sizeof(int64_t) * rk.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        return QH_EDEVICE;
    }
    if (off[0] != 0 || off[(size_t)k] != n) return QH_EINVAL;
    for (int32_t g = 0; g < k; ++g)
        if (off[(size_t)g + 1] <= off[(size_t)g] || rk[(size_t)g] < 0 ||
            rk[(size_t)g] >= off[(size_t)g + 1] - off[(size_t)g])
            return QH_EINVAL;

    qh_status rc = QH_OK;
    const size_t N = (size_t)n, K = (size_t)k;
    // element arrays: values and segment ids twice, states twice, positions
    // twice, flags (heads, permuted heads, keep, compacted heads); segment
    // arrays; the primitives' scratch
    const size_t fp_b = qhfp::fp_scratch_bytes(n, 3), cp_b = qhfp::cp_scratch_bytes(n);
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t e32 = al(sizeof(int32_t) * N), e8 = al(N), s32 = al(sizeof(int32_t) * K);
    const size_t total = 8 * e32 + 4 * e8 + 6 * s32 + al(sizeof(int64_t) * K) + al(3 * sizeof(uint32_t) * K) +
                         2 * al(K) + al(fp_b) + al(cp_b) + 256;
    char *buf = nullptr;
    if (hipMalloc((void **)&buf, total) != hipSuccess) {
        (void)hipGetLastError();
        return QH_ENOMEM;
    }
    {
        char *q = buf;
        auto take = [&](size_t b) {
            char *r = q;
            q += b;
            return r;
        };
        int32_t *v = (int32_t *)take(e32), *v2 = (int32_t *)take(e32);
        int32_t *sid = (int32_t *)take(e32), *sid2 = (int32_t *)take(e32);
        int32_t *f = (int32_t *)take(e32), *f2 = (int32_t *)take(e32);
        int32_t *p = (int32_t *)take(e32), *pc = (int32_t *)take(e32);
        uint8_t *s = (uint8_t *)take(e8), *sp = (uint8_t *)take(e8), *b = (uint8_t *)take(e8),
                *sc = (uint8_t *)take(e8);
        int32_t *start = (int32_t *)take(s32), *len = (int32_t *)take(s32), *pivot = (int32_t *)take(s32);
        int32_t *misc = (int32_t *)take(s32);  // [0] flagPermute error, [1] kept count
        (void)take(s32);
        (void)take(s32);
        int64_t *rkd = (int64_t *)take(al(sizeof(int64_t) * K));
        uint32_t *cnt = (uint32_t *)take(al(3 * sizeof(uint32_t) * K));
        int8_t *open = (int8_t *)take(al(K)), *keep = (int8_t *)take(al(K));
        void *fps = take(al(fp_b)), *cps = take(al(cp_b));
        int32_t hm[2] = {0, 0};
        int32_t m = (int32_t)n;
        const dim3 eb(256), sb(256);
        auto eg = [](int32_t c) { return dim3((unsigned)((c + 255) / 256)); };
        hipLaunchKernelGGL(k_sel_init, eg(m), eb, 0, st, vals, m, offsets, k, v, sid, s);
        hipLaunchKernelGGL(k_sel_segs, eg(k), sb, 0, st, offsets, ranks, k, start, len, rkd, open);
        QS_TRY(hipGetLastError());
        QS_TRY(hipMemsetAsync(misc, 0, 2 * sizeof(int32_t), st));
        for (int32_t round = 0; m > 0; ++round) {
            if (round > n + 1) {  // every round shrinks every open segment
                rc = QH_EDEVICE;
                goto done;
            }
            hipLaunchKernelGGL(k_sel_pivot, eg(k), sb, 0, st, v, k, round, start, len, open, pivot, cnt);
            hipLaunchKernelGGL(k_sel_state, eg(m), dim3(kB), 0, st, v, sid, m, pivot, f, cnt);
            QS_TRY(hipGetLastError());
            QS_TRY(hipMemsetAsync(sp, 0, (size_t)m, st));
            QS_TRY(qhfp::fp_enqueue(f, s, m, 3, p, sp, fps, misc, st));
            hipLaunchKernelGGL(k_sel_scatter, eg(m), eb, 0, st, p, m, v, sid, f, v2, sid2, f2);
            hipLaunchKernelGGL(k_sel_decide, eg(k), sb, 0, st, k, cnt, pivot, rkd, len, open, keep, out);
            hipLaunchKernelGGL(k_sel_keep, eg(m), eb, 0, st, sid2, f2, m, keep, b);
            QS_TRY(hipGetLastError());
            QS_TRY(hipMemsetAsync(sc, 0, (size_t)m, st));
            QS_TRY(qhfp::cp_enqueue(b, sp, m, pc, sc, cps, misc + 1, st));
            hipLaunchKernelGGL(k_sel_pack, eg(m), eb, 0, st, b, pc, m, v2, sid2, sc, v, sid, start);
            QS_TRY(hipGetLastError());
            // the compacted head flags are the next round's segments
            QS_TRY(hipMemcpyAsync(s, sc, (size_t)m, hipMemcpyDeviceToDevice, st));
            QS_TRY(hipMemcpyAsync(hm, misc, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
            QS_TRY(hipStreamSynchronize(st));
            if (hm[0]) {  // a state outside [0, 3): cannot happen
                rc = QH_EDEVICE;
                goto done;
            }
            m = hm[1];
        }
    }
done:
    (void)hipGetLastError();
    (void)hipFree(buf);
    return rc;
}
