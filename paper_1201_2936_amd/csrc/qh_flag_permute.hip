// qh_flag_permute.hip -- the k-state segmented stable partition on its own
// (flagPermute, Tzeng & Owens Section 4.1 and Figure 1).
//
// For element i with state f[i] in segment [h, e) (h = the nearest head at or
// before i), its new position is
//     p[i] = h + #{j in [h, e) : f[j] < f[i]} + #{j in [h, i) : f[j] = f[i]},
// so every segment keeps its range and its elements are grouped by state,
// stably.  s_new flags the first slot of every non-empty state group of every
// segment (the segment heads among them).
//
// With G_c(i) = #{j < i : f[j] = c} (a plain prefix count per state) both
// counts are differences of G at i, h and e.  Three launches over tiles give
// G, h and e (per-tile totals, a scan over the tiles, per-tile scans from
// their carries); a grid then writes p and s_new.  The Quickhull rounds do
// not call this: they fuse the same partition into their scatter.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <mutex>

#include "../../include/qh.h"
#include "qh_device.h"

namespace qhfp {

using qh::kWave;
using qh::lane_id;

constexpr int kB = 1024;
constexpr int kMaxStates = 16;

__device__ __forceinline__ uint32_t block_incl_sum(uint32_t v, uint32_t *lds) {
    const int w = threadIdx.x / kWave;
    const uint32_t inc = qh::wave_incl_sum(v);
    if (lane_id() == kWave - 1) lds[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int j = 0; j < w; ++j) before += lds[j];
    __syncthreads();
    return before + inc;
}

__device__ __forceinline__ int32_t block_incl_max(int32_t v, int32_t *lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kB; off <<= 1) {
        const int32_t o = threadIdx.x >= (unsigned)off ? lds[threadIdx.x - off] : INT32_MIN;
        __syncthreads();
        if (o > v) v = o;
        lds[threadIdx.x] = v;
        __syncthreads();
    }
    return v;
}

__device__ __forceinline__ int32_t block_incl_min_rev(int32_t v, int32_t *lds) {
    // minimum over this thread and every later thread
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kB; off <<= 1) {
        const int32_t o = threadIdx.x + off < (unsigned)kB ? lds[threadIdx.x + off] : INT32_MAX;
        __syncthreads();
        if (o < v) v = o;
        lds[threadIdx.x] = v;
        __syncthreads();
    }
    return v;
}

__global__ void k_fp_apply(const int32_t *f, int32_t n, int32_t k, const int32_t *G,
                           const int32_t *head, const int32_t *end, int32_t *p, uint8_t *s_new) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t fi = f[i], h = head[i], e = end[i];
    if (fi < 0 || fi >= k) return;  // reported through the error flag
    int32_t pos = h;
    for (int c = 0; c < fi; ++c) {
        const int32_t *Gc = G + (int64_t)c * (n + 1);
        pos += Gc[e] - Gc[h];
    }
    const int32_t *Gf = G + (int64_t)fi * (n + 1);
    const int32_t rank = Gf[i] - Gf[h];
    pos += rank;
    p[i] = pos;
    if (rank == 0) s_new[pos] = 1;
}

// p[i] = P[i]; a kept element with no kept element between its segment's
// head and itself starts the segment in the compacted array
__global__ void k_cp_apply(const uint8_t *b, int32_t n, const int32_t *P, const int32_t *head, int32_t *p,
                           uint8_t *s_new) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t pi = P[i];
    p[i] = pi;
    if (b[i] && pi == P[head[i]]) s_new[pi] = 1;
}

// ---------------------------------------------------------------------------
// The same prefix counts, heads and ends from three launches over tiles of
// kB elements instead of one block's sweep: per-tile totals, a scan over the
// tiles in one block, then every tile's own scans started from its carry.
// CP: compact (state 0 = kept, nothing else counted); else flagPermute.
// ---------------------------------------------------------------------------
template <bool CP>
__device__ __forceinline__ int32_t ms_state(const int32_t *f, const uint8_t *b, int32_t i) {
    return CP ? (b[i] ? 0 : -1) : f[i];
}

__device__ __forceinline__ int32_t block_max_all(int32_t v, int32_t *lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = kB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s && lds[threadIdx.x + s] > lds[threadIdx.x]) lds[threadIdx.x] = lds[threadIdx.x + s];
        __syncthreads();
    }
    const int32_t r = lds[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ int32_t block_min_all(int32_t v, int32_t *lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = kB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s && lds[threadIdx.x + s] < lds[threadIdx.x]) lds[threadIdx.x] = lds[threadIdx.x + s];
        __syncthreads();
    }
    const int32_t r = lds[0];
    __syncthreads();
    return r;
}

// pass 1: per tile, the count of every state, the last head and the first
// "next head" (ev) of the tile
template <bool CP>
__global__ __launch_bounds__(kB) void k_ms_tiles(const int32_t *f, const uint8_t *b, const uint8_t *s, int32_t n,
                                                 int32_t k, int32_t nt, int32_t *tcount, int32_t *tmaxh,
                                                 int32_t *tminev, int32_t *err) {
    __shared__ uint32_t red[kB / kWave];
    __shared__ int32_t mx[kB];
    const int32_t t = blockIdx.x;
    const int32_t i = t * kB + (int32_t)threadIdx.x;
    const bool in = i < n;
    const int32_t st = in ? ms_state<CP>(f, b, i) : -1;
    if (!CP && in && (st < 0 || st >= k)) atomicOr(err, 1);
    for (int c = 0; c < k; ++c) {
        const uint32_t inc = block_incl_sum(st == c ? 1u : 0u, red);
        if (threadIdx.x == kB - 1) tcount[(size_t)c * nt + t] = (int32_t)inc;
    }
    const int32_t hv = (in && (s[i] || i == 0)) ? i : -1;
    const int32_t hm = block_max_all(hv, mx);
    const int32_t ev = (in && i + 1 < n && s[i + 1]) ? i + 1 : INT32_MAX;
    const int32_t em = block_min_all(ev, mx);
    if (threadIdx.x == 0) {
        tmaxh[t] = hm;
        tminev[t] = em;
    }
}

// pass 2 (one block): exclusive sums of the tile counts per state, the last
// head before each tile, the first next-head after each tile; the totals
// go to G[c][n]
__global__ __launch_bounds__(kB) void k_ms_scan(int32_t n, int32_t k, int32_t nt, const int32_t *tcount,
                                                const int32_t *tmaxh, const int32_t *tminev, int32_t *tbase,
                                                int32_t *thead, int32_t *tnext, int32_t *G) {
    __shared__ uint32_t red[kB / kWave];
    __shared__ int32_t mx[kB];
    __shared__ uint32_t carry;
    __shared__ int32_t hcarry;
    for (int c = 0; c < k; ++c) {
        if (threadIdx.x == 0) carry = 0;
        __syncthreads();
        for (int32_t base = 0; base < nt; base += kB) {
            const int32_t t = base + (int32_t)threadIdx.x;
            const uint32_t v = t < nt ? (uint32_t)tcount[(size_t)c * nt + t] : 0u;
            const uint32_t inc = block_incl_sum(v, red);
            if (t < nt) tbase[(size_t)c * nt + t] = (int32_t)(carry + inc - v);
            __syncthreads();
            if (threadIdx.x == kB - 1) carry += inc;
            __syncthreads();
        }
        if (threadIdx.x == 0) G[(size_t)c * (size_t)(n + 1) + n] = (int32_t)carry;
        __syncthreads();
    }
    // heads: the last head of the earlier tiles (element 0 is one)
    if (threadIdx.x == 0) hcarry = 0;
    __syncthreads();
    for (int32_t base = 0; base < nt; base += kB) {
        const int32_t t = base + (int32_t)threadIdx.x;
        const int32_t v = t < nt ? tmaxh[t] : -1;
        int32_t h = block_incl_max(v, mx);  // over this chunk's tiles up to t
        // exclusive: the tiles before t
        mx[threadIdx.x] = h;
        __syncthreads();
        int32_t ex = threadIdx.x ? mx[threadIdx.x - 1] : -1;
        if (ex < hcarry) ex = hcarry;
        if (t < nt) thead[t] = ex;
        __syncthreads();
        if (threadIdx.x == kB - 1 && h > hcarry) hcarry = h;
        __syncthreads();
    }
    // next heads: the first of the later tiles (n when none)
    if (threadIdx.x == 0) hcarry = n;
    __syncthreads();
    const int32_t last = ((nt + kB - 1) / kB - 1) * kB;
    for (int32_t base = last; base >= 0; base -= kB) {
        const int32_t t = base + (int32_t)threadIdx.x;
        const int32_t v = t < nt ? tminev[t] : INT32_MAX;
        int32_t e = block_incl_min_rev(v, mx);  // over this chunk's tiles from t on
        mx[threadIdx.x] = e;
        __syncthreads();
        int32_t ex = threadIdx.x + 1 < kB ? mx[threadIdx.x + 1] : INT32_MAX;
        if (ex > hcarry) ex = hcarry;
        if (t < nt) tnext[t] = ex;
        __syncthreads();
        if (threadIdx.x == 0 && e < hcarry) hcarry = e;
        __syncthreads();
    }
}

// pass 3: every tile's prefix counts, heads and ends from its carries
template <bool CP>
__global__ __launch_bounds__(kB) void k_ms_fill(const int32_t *f, const uint8_t *b, const uint8_t *s, int32_t n,
                                                int32_t k, int32_t nt, const int32_t *tbase, const int32_t *thead,
                                                const int32_t *tnext, int32_t *G, int32_t *head, int32_t *end) {
    __shared__ uint32_t red[kB / kWave];
    __shared__ int32_t mx[kB];
    const int32_t t = blockIdx.x;
    const int32_t i = t * kB + (int32_t)threadIdx.x;
    const bool in = i < n;
    const int32_t st = in ? ms_state<CP>(f, b, i) : -1;
    for (int c = 0; c < k; ++c) {
        const uint32_t m = st == c ? 1u : 0u;
        const uint32_t inc = block_incl_sum(m, red);
        if (in) G[(size_t)c * (size_t)(n + 1) + i] = tbase[(size_t)c * nt + t] + (int32_t)(inc - m);
    }
    const int32_t hv = (in && (s[i] || i == 0)) ? i : -1;
    int32_t h = block_incl_max(hv, mx);
    if (h < thead[t]) h = thead[t];
    if (in) head[i] = h;
    if (!CP) {
        const int32_t ev = (in && i + 1 < n && s[i + 1]) ? i + 1 : INT32_MAX;
        int32_t e = block_incl_min_rev(ev, mx);
        if (e > tnext[t]) e = tnext[t];
        if (e > n) e = n;
        if (in) end[i] = e;
    }
}

inline int32_t ms_tiles(int64_t n) { return (int32_t)((n + kB - 1) / kB); }

size_t fp_scratch_bytes(int64_t n, int32_t k) {
    return sizeof(int32_t) * ((size_t)k * (size_t)(n + 1) + 2 * (size_t)n + 64 +
                              (size_t)(2 * k + 4) * (size_t)ms_tiles(n));
}

// flagPermute into caller scratch (fp_scratch_bytes); *err_dev gets 1 for a
// state outside [0, k) (s_new must be zero on entry)
hipError_t fp_enqueue(const int32_t *f, const uint8_t *s, int32_t n, int32_t k, int32_t *p, uint8_t *s_new,
                      void *scratch, int32_t *err_dev, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int32_t nt = ms_tiles(n);
    int32_t *G = reinterpret_cast<int32_t *>(scratch);
    int32_t *head = G + (size_t)k * (size_t)(n + 1);
    int32_t *end = head + n;
    int32_t *tcount = end + n + 64, *tbase = tcount + (size_t)k * nt;
    int32_t *tmaxh = tbase + (size_t)k * nt, *tminev = tmaxh + nt, *thead = tminev + nt, *tnext = thead + nt;
    hipLaunchKernelGGL(k_ms_tiles<false>, dim3(nt), dim3(kB), 0, st, f, nullptr, s, n, k, nt, tcount, tmaxh,
                       tminev, err_dev);
    hipLaunchKernelGGL(k_ms_scan, dim3(1), dim3(kB), 0, st, n, k, nt, tcount, tmaxh, tminev, tbase, thead, tnext,
                       G);
    hipLaunchKernelGGL(k_ms_fill<false>, dim3(nt), dim3(kB), 0, st, f, nullptr, s, n, k, nt, tbase, thead, tnext,
                       G, head, end);
    hipLaunchKernelGGL(k_fp_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, f, n, k, G, head,
                       end, p, s_new);
    return hipGetLastError();
}

size_t cp_scratch_bytes(int64_t n) {
    return sizeof(int32_t) * (2 * (size_t)n + 64 + 6 * (size_t)ms_tiles(n));
}

// compact into caller scratch (cp_scratch_bytes); the kept count is left at
// *count_dev (s_new must be zero on entry)
hipError_t cp_enqueue(const uint8_t *b, const uint8_t *s, int32_t n, int32_t *p, uint8_t *s_new, void *scratch,
                      int32_t *count_dev, hipStream_t st) {
    int32_t *P = reinterpret_cast<int32_t *>(scratch);
    int32_t *head = P + n + 1;
    if (n <= 0) return hipMemsetAsync(count_dev, 0, sizeof(int32_t), st);
    const int32_t nt = ms_tiles(n);
    int32_t *tcount = head + n + 32, *tbase = tcount + nt;
    int32_t *tmaxh = tbase + nt, *tminev = tmaxh + nt, *thead = tminev + nt, *tnext = thead + nt;
    hipLaunchKernelGGL(k_ms_tiles<true>, dim3(nt), dim3(kB), 0, st, nullptr, b, s, n, 1, nt, tcount, tmaxh, tminev,
                       nullptr);
    hipLaunchKernelGGL(k_ms_scan, dim3(1), dim3(kB), 0, st, n, 1, nt, tcount, tmaxh, tminev, tbase, thead, tnext, P);
    hipLaunchKernelGGL(k_ms_fill<true>, dim3(nt), dim3(kB), 0, st, nullptr, b, s, n, 1, nt, tbase, thead, tnext, P,
                       head, nullptr);
    hipLaunchKernelGGL(k_cp_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, b, n, P, head, p,
                       s_new);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    return hipMemcpyAsync(count_dev, P + n, sizeof(int32_t), hipMemcpyDeviceToDevice, st);
}

// ---------------------------------------------------------------------------
// Fixed scratch of the entry point that allocates nothing: one copy of this
// array per device (it lives as long as the process), reached from the host
// only through the address hipGetSymbolAddress returns on that device.
// Bytes 0 .. 255 hold the bad-state flag, the rest the prefix counts.
// ---------------------------------------------------------------------------
constexpr size_t kFixedScratchBytes = (size_t)64 << 20;
constexpr size_t kFixedHeader = 256;
__device__ __align__(256) char scratch[kFixedScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void *g_fixed_ptr[kMaxDevices];

// the device address of scratch on the current device (looked up once per
// device, with that device current)
hipError_t fixed_scratch(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    if (!g_fixed_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_fixed_ptr[dev] = ptr;
    }
    *out = g_fixed_ptr[dev];
    return hipSuccess;
}

// zero s_new[0, n) and the flag word (a kernel, not a memset node, so the
// launches stay valid inside a captured graph)
__global__ void k_fp_clear(uint8_t *s_new, int32_t n, int32_t *err) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *err = 0;
    if (i < n) s_new[i] = 0;
}

}  // namespace qhfp

extern "C" qh_status qh_test_compact(const uint8_t *b, const uint8_t *s, int64_t n, int32_t *p, uint8_t *s_new,
                                     int64_t *m, void *stream) {
    if (m) *m = 0;
    if (!m || n < 0 || n > (int64_t)INT32_MAX / 2) return QH_EINVAL;
    if (n == 0) return QH_OK;
    if (!b || !s || !p || !s_new) return QH_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    char *buf = nullptr;
    if (hipMalloc((void **)&buf, qhfp::cp_scratch_bytes(n) + 256) != hipSuccess) {
        (void)hipGetLastError();
        return QH_ENOMEM;
    }
    int32_t *cnt = reinterpret_cast<int32_t *>(buf + qhfp::cp_scratch_bytes(n));
    int32_t hc = 0;
    qh_status rc = QH_OK;
    if (hipMemsetAsync(s_new, 0, (size_t)n, st) != hipSuccess ||
        qhfp::cp_enqueue(b, s, (int32_t)n, p, s_new, buf, cnt, st) != hipSuccess ||
        hipMemcpyAsync(&hc, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        rc = QH_EDEVICE;
    (void)hipGetLastError();
    (void)hipFree(buf);
    if (rc == QH_OK) *m = hc;
    return rc;
}

extern "C" qh_status qh_test_flag_permute(const int32_t *f, const uint8_t *s, int64_t n, int32_t k,
                                          int32_t *p, uint8_t *s_new, void *stream) {
    if (n < 0 || n > (int64_t)INT32_MAX / 2 || k < 1 || k > qhfp::kMaxStates) return QH_EINVAL;
    if (n == 0) return QH_OK;
    if (!f || !s || !p || !s_new) return QH_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const size_t sb = qhfp::fp_scratch_bytes(n, k);
    char *buf = nullptr;
    if (hipMalloc((void **)&buf, sb + 256) != hipSuccess) {
        (void)hipGetLastError();
        return QH_ENOMEM;
    }
    int32_t *err = reinterpret_cast<int32_t *>(buf + sb);
    int32_t herr = 0;
    qh_status rc = QH_OK;
    if (hipMemsetAsync(err, 0, sizeof(int32_t), st) != hipSuccess ||
        hipMemsetAsync(s_new, 0, (size_t)n, st) != hipSuccess ||
        qhfp::fp_enqueue(f, s, (int32_t)n, k, p, s_new, buf, err, st) != hipSuccess ||
        hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        rc = QH_EDEVICE;
    else if (herr)
        rc = QH_EINVAL;  // a state outside [0, k): the outputs are not written for it
    (void)hipGetLastError();
    (void)hipFree(buf);
    return rc;
}

extern "C" qh_status qh_test_flag_permute_noalloc(const int32_t *f, const uint8_t *s, int64_t n, int32_t k,
                                                  int32_t *p, uint8_t *s_new, void *stream) {
    if (n < 0 || n > (int64_t)INT32_MAX / 2 || k < 1 || k > qhfp::kMaxStates) return QH_EINVAL;
    if (n == 0) return QH_OK;
    if (!f || !s || !p || !s_new) return QH_EINVAL;
    if (qhfp::fp_scratch_bytes(n, k) > qhfp::kFixedScratchBytes - qhfp::kFixedHeader) return QH_ECAPACITY;
    hipStream_t st = (hipStream_t)stream;
    void *base = nullptr;
    if (qhfp::fixed_scratch(&base) != hipSuccess) {
        (void)hipGetLastError();
        return QH_EDEVICE;
    }
    int32_t *err = reinterpret_cast<int32_t *>(base);
    char *buf = reinterpret_cast<char *>(base) + qhfp::kFixedHeader;
    int32_t herr = 0;
    qh_status rc = QH_OK;
    hipLaunchKernelGGL(qhfp::k_fp_clear, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s_new, (int32_t)n,
                       err);
    if (hipGetLastError() != hipSuccess ||
        qhfp::fp_enqueue(f, s, (int32_t)n, k, p, s_new, buf, err, st) != hipSuccess ||
        hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        rc = QH_EDEVICE;
    else if (herr)
        rc = QH_EINVAL;
    (void)hipGetLastError();
    return rc;
}
