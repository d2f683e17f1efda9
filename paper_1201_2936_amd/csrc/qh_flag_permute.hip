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
// counts are differences of G at i, h and e.  One block sweeps the array
// forward (G for every state, h) and backward (e); a grid then writes p and
// s_new.  The Quickhull rounds do not call this: they fuse the same partition
// into their scatter.
#include <hip/hip_runtime.h>

#include <stdint.h>

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

// G: [k][n + 1] prefix counts, head: [n], end: [n]
__global__ __launch_bounds__(kB) void k_fp_sweep(const int32_t *f, const uint8_t *s, int32_t n,
                                                 int32_t k, int32_t *G, int32_t *head, int32_t *end,
                                                 int32_t *err) {
    __shared__ uint32_t red[kB / kWave];
    __shared__ int32_t mx[kB];
    __shared__ uint32_t carry[kMaxStates];
    __shared__ int32_t hcarry;
    if (threadIdx.x < kMaxStates) carry[threadIdx.x] = 0;
    if (threadIdx.x == 0) hcarry = 0;
    __syncthreads();
    bool bad = false;
    for (int32_t base = 0; base < n; base += kB) {
        const int32_t i = base + (int32_t)threadIdx.x;
        const bool in = i < n;
        const int32_t fi = in ? f[i] : -1;
        bad |= in && (fi < 0 || fi >= k);
        for (int c = 0; c < k; ++c) {
            const uint32_t m = (fi == c) ? 1u : 0u;
            const uint32_t inc = block_incl_sum(m, red);
            if (in) G[(int64_t)c * (n + 1) + i] = (int32_t)(carry[c] + inc - m);
            __syncthreads();
            if (threadIdx.x == kB - 1) carry[c] += inc;
            __syncthreads();
        }
        const int32_t hv = (in && (s[i] || i == 0)) ? i : hcarry;
        const int32_t h = block_incl_max(hv, mx);
        if (in) head[i] = h;
        __syncthreads();
        if (threadIdx.x == kB - 1) hcarry = h;
        __syncthreads();
    }
    if (threadIdx.x < k) G[(int64_t)threadIdx.x * (n + 1) + n] = (int32_t)carry[threadIdx.x];
    // backward: the end of every element's segment is the next head after it
    if (threadIdx.x == 0) hcarry = n;
    __syncthreads();
    const int32_t last = ((n + kB - 1) / kB - 1) * kB;
    for (int32_t base = last; base >= 0; base -= kB) {
        const int32_t i = base + (int32_t)threadIdx.x;
        const bool in = i < n;
        // a head at j ends the segment of every element before it
        const int32_t ev = (in && i + 1 < n && s[i + 1]) ? i + 1 : INT32_MAX;
        int32_t e = block_incl_min_rev(ev, mx);
        if (e > hcarry) e = hcarry;
        if (in) end[i] = e;
        __syncthreads();
        if (threadIdx.x == 0) hcarry = e;
        __syncthreads();
    }
    if (bad) atomicOr(err, 1);
}

__global__ void k_fp_apply(const int32_t *f, int32_t n, int32_t k, const int32_t *G,
                           const int32_t *head, const int32_t *end, int32_t *p, uint8_t *s_new) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t fi = f[i], h = head[i], e = end[i];
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

// compact (Section 4.2): P = exclusive sum of the keep flags b (n + 1
// entries), head = each element's segment head, as in the sweep above
__global__ __launch_bounds__(kB) void k_cp_sweep(const uint8_t *b, const uint8_t *s, int32_t n, int32_t *P,
                                                 int32_t *head) {
    __shared__ uint32_t red[kB / kWave];
    __shared__ int32_t mx[kB];
    __shared__ uint32_t carry;
    __shared__ int32_t hcarry;
    if (threadIdx.x == 0) {
        carry = 0;
        hcarry = 0;
    }
    __syncthreads();
    for (int32_t base = 0; base < n; base += kB) {
        const int32_t i = base + (int32_t)threadIdx.x;
        const bool in = i < n;
        const uint32_t m = (in && b[i]) ? 1u : 0u;
        const uint32_t inc = block_incl_sum(m, red);
        if (in) P[i] = (int32_t)(carry + inc - m);
        __syncthreads();
        if (threadIdx.x == kB - 1) carry += inc;
        __syncthreads();
        const int32_t hv = (in && (s[i] || i == 0)) ? i : hcarry;
        const int32_t h = block_incl_max(hv, mx);
        if (in) head[i] = h;
        __syncthreads();
        if (threadIdx.x == kB - 1) hcarry = h;
        __syncthreads();
    }
    if (threadIdx.x == 0) P[n] = (int32_t)carry;
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

size_t fp_scratch_bytes(int64_t n, int32_t k) {
    return sizeof(int32_t) * ((size_t)k * (size_t)(n + 1) + 2 * (size_t)n + 64);
}

// flagPermute into caller scratch (fp_scratch_bytes); *err_dev gets 1 for a
// state outside [0, k) (s_new must be zero on entry)
hipError_t fp_enqueue(const int32_t *f, const uint8_t *s, int32_t n, int32_t k, int32_t *p, uint8_t *s_new,
                      void *scratch, int32_t *err_dev, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int32_t *G = reinterpret_cast<int32_t *>(scratch);
    int32_t *head = G + (size_t)k * (size_t)(n + 1);
    int32_t *end = head + n;
    hipLaunchKernelGGL(k_fp_sweep, dim3(1), dim3(kB), 0, st, f, s, n, k, G, head, end, err_dev);
    hipLaunchKernelGGL(k_fp_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, f, n, k, G, head,
                       end, p, s_new);
    return hipGetLastError();
}

size_t cp_scratch_bytes(int64_t n) { return sizeof(int32_t) * (2 * (size_t)n + 64); }

// compact into caller scratch (cp_scratch_bytes); the kept count is left at
// *count_dev (s_new must be zero on entry)
hipError_t cp_enqueue(const uint8_t *b, const uint8_t *s, int32_t n, int32_t *p, uint8_t *s_new, void *scratch,
                      int32_t *count_dev, hipStream_t st) {
    int32_t *P = reinterpret_cast<int32_t *>(scratch);
    int32_t *head = P + n + 1;
    if (n <= 0) return hipMemsetAsync(count_dev, 0, sizeof(int32_t), st);
    hipLaunchKernelGGL(k_cp_sweep, dim3(1), dim3(kB), 0, st, b, s, n, P, head);
    hipLaunchKernelGGL(k_cp_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, b, n, P, head, p,
                       s_new);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
    return hipMemcpyAsync(count_dev, P + n, sizeof(int32_t), hipMemcpyDeviceToDevice, st);
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
    const size_t gbytes = sizeof(int32_t) * (size_t)k * (size_t)(n + 1);
    char *buf = nullptr;
    const size_t bytes = gbytes + sizeof(int32_t) * 2 * (size_t)n + 256;
    if (hipMalloc((void **)&buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return QH_ENOMEM;
    }
    int32_t *G = reinterpret_cast<int32_t *>(buf);
    int32_t *head = G + (size_t)k * (size_t)(n + 1);
    int32_t *end = head + n;
    int32_t *err = end + n;
    qh_status rc = QH_OK;
    int32_t herr = 0;
    if (hipMemsetAsync(err, 0, sizeof(int32_t), st) != hipSuccess ||
        hipMemsetAsync(s_new, 0, (size_t)n, st) != hipSuccess) {
        rc = QH_EDEVICE;
    } else {
        hipLaunchKernelGGL(qhfp::k_fp_sweep, dim3(1), dim3(qhfp::kB), 0, st, f, s, (int32_t)n, k, G,
                           head, end, err);
        if (hipMemcpyAsync(&herr, err, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = QH_EDEVICE;
        } else if (herr) {
            rc = QH_EINVAL;  // a state outside [0, k)
        } else {
            hipLaunchKernelGGL(qhfp::k_fp_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                               f, (int32_t)n, k, G, head, end, p, s_new);
            if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
                rc = QH_EDEVICE;
        }
    }
    (void)hipGetLastError();
    (void)hipFree(buf);
    return rc;
}
