// qh3d_kernels.hip -- the device side of the 3D segmented Quickhull on gfx950.
//
// Quickhull in three dimensions (Tzeng & Owens, Section 3.2 and Algorithm 1;
// the 3D discussion of Section 4.3) as kernels around a host topology step:
//
//   init       the first simplex: lexicographic extremes a, b (and the
//              coordinate range check), the point c farthest from the line
//              ab, the point d farthest from the plane abc; three block
//              reductions over the input, each finished by one block
//   classify   every point of a removed facet is tested against the new
//              facets of its cone in id order and goes to the first one it
//              is strictly above, or is dropped (inside the hull of the old
//              hull and the apex); pass 1 counts per new facet, pass 2
//              scatters into the ranges the host allocated (a k-state
//              flagPermute with compact, Sections 4.1-4.2)
//   apex       per facet with outside points, the farthest point above it
//              (segmented argmax, per tile in a block, tiles merged per
//              facet by one wave)
//   gather     compaction of the point pool (live ranges copied)
//
// Points live in a pool of structure-of-arrays planes x, y, z, idx; the
// outside set of a facet is one contiguous range of it.  Every predicate is
// an exact int64 expression: with |coordinate| <= 2^19 the normal has
// components below 2^41 and n . p stays below 3 * 2^60.
#include "qh3d.h"

namespace qh3 {

using qh::kWave;
using qh::lane_id;

// ---------------------------------------------------------------------------
// initial simplex
// ---------------------------------------------------------------------------
// Reduction key: primary (unsigned 128-bit, larger wins), then s1, s2 and the
// index (smaller wins).  idx < 0 marks an empty key.
struct IKey {
    unsigned __int128 k;
    int64_t s1, s2;
    int32_t idx;
    int32_t pad;
};

__device__ __forceinline__ bool ikey_better(const IKey &a, const IKey &b) {
    if (a.idx < 0) return false;
    if (b.idx < 0) return true;
    if (a.k != b.k) return a.k > b.k;
    if (a.s1 != b.s1) return a.s1 < b.s1;
    if (a.s2 != b.s2) return a.s2 < b.s2;
    return a.idx < b.idx;
}

__device__ __forceinline__ IKey ikey_empty() {
    IKey e;
    e.k = 0;
    e.s1 = 0;
    e.s2 = 0;
    e.idx = -1;
    e.pad = 0;
    return e;
}

__device__ __forceinline__ void ikey_take(IKey &dst, const IKey &src) {
    if (ikey_better(src, dst)) {
        dst.k = src.k;
        dst.s1 = src.s1;
        dst.s2 = src.s2;
        dst.idx = src.idx;
    }
}

// Block-wide best of NK keys per thread; thread 0 gets the result.
template <int NK>
__device__ __forceinline__ void block_best(IKey (&v)[NK], IKey *lds) {
    for (int j = 0; j < NK; ++j) {
        lds[j * kBlock + threadIdx.x] = v[j];
    }
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int j = 0; j < NK; ++j) {
                IKey o = lds[j * kBlock + threadIdx.x + s];
                IKey m = lds[j * kBlock + threadIdx.x];
                ikey_take(m, o);
                lds[j * kBlock + threadIdx.x] = m;
            }
        }
        __syncthreads();
    }
    for (int j = 0; j < NK; ++j) v[j] = lds[j * kBlock];
}

// 21 bits per coordinate, monotone in (x, y, z) for |c| < 2^20
__device__ __forceinline__ unsigned __int128 lex_pack(int32_t x, int32_t y, int32_t z) {
    const uint64_t ux = (uint64_t)(int64_t)(x + (1 << 20));
    const uint64_t uy = (uint64_t)(int64_t)(y + (1 << 20));
    const uint64_t uz = (uint64_t)(int64_t)(z + (1 << 20));
    return (unsigned __int128)((ux << 42) | (uy << 21) | uz);
}

struct InitScratch {
    IKey part[1];  // [2 * grid]
};

// The per-point keys of the three searches (index i, coordinates p):
// the lexicographic minimum and maximum (ties to the smaller index) ...
__device__ __forceinline__ void ext_keys(int32_t i, int32_t px, int32_t py, int32_t pz, IKey &kmin, IKey &kmax) {
    const unsigned __int128 all = ((unsigned __int128)1 << 63) * 2 - 1;
    const unsigned __int128 k = lex_pack(px, py, pz);
    kmin.k = all - k;  // smaller coordinates win
    kmin.s1 = kmin.s2 = 0;
    kmin.idx = i;
    kmax.k = k;
    kmax.s1 = kmax.s2 = 0;
    kmax.idx = i;
}

__device__ __forceinline__ bool out_of_range(int32_t px, int32_t py, int32_t pz) {
    return px < -kCoordMax || px > kCoordMax || py < -kCoordMax || py > kCoordMax || pz < -kCoordMax ||
           pz > kCoordMax;
}

// ... the distance from the line a + t e (squared |e x r|, r = p - a; then
// the smallest r . e); false for a point on the line ...
__device__ __forceinline__ bool line_key(int32_t i, int32_t px, int32_t py, int32_t pz, int64_t ax, int64_t ay,
                                         int64_t az, int64_t ex, int64_t ey, int64_t ez, IKey &k) {
    const int64_t rx = px - ax, ry = py - ay, rz = pz - az;
    const int64_t wx = ey * rz - ez * ry, wy = ez * rx - ex * rz, wz = ex * ry - ey * rx;
    if ((wx | wy | wz) == 0) return false;
    k.k = (unsigned __int128)((__int128)wx * wx) + (unsigned __int128)((__int128)wy * wy) +
          (unsigned __int128)((__int128)wz * wz);
    k.s1 = rx * ex + ry * ey + rz * ez;
    k.s2 = 0;
    k.idx = i;
    return true;
}

// ... and the distance from the plane through a with normal n (|n . r|;
// then the smallest r . b', r . c' with b', c' the edges from a); false for
// a point on the plane
__device__ __forceinline__ bool plane_key(int32_t i, int32_t px, int32_t py, int32_t pz, int64_t ax, int64_t ay,
                                          int64_t az, int64_t nx, int64_t ny, int64_t nz, int64_t bx, int64_t by,
                                          int64_t bz, int64_t cx, int64_t cy, int64_t cz, IKey &k) {
    const int64_t rx = px - ax, ry = py - ay, rz = pz - az;
    int64_t s = nx * rx + ny * ry + nz * rz;
    if (s == 0) return false;
    if (s < 0) s = -s;
    k.k = (unsigned __int128)(uint64_t)s;
    k.s1 = rx * bx + ry * by + rz * bz;
    k.s2 = rx * cx + ry * cy + rz * cz;
    k.idx = i;
    return true;
}

__global__ __launch_bounds__(kBlock) void k3_ext_partial(const int32_t *x, const int32_t *y,
                                                         const int32_t *z, int32_t n, IKey *part,
                                                         InitRes *res) {
    __shared__ IKey lds[2 * kBlock];
    IKey v[2] = {ikey_empty(), ikey_empty()};
    bool bad = false;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const int32_t px = x[i], py = y[i], pz = z[i];
        bad |= out_of_range(px, py, pz);
        IKey kmin, kmax;
        ext_keys(i, px, py, pz, kmin, kmax);
        ikey_take(v[0], kmin);
        ikey_take(v[1], kmax);
    }
    if (bad) atomicOr(&res->error, 1);
    block_best<2>(v, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x + 0] = v[0];
        part[2 * blockIdx.x + 1] = v[1];
    }
}

__global__ __launch_bounds__(kBlock) void k3_ext_final(const int32_t *x, const int32_t *y,
                                                       const int32_t *z, const IKey *part, int grid,
                                                       InitRes *res) {
    __shared__ IKey lds[2 * kBlock];
    IKey v[2] = {ikey_empty(), ikey_empty()};
    for (int b = threadIdx.x; b < grid; b += kBlock) {
        ikey_take(v[0], part[2 * b + 0]);
        ikey_take(v[1], part[2 * b + 1]);
    }
    block_best<2>(v, lds);
    if (threadIdx.x == 0) {
        res->a = v[0].idx;
        res->b = v[1].idx;
        res->c = -1;
        res->d = -1;
        for (int j = 0; j < 2; ++j) {
            const int32_t i = v[j].idx;
            res->coords[j][0] = i >= 0 ? x[i] : 0;
            res->coords[j][1] = i >= 0 ? y[i] : 0;
            res->coords[j][2] = i >= 0 ? z[i] : 0;
        }
    }
}

// c: the point farthest from the line ab, |(b - a) x (p - a)|^2, then the
// smallest (p - a).(b - a), then the index
__global__ __launch_bounds__(kBlock) void k3_line_partial(const int32_t *x, const int32_t *y,
                                                          const int32_t *z, int32_t n, IKey *part,
                                                          const InitRes *res) {
    __shared__ IKey lds[kBlock];
    IKey v[1] = {ikey_empty()};
    const int64_t ax = res->coords[0][0], ay = res->coords[0][1], az = res->coords[0][2];
    const int64_t ex = res->coords[1][0] - ax, ey = res->coords[1][1] - ay,
                  ez = res->coords[1][2] - az;
    if (res->error == 0) {
        for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
            IKey k;
            if (line_key(i, x[i], y[i], z[i], ax, ay, az, ex, ey, ez, k)) ikey_take(v[0], k);
        }
    }
    block_best<1>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(kBlock) void k3_line_final(const int32_t *x, const int32_t *y,
                                                        const int32_t *z, const IKey *part,
                                                        int grid, InitRes *res) {
    __shared__ IKey lds[kBlock];
    IKey v[1] = {ikey_empty()};
    for (int b = threadIdx.x; b < grid; b += kBlock) ikey_take(v[0], part[b]);
    block_best<1>(v, lds);
    if (threadIdx.x == 0) {
        const int32_t i = v[0].idx;
        res->c = i;
        res->coords[2][0] = i >= 0 ? x[i] : 0;
        res->coords[2][1] = i >= 0 ? y[i] : 0;
        res->coords[2][2] = i >= 0 ? z[i] : 0;
    }
}

// d: the point farthest from the plane abc on either side, then the smallest
// (p - a).(b - a), then (p - a).(c - a), then the index
__global__ __launch_bounds__(kBlock) void k3_plane_partial(const int32_t *x, const int32_t *y,
                                                           const int32_t *z, int32_t n, IKey *part,
                                                           const InitRes *res) {
    __shared__ IKey lds[kBlock];
    IKey v[1] = {ikey_empty()};
    if (res->error == 0 && res->c >= 0) {
        const int64_t ax = res->coords[0][0], ay = res->coords[0][1], az = res->coords[0][2];
        const int64_t bx = res->coords[1][0] - ax, by = res->coords[1][1] - ay,
                      bz = res->coords[1][2] - az;
        const int64_t cx = res->coords[2][0] - ax, cy = res->coords[2][1] - ay,
                      cz = res->coords[2][2] - az;
        const int64_t nx = by * cz - bz * cy, ny = bz * cx - bx * cz, nz = bx * cy - by * cx;
        for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
            IKey k;
            if (plane_key(i, x[i], y[i], z[i], ax, ay, az, nx, ny, nz, bx, by, bz, cx, cy, cz, k))
                ikey_take(v[0], k);
        }
    }
    block_best<1>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(kBlock) void k3_plane_final(const int32_t *x, const int32_t *y,
                                                         const int32_t *z, const IKey *part,
                                                         int grid, InitRes *res) {
    __shared__ IKey lds[kBlock];
    IKey v[1] = {ikey_empty()};
    for (int b = threadIdx.x; b < grid; b += kBlock) ikey_take(v[0], part[b]);
    block_best<1>(v, lds);
    if (threadIdx.x == 0) {
        const int32_t i = v[0].idx;
        res->d = i;
        res->coords[3][0] = i >= 0 ? x[i] : 0;
        res->coords[3][1] = i >= 0 ? y[i] : 0;
        res->coords[3][2] = i >= 0 ? z[i] : 0;
    }
}

__global__ void k3_init_clear(InitRes *res) {
    if (threadIdx.x == 0) {
        res->a = res->b = res->c = res->d = -1;
        res->error = 0;
    }
}

// The first simplex of many small instances, one block each: the same three
// searches and keys as above, in turn, with block reductions only.  Instance
// list[blockIdx.x] is the points [off[i], off[i+1]); its indices are local.
__global__ __launch_bounds__(kBlock) void k3_init_small(const int32_t *x, const int32_t *y, const int32_t *z,
                                                        const int64_t *off, const int32_t *list, InitRes *res) {
    __shared__ IKey lds[2 * kBlock];
    __shared__ int32_t sp[4][3];
    const int32_t inst = list[blockIdx.x];
    const int64_t lo = off[inst];
    const int32_t n = (int32_t)(off[inst + 1] - lo);
    const int32_t *px = x + lo, *py = y + lo, *pz = z + lo;
    InitRes *r = res + inst;
    // a, b: the lexicographic extremes, and the range check
    IKey v[2] = {ikey_empty(), ikey_empty()};
    bool bad = false;
    for (int32_t i = threadIdx.x; i < n; i += kBlock) {
        bad |= out_of_range(px[i], py[i], pz[i]);
        IKey kmin, kmax;
        ext_keys(i, px[i], py[i], pz[i], kmin, kmax);
        ikey_take(v[0], kmin);
        ikey_take(v[1], kmax);
    }
    const bool anybad = __syncthreads_or(bad);
    block_best<2>(v, lds);
    const int32_t ia = v[0].idx, ib = v[1].idx;
    if (threadIdx.x == 0) {
        sp[0][0] = px[ia]; sp[0][1] = py[ia]; sp[0][2] = pz[ia];
        sp[1][0] = px[ib]; sp[1][1] = py[ib]; sp[1][2] = pz[ib];
    }
    __syncthreads();
    const int64_t ax = sp[0][0], ay = sp[0][1], az = sp[0][2];
    // c: farthest from the line ab
    IKey w[1] = {ikey_empty()};
    if (!anybad) {
        const int64_t ex = sp[1][0] - ax, ey = sp[1][1] - ay, ez = sp[1][2] - az;
        for (int32_t i = threadIdx.x; i < n; i += kBlock) {
            IKey k;
            if (line_key(i, px[i], py[i], pz[i], ax, ay, az, ex, ey, ez, k)) ikey_take(w[0], k);
        }
    }
    block_best<1>(w, lds);
    const int32_t ic = w[0].idx;
    if (threadIdx.x == 0 && ic >= 0) { sp[2][0] = px[ic]; sp[2][1] = py[ic]; sp[2][2] = pz[ic]; }
    __syncthreads();
    // d: farthest from the plane abc
    IKey u[1] = {ikey_empty()};
    if (!anybad && ic >= 0) {
        const int64_t bx = sp[1][0] - ax, by = sp[1][1] - ay, bz = sp[1][2] - az;
        const int64_t cx = sp[2][0] - ax, cy = sp[2][1] - ay, cz = sp[2][2] - az;
        const int64_t nx = by * cz - bz * cy, ny = bz * cx - bx * cz, nz = bx * cy - by * cx;
        for (int32_t i = threadIdx.x; i < n; i += kBlock) {
            IKey k;
            if (plane_key(i, px[i], py[i], pz[i], ax, ay, az, nx, ny, nz, bx, by, bz, cx, cy, cz, k))
                ikey_take(u[0], k);
        }
    }
    block_best<1>(u, lds);
    if (threadIdx.x == 0) {
        const int32_t id = u[0].idx;
        r->a = ia;
        r->b = ib;
        r->c = ic;
        r->d = id;
        for (int q = 0; q < 3; ++q) {
            r->coords[0][q] = sp[0][q];
            r->coords[1][q] = sp[1][q];
            r->coords[2][q] = ic >= 0 ? sp[2][q] : 0;
        }
        r->coords[3][0] = id >= 0 ? px[id] : 0;
        r->coords[3][1] = id >= 0 ? py[id] : 0;
        r->coords[3][2] = id >= 0 ? pz[id] : 0;
        r->error = anybad ? 1 : 0;
        r->pad[0] = r->pad[1] = r->pad[2] = 0;
    }
}

hipError_t launch_init_small(const int32_t *x, const int32_t *y, const int32_t *z, const int64_t *off,
                             const int32_t *list, int32_t count, InitRes *res, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k3_init_small, dim3(count), dim3(kBlock), 0, st, x, y, z, off, list, res);
    return hipGetLastError();
}

size_t init_scratch_bytes(int grid) { return sizeof(IKey) * 2 * (size_t)grid; }

hipError_t launch_init(const int32_t *x, const int32_t *y, const int32_t *z, int32_t n,
                       void *scratch, InitRes *res, int grid, hipStream_t st) {
    IKey *part = reinterpret_cast<IKey *>(scratch);
    hipLaunchKernelGGL(k3_init_clear, dim3(1), dim3(64), 0, st, res);
    hipLaunchKernelGGL(k3_ext_partial, dim3(grid), dim3(kBlock), 0, st, x, y, z, n, part, res);
    hipLaunchKernelGGL(k3_ext_final, dim3(1), dim3(kBlock), 0, st, x, y, z, part, grid, res);
    hipLaunchKernelGGL(k3_line_partial, dim3(grid), dim3(kBlock), 0, st, x, y, z, n, part, res);
    hipLaunchKernelGGL(k3_line_final, dim3(1), dim3(kBlock), 0, st, x, y, z, part, grid, res);
    hipLaunchKernelGGL(k3_plane_partial, dim3(grid), dim3(kBlock), 0, st, x, y, z, n, part, res);
    hipLaunchKernelGGL(k3_plane_final, dim3(1), dim3(kBlock), 0, st, x, y, z, part, grid, res);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// tile -> range lookup (uniform per block)
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ int32_t find_range(const R *r, int32_t nr, int32_t t) {
    int32_t lo = 0, hi = nr - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (r[mid].tile0 <= t) lo = mid;
        else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l ? (~0ull >> (64 - l)) : 0ull;
}

// FP32 filter of the plane test d = n.p - off.  With |coordinate| <= 2^19
// the coordinates are exact floats; the normal components and the offset
// are rounded once when converted.  Each of the four terms then passes
// through at most five roundings (conversion, product, two sums, the final
// difference), so |fl(d) - d| <= gamma_5 (|n_x p_x| + |n_y p_y| + |n_z p_z| +
// |off|) with gamma_5 = 5 eps / (1 - 5 eps), eps = 2^-24.  In terms of the
// computed magnitudes (each within a factor (1 - eps)^2 of the exact ones)
// the bound is below 5.0001 eps times their sum; 8 eps also covers the
// rounding of the sum and of the product that form the bound.
constexpr float kErr3 = 8.0f / 16777216.0f;

__device__ __forceinline__ int classify_point(const FacetRec *fac, int32_t gfirst, int32_t gcount,
                                              int32_t x, int32_t y, int32_t z, int mode,
                                              uint32_t &tests, uint32_t &falls) {
    for (int32_t g = 0; g < gcount; ++g) {
        const FacetRec &F = fac[gfirst + g];
        if (mode == 1) {
            const float fx = __fmul_rn((float)F.nx, (float)x);
            const float fy = __fmul_rn((float)F.ny, (float)y);
            const float fz = __fmul_rn((float)F.nz, (float)z);
            const float fo = (float)F.off;
            const float d = __fsub_rn(__fadd_rn(__fadd_rn(fx, fy), fz), fo);
            const float bnd = __fmul_rn(
                __fadd_rn(__fadd_rn(__fadd_rn(fabsf(fx), fabsf(fy)), fabsf(fz)), fabsf(fo)), kErr3);
            ++tests;
            if (d > bnd) return g;
            if (d < -bnd) continue;
            ++falls;
        }
        const int64_t d = F.nx * (int64_t)x + F.ny * (int64_t)y + F.nz * (int64_t)z - F.off;
        if (d > 0) return g;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// classify + count (PASS 1) / classify + scatter (PASS 2)
// ---------------------------------------------------------------------------
struct ClassArgs {
    const int32_t *ix, *iy, *iz;
    int32_t from_input;
    int32_t nsrc;
    Pool in, out;
    const SrcRec *src;
    const FacetRec *fac;
    uint32_t *counts;
    uint32_t *cursor;
    const int64_t *range;
    unsigned long long *filter_ctr;
    int32_t ntiles;
    int32_t mode;
};

template <int PASS>
__global__ __launch_bounds__(kBlock) void k3_classify(ClassArgs a) {
    __shared__ uint32_t lcnt[kGroupLds];
    __shared__ uint32_t lbase[kGroupLds];
    __shared__ uint32_t lfilt[2];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    uint32_t tests = 0, falls = 0;
    if (tid < 2) lfilt[tid] = 0;
    for (int32_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const int32_t s = find_range(a.src, a.nsrc, t);
        const SrcRec sr = a.src[s];
        const int32_t base = (t - sr.tile0) * kTile;
        const int32_t ng = sr.gcount;
        const int32_t nl = ng < kGroupLds ? ng : kGroupLds;
        for (int j = tid; j < nl; j += kBlock) lcnt[j] = 0;
        __syncthreads();
        int32_t px[kItems], py[kItems], pz[kItems], pi[kItems], tg[kItems];
        uint32_t rk[kItems];
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const int32_t pos = base + i * kBlock + tid;
            tg[i] = -1;
            rk[i] = 0;
            px[i] = py[i] = pz[i] = pi[i] = 0;
            if (pos < sr.len) {
                const int64_t g = sr.start + pos;
                if (a.from_input) {
                    px[i] = a.ix[g];
                    py[i] = a.iy[g];
                    pz[i] = a.iz[g];
                    pi[i] = (int32_t)g;
                } else {
                    px[i] = a.in.x[g];
                    py[i] = a.in.y[g];
                    pz[i] = a.in.z[g];
                    pi[i] = a.in.idx[g];
                }
                tg[i] = classify_point(a.fac, sr.gfirst, ng, px[i], py[i], pz[i], a.mode, tests,
                                       falls);
            }
            // rank among the block's points of the same target: one LDS
            // atomic per distinct target of the wave
            uint64_t pend = __ballot(tg[i] >= 0 && tg[i] < kGroupLds);
            while (pend) {
                const int leader = __builtin_ctzll(pend);
                const int lt = __builtin_amdgcn_readlane(tg[i], leader);
                const uint64_t m = __ballot(tg[i] == lt);
                uint32_t b = 0;
                if (lane == leader) b = atomicAdd(&lcnt[lt], (uint32_t)__popcll(m));
                b = (uint32_t)__builtin_amdgcn_readlane((int)b, leader);
                if (tg[i] == lt) rk[i] = b + (uint32_t)__popcll(m & lanemask_lt());
                pend &= ~m;
            }
            if (tg[i] >= kGroupLds) {
                if (PASS == 1) atomicAdd(&a.counts[sr.gfirst + tg[i]], 1u);
                else rk[i] = atomicAdd(&a.cursor[sr.gfirst + tg[i]], 1u);
            }
        }
        __syncthreads();
        for (int j = tid; j < nl; j += kBlock) {
            const uint32_t c = lcnt[j];
            if (c) {
                if (PASS == 1) atomicAdd(&a.counts[sr.gfirst + j], c);
                else lbase[j] = atomicAdd(&a.cursor[sr.gfirst + j], c);
            }
        }
        if (PASS == 2) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kItems; ++i) {
                if (tg[i] < 0) continue;
                const uint32_t slot = tg[i] < kGroupLds ? lbase[tg[i]] + rk[i] : rk[i];
                const int64_t dst = a.range[sr.gfirst + tg[i]] + slot;
                a.out.x[dst] = px[i];
                a.out.y[dst] = py[i];
                a.out.z[dst] = pz[i];
                a.out.idx[dst] = pi[i];
            }
        }
        __syncthreads();
    }
    if (a.mode == 1 && PASS == 1) {
        const uint32_t wt = (uint32_t)__builtin_amdgcn_readfirstlane(0) + 0;
        (void)wt;
        atomicAdd(&lfilt[0], tests);
        atomicAdd(&lfilt[1], falls);
        __syncthreads();
        if (tid == 0 && (lfilt[0] | lfilt[1])) {
            atomicAdd(&a.filter_ctr[0], (unsigned long long)lfilt[0]);
            atomicAdd(&a.filter_ctr[1], (unsigned long long)lfilt[1]);
        }
    }
}

hipError_t launch_classify(int pass, const int32_t *ix, const int32_t *iy, const int32_t *iz,
                           int from_input, Pool in, Pool out, const SrcRec *src, int32_t nsrc,
                           int32_t ntiles, const FacetRec *fac, uint32_t *counts,
                           uint32_t *cursor, const int64_t *range, int mode,
                           unsigned long long *filter_ctr, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    ClassArgs a;
    a.ix = ix;
    a.iy = iy;
    a.iz = iz;
    a.from_input = from_input;
    a.nsrc = nsrc;
    a.in = in;
    a.out = out;
    a.src = src;
    a.fac = fac;
    a.counts = counts;
    a.cursor = cursor;
    a.range = range;
    a.filter_ctr = filter_ctr;
    a.ntiles = ntiles;
    a.mode = mode;
    const int grid = ntiles < 65536 ? ntiles : 65536;
    if (pass == 1)
        hipLaunchKernelGGL(k3_classify<1>, dim3(grid), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL(k3_classify<2>, dim3(grid), dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// apex of every facet with outside points
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool akey_better(const ApexKey &a, const ApexKey &b) {
    if (a.idx < 0) return false;
    if (b.idx < 0) return true;
    if (a.d != b.d) return a.d > b.d;
    if (a.t1 != b.t1) return a.t1 < b.t1;
    if (a.t2 != b.t2) return a.t2 < b.t2;
    return a.idx < b.idx;
}

__device__ __forceinline__ void akey_take(ApexKey &dst, const ApexKey &s) {
    if (akey_better(s, dst)) {
        dst.d = s.d;
        dst.t1 = s.t1;
        dst.t2 = s.t2;
        dst.idx = s.idx;
        dst.x = s.x;
        dst.y = s.y;
        dst.z = s.z;
    }
}

__device__ __forceinline__ ApexKey akey_empty() {
    ApexKey e;
    e.d = e.t1 = e.t2 = 0;
    e.idx = -1;
    e.x = e.y = e.z = 0;
    e.pad = 0;
    return e;
}

__device__ __forceinline__ ApexKey akey_shfl(const ApexKey &k, int src) {
    ApexKey o;
    o.d = __shfl(k.d, src);
    o.t1 = __shfl(k.t1, src);
    o.t2 = __shfl(k.t2, src);
    o.idx = __shfl(k.idx, src);
    o.x = __shfl(k.x, src);
    o.y = __shfl(k.y, src);
    o.z = __shfl(k.z, src);
    o.pad = 0;
    return o;
}

__device__ __forceinline__ void wave_best(ApexKey &k) {
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const ApexKey o = akey_shfl(k, lane_id() ^ off);
        akey_take(k, o);
    }
}

__global__ __launch_bounds__(kBlock) void k3_apex_tiles(Pool pool, const SegRec *seg, const ScanTot *tot,
                                                        const FacetRec *fac, ApexKey *tile_keys) {
    __shared__ ApexKey lds[kBlock / kWave];
    const int32_t nseg = tot->nseg, ntiles = tot->ntiles;
    for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int32_t s = find_range(seg, nseg, t);
        const SegRec sg = seg[s];
        const FacetRec F = fac[sg.facet];
        const int32_t base = (t - sg.tile0) * kTile;
        ApexKey best = akey_empty();
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const int32_t pos = base + i * kBlock + threadIdx.x;
            if (pos >= sg.len) continue;
            const int64_t g = sg.start + pos;
            const int32_t x = pool.x[g], y = pool.y[g], z = pool.z[g];
            const int64_t rx = x - F.ax, ry = y - F.ay, rz = z - F.az;
            ApexKey k;
            k.d = F.nx * (int64_t)x + F.ny * (int64_t)y + F.nz * (int64_t)z - F.off;
            k.t1 = rx * F.ebx + ry * F.eby + rz * F.ebz;
            k.t2 = rx * F.ecx + ry * F.ecy + rz * F.ecz;
            k.idx = pool.idx[g];
            k.x = x;
            k.y = y;
            k.z = z;
            k.pad = 0;
            akey_take(best, k);
        }
        wave_best(best);
        const int w = threadIdx.x / kWave;
        if (lane_id() == 0) lds[w] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            ApexKey b = lds[0];
            for (int j = 1; j < kBlock / kWave; ++j) akey_take(b, lds[j]);
            tile_keys[t] = b;
        }
        __syncthreads();
    }
}

// one wave per facet: the best of its tiles
__global__ __launch_bounds__(kBlock) void k3_apex_merge(const SegRec *seg, const ScanTot *tot,
                                                        const ApexKey *tile_keys,
                                                        ApexKey *seg_keys) {
    const int32_t s = (int32_t)((blockIdx.x * kBlock + threadIdx.x) / kWave);
    if (s >= tot->nseg) return;
    const SegRec sg = seg[s];
    const int32_t nt = (sg.len + kTile - 1) / kTile;
    ApexKey best = akey_empty();
    for (int32_t j = lane_id(); j < nt; j += kWave) akey_take(best, tile_keys[sg.tile0 + j]);
    wave_best(best);
    if (lane_id() == 0) seg_keys[s] = best;
}

hipError_t launch_apex(Pool pool, const SegRec *seg, int32_t nseg_max, int32_t ntiles_max,
                       const ScanTot *tot, const FacetRec *fac, ApexKey *tile_keys,
                       ApexKey *seg_keys, hipStream_t st) {
    if (nseg_max <= 0 || ntiles_max <= 0) return hipSuccess;
    const int grid = ntiles_max < 65536 ? ntiles_max : 65536;
    hipLaunchKernelGGL(k3_apex_tiles, dim3(grid), dim3(kBlock), 0, st, pool, seg, tot, fac, tile_keys);
    const int gm = (int)(((int64_t)nseg_max * kWave + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k3_apex_merge, dim3(gm), dim3(kBlock), 0, st, seg, tot, tile_keys, seg_keys);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// outside-set ranges of the new facets: an exclusive scan of pass 1's counts
// ---------------------------------------------------------------------------
// The compact step of the flagPermute (Sections 4.1-4.2): facet j's points go
// to [top + P_j, top + P_j + c_j), P_j the count of the facets before it, and
// the facets with points are listed in facet order for the apex step, each
// with the first of its tiles.  Three launches and no host wait: per-chunk
// sums, their scan in one block, each chunk's own scan.  A thread owns eight
// consecutive facets of a chunk.
__device__ __forceinline__ void scan_vals(const uint32_t *counts, int32_t nf, int32_t j0, uint32_t (&c)[8],
                                          uint32_t (&sum)[3]) {
    sum[0] = sum[1] = sum[2] = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        c[i] = j0 + i < nf ? counts[j0 + i] : 0u;
        sum[0] += c[i];
        sum[1] += c[i] ? 1u : 0u;
        sum[2] += (c[i] + kTile - 1) / kTile;
    }
}

__global__ __launch_bounds__(kBlock) void k3_scan_part(const uint32_t *counts, int32_t nf, uint32_t *part) {
    __shared__ uint32_t scratch[3 * (kBlock / kWave)];
    uint32_t c[8], v[3], tot[3];
    scan_vals(counts, nf, blockIdx.x * kScanChunk + threadIdx.x * 8, c, v);
    qh::block_excl_scan<kBlock, 3>(v, tot, scratch);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = tot[0];
        part[3 * blockIdx.x + 1] = tot[1];
        part[3 * blockIdx.x + 2] = tot[2];
    }
}

// one block: the chunk sums become exclusive prefixes (each thread a run of
// consecutive chunks)
__global__ __launch_bounds__(kBlock) void k3_scan_top(uint32_t *part, int32_t nchunk, ScanTot *out) {
    __shared__ uint32_t scratch[3 * (kBlock / kWave)];
    const int32_t per = (nchunk + kBlock - 1) / kBlock;
    const int32_t c0 = min(nchunk, (int32_t)threadIdx.x * per), c1 = min(nchunk, c0 + per);
    uint32_t v[3] = {0, 0, 0}, tot[3];
    for (int32_t c = c0; c < c1; ++c) {
        v[0] += part[3 * c + 0];
        v[1] += part[3 * c + 1];
        v[2] += part[3 * c + 2];
    }
    qh::block_excl_scan<kBlock, 3>(v, tot, scratch);
    for (int32_t c = c0; c < c1; ++c) {
        const uint32_t a0 = part[3 * c + 0], a1 = part[3 * c + 1], a2 = part[3 * c + 2];
        part[3 * c + 0] = v[0];
        part[3 * c + 1] = v[1];
        part[3 * c + 2] = v[2];
        v[0] += a0;
        v[1] += a1;
        v[2] += a2;
    }
    if (threadIdx.x == 0) {
        out->written = (int64_t)tot[0];
        out->nseg = (int32_t)tot[1];
        out->ntiles = (int32_t)tot[2];
    }
}

__global__ __launch_bounds__(kBlock) void k3_scan_apply(const uint32_t *counts, int32_t nf, int64_t top,
                                                        const uint32_t *part, int64_t *range, SegRec *seg,
                                                        uint32_t *cursor) {
    __shared__ uint32_t scratch[3 * (kBlock / kWave)];
    const int32_t j0 = blockIdx.x * kScanChunk + threadIdx.x * 8;
    uint32_t c[8], v[3], tot[3];
    scan_vals(counts, nf, j0, c, v);
    qh::block_excl_scan<kBlock, 3>(v, tot, scratch);
    int64_t at = top + (int64_t)part[3 * blockIdx.x + 0] + v[0];
    int32_t q = (int32_t)(part[3 * blockIdx.x + 1] + v[1]);
    int32_t tl = (int32_t)(part[3 * blockIdx.x + 2] + v[2]);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if (j0 + i >= nf) break;
        range[j0 + i] = at;
        cursor[j0 + i] = 0;  // pass 2's per-facet write positions start at 0
        if (c[i]) {
            SegRec sg;
            sg.start = at;
            sg.len = (int32_t)c[i];
            sg.facet = j0 + i;
            sg.tile0 = tl;
            sg.pad = 0;
            seg[q++] = sg;
            tl += (int32_t)((c[i] + kTile - 1) / kTile);
        }
        at += c[i];
    }
}

hipError_t launch_scan(const uint32_t *counts, int32_t nf, int64_t top, int64_t *range, SegRec *seg,
                       uint32_t *cursor, uint32_t *part, ScanTot *tot, hipStream_t st) {
    const int32_t nchunk = (nf + kScanChunk - 1) / kScanChunk;
    if (nchunk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k3_scan_part, dim3(nchunk), dim3(kBlock), 0, st, counts, nf, part);
    hipLaunchKernelGGL(k3_scan_top, dim3(1), dim3(kBlock), 0, st, part, nchunk, tot);
    hipLaunchKernelGGL(k3_scan_apply, dim3(nchunk), dim3(kBlock), 0, st, counts, nf, top, part, range, seg,
                       cursor);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pool compaction: copy live ranges
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k3_gather(Pool in, Pool out, const SegRec *seg,
                                                    int32_t nseg, int32_t ntiles,
                                                    const int64_t *dst) {
    for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int32_t s = find_range(seg, nseg, t);
        const SegRec sg = seg[s];
        const int32_t base = (t - sg.tile0) * kTile;
        const int64_t d0 = dst[s];
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const int32_t pos = base + i * kBlock + threadIdx.x;
            if (pos >= sg.len) continue;
            const int64_t g = sg.start + pos;
            out.x[d0 + pos] = in.x[g];
            out.y[d0 + pos] = in.y[g];
            out.z[d0 + pos] = in.z[g];
            out.idx[d0 + pos] = in.idx[g];
        }
    }
}

hipError_t launch_gather(Pool in, Pool out, const SegRec *seg, int32_t nseg, int32_t ntiles,
                         const int64_t *dst, hipStream_t st) {
    if (nseg <= 0 || ntiles <= 0) return hipSuccess;
    const int grid = ntiles < 65536 ? ntiles : 65536;
    hipLaunchKernelGGL(k3_gather, dim3(grid), dim3(kBlock), 0, st, in, out, seg, nseg, ntiles, dst);
    return hipGetLastError();
}

}  // namespace qh3
