// qh_api.hip -- the C ABI of include/qh.h: workspace context and the host
// driver of a call.
//
// A call enqueues the set-up and extremes kernels, the first split, and then
// Quickhull rounds in batches (two launches per round).  Every kernel reads the
// round state from device memory and does nothing once no segment is left,
// so a batch may overshoot the last round; the host reads the small control
// block back once per batch instead of once per round, which is what the
// paper's GPU loop paid for (Section 5).  Back-to-back launches were chosen
// over a persistent kernel with grid barriers: on MI355X a grid-wide barrier
// (with the cross-XCD fences it needs) costs tens of microseconds, a
// dependent launch a few.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "../../include/qh.h"
#include "qh2d.h"
#include "qh_ctx.h"

using namespace qh;

namespace qh {
hipError_t fill_single_offsets(int64_t *off, int64_t n, hipStream_t st);
}

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Carve {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t count) {
        off = align_up(off, 256);
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += count * sizeof(T);
        return p;
    }
};

// Lay the whole workspace out in one allocation (base == nullptr: size only).
size_t carve(qh_ctx *c, char *base) {
    Carve cv{base};
    Ws2 &w = c->ws;
    w.ctl = cv.take<Control>(1);
    w.pts_ = cv.take<int32_t>((size_t)12 * c->cap_pts);
    w.geo_ = cv.take<SegGeo>((size_t)4 * c->scap);
    w.top_ = cv.take<SegTop>((size_t)4 * c->scap);
    w.tinfo_ = cv.take<TileInfo>((size_t)4 * c->tcap);
    w.adir = cv.take<Best>(4 * (size_t)c->scap);
    w.recF = cv.take<Best>(2 * (size_t)c->tcap);
    w.recL = cv.take<Best>(2 * (size_t)c->tcap);
    w.tcnt_ = cv.take<uint32_t>((size_t)2 * c->tcap);
    w.pv_ = cv.take<int32_t>((size_t)4 * (c->tcap + 2));
    w.pp_ = cv.take<int32_t>((size_t)4 * (c->tcap + 2));
    w.kf_ = cv.take<int32_t>((size_t)4 * (c->tcap + 2));
    w.ml_ = cv.take<int32_t>((size_t)2 * c->tcap);
    w.st5_ = cv.take<uint64_t>((size_t)2 * c->s5cap);
    w.st5b_ = cv.take<uint64_t>((size_t)2 * c->s5cap);
    w.st4_ = cv.take<uint64_t>((size_t)2 * c->s4cap);
    w.st4b_ = cv.take<uint64_t>((size_t)2 * c->s4cap);
    w.recF0 = cv.take<Best>(2 * (size_t)c->tcap);
    w.recL0 = cv.take<Best>(2 * (size_t)c->tcap);
    w.dir0 = cv.take<Best>(2 * (size_t)c->kcap);
    w.inst_rank = cv.take<int32_t>(c->kcap);
    w.V = cv.take<int32_t>(c->hcap);
    w.hinst = cv.take<int32_t>(c->hcap);
    w.nxt = cv.take<int32_t>(c->hcap);
    w.succ_ = cv.take<int32_t>((size_t)2 * c->hcap);
    w.dist_ = cv.take<int32_t>((size_t)2 * c->hcap);
    w.cap_pts = c->cap_pts;
    w.scap = c->scap;
    w.hcap = c->hcap;
    w.tcap = c->tcap;
    w.s4cap = c->s4cap;
    w.s5cap = c->s5cap;
    return align_up(cv.off, 256);
}

qh_status ensure(qh_ctx *c, int64_t n, int32_t k) {
    // a round writes the survivors of tile t at t * kTile of each region, and a
    // round has at most n / kTile + 2 tiles (two regions with a ragged tail),
    // except the round after the split, whose two regions are both the input
    // (twice n / kTile + 1 tiles, written to the slots of the input tiles)
    const int64_t cap_pts = (std::max<int64_t>(1, (n + kTile - 1) / kTile) + 2) * kTile;
    const int32_t tcap = (int32_t)(2 * (cap_pts / kTile) + 2);
    const int32_t s5cap = (int32_t)(tcap / (kSegBlock * kPieceItems) + 8);
    const int64_t smax = n + k + 16;
    int64_t scap = std::max<int64_t>({4096, n / 16 + 2 * (int64_t)k + 1024, c->want_scap});
    scap = std::min(scap, std::max<int64_t>(smax, 4096));
    int64_t hcap = std::max<int64_t>({(int64_t)2 * k + 4096, n / 16 + 2 * (int64_t)k + 1024,
                                      c->want_hcap});
    // (every point can be a vertex; every instance also takes an id for its
    // minimum, one for its first split and two for the split's children,
    // which an instance with points on one side only leaves unused)
    hcap = std::min(hcap, std::max<int64_t>(4 * (int64_t)k + n + 16, 4096));
    const int32_t kcap = std::max(k, 1);
    const int32_t s4cap = (int32_t)(2 * ((2 * scap + kSegBlock - 1) / kSegBlock) + 8);
    if (c->dmem && cap_pts <= c->cap_pts && scap <= c->scap && hcap <= c->hcap && tcap <= c->tcap &&
        kcap <= c->kcap && s5cap <= c->s5cap)
        return QH_OK;
    if (c->dmem) {
        (void)hipFree(c->dmem);
        c->dmem = nullptr;
    }
    c->cap_pts = std::max(cap_pts, c->cap_pts);
    c->tcap = std::max(tcap, c->tcap);
    c->scap = std::max((int32_t)scap, c->scap);
    c->hcap = std::max((int32_t)hcap, c->hcap);
    c->kcap = std::max(kcap, c->kcap);
    c->s4cap = std::max(s4cap, c->s4cap);
    c->s5cap = std::max(s5cap, c->s5cap);
    const size_t bytes = carve(c, nullptr);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        c->cap_pts = 0;
        c->scap = c->hcap = c->tcap = c->kcap = c->s4cap = c->s5cap = 0;
        return QH_ENOMEM;
    }
    c->dmem = p;
    c->dbytes = bytes;
    carve(c, static_cast<char *>(p));
    return QH_OK;
}

}  // namespace

namespace qhi {

qh_status ctx_init(qh_ctx *c) {
    if (hipGetDevice(&c->device) != hipSuccess) return QH_EDEVICE;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess &&
        cus > 0)
        c->cus = cus;
    for (int m = 0; m < 2; ++m) {
        int g[3];
        if (round_grids(m, c->cus, g) != hipSuccess) return QH_EDEVICE;
        c->grid_pre[m][0] = g[0];
        c->grid_pre[m][1] = g[1];
        c->grid[m] = g[2];
        if (g[0] <= 0 || g[1] <= 0 || g[2] <= 0) return QH_EDEVICE;
    }
    if (extremes_grid(c->cus, &c->grid_ext) != hipSuccess || c->grid_ext <= 0) return QH_EDEVICE;
    if (hipHostMalloc((void **)&c->ctl_host, sizeof(Control), hipHostMallocDefault) != hipSuccess)
        return QH_ENOMEM;
    if (hipHostMalloc((void **)&c->h_host, sizeof(int64_t) * 2, hipHostMallocDefault) != hipSuccess)
        return QH_ENOMEM;
    if (hipMalloc((void **)&c->single_off, sizeof(int64_t) * 2) != hipSuccess) return QH_ENOMEM;
    if (hipMalloc((void **)&c->single_hoff, sizeof(int64_t) * 2) != hipSuccess) return QH_ENOMEM;

    return QH_OK;
}

void drop_graphs(qh_ctx *c) {
    for (QhGraph &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
    c->gkey.clear();
}

void ctx_free(qh_ctx *c) {
    if (!c) return;
    drop_graphs(c);
    if (c->digest) (void)hipFree(c->digest);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    if (c->dmem) (void)hipFree(c->dmem);
    if (c->single_off) (void)hipFree(c->single_off);
    if (c->single_hoff) (void)hipFree(c->single_hoff);

    if (c->ctl_host) (void)hipHostFree(c->ctl_host);
    if (c->h_host) (void)hipHostFree(c->h_host);
    ctx3_free(c->c3);
    delete c;
}

}  // namespace qhi

namespace {

using qhi::ctx_free;
using qhi::drop_graphs;
using qhi::ctx_init;

#define QH_TRY(expr)                                  \
    do {                                              \
        if ((expr) != hipSuccess) {                   \
            (void)hipGetLastError();                  \
            return QH_EDEVICE;                        \
        }                                             \
    } while (0)



// HIP events around launches (QH_FLAG_TIMING), summed per kind of kernel
struct Timing {
    enum Kind { kSetup = 0, kExtremes, kSplit, kRound, kSegments, kOutput, kKinds };
    qh_ctx *c;
    bool on;
    std::vector<int> kind;
    hipError_t before(hipStream_t st, int k) {
        if (!on) return hipSuccess;
        const size_t i = kind.size() * 2;
        while (c->ev.size() < i + 2) {
            hipEvent_t e;
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return err;
            c->ev.push_back(e);
        }
        kind.push_back(k);
        return hipEventRecord(c->ev[i], st);
    }
    hipError_t after(hipStream_t st) {
        if (!on) return hipSuccess;
        return hipEventRecord(c->ev[kind.size() * 2 - 1], st);
    }
    void totals(double (&ms)[kKinds]) {
        for (double &m : ms) m = 0;
        for (size_t j = 0; j < kind.size(); ++j) {
            float t = 0;
            if (hipEventElapsedTime(&t, c->ev[2 * j], c->ev[2 * j + 1]) == hipSuccess) ms[kind[j]] += t;
        }
    }
};

// The bytes a cached graph depends on: every kernel argument and the stream.
template <typename T>
void key_add(std::vector<unsigned char> &key, const T &v) {
    const unsigned char *b = reinterpret_cast<const unsigned char *>(&v);
    key.insert(key.end(), b, b + sizeof(T));
}

qh_status run2d(qh_ctx *c, const int32_t *pts, int64_t n, const int64_t *offsets, int32_t k,
                int32_t *hull_idx, int64_t *hull_offsets, int64_t *h_total, int64_t *single_off,
                const qh_opts *o, const QhLaunch &cfg, int64_t tuned_configs) {
    hipStream_t st = o ? (hipStream_t)o->stream : nullptr;
    const int mode = o ? (int)o->mode : 0;
    const bool timing = o && (o->flags & QH_FLAG_TIMING);
    const bool graph = o && (o->flags & QH_FLAG_GRAPH) && !timing;
    qh_stats *stats = o ? o->stats : nullptr;
    if (stats) memset(stats, 0, sizeof(*stats));
    if (h_total) *h_total = 0;
    if (mode != QH_EXACT_INT64 && mode != QH_FP32_FILTER) return QH_EINVAL;
    int64_t graph_launches = 0;

    HullArgs args = {};
    args.x = pts;
    args.y = pts + n;
    args.offsets = offsets;
    args.hull_idx = hull_idx;
    args.hull_offsets = hull_offsets;
    args.n = (int32_t)n;
    args.k = k;
    args.vec_ok = ((uintptr_t)pts & 3u) == 0 ? 1 : 0;
    args.fin_cap = (o && (o->flags & QH_FLAG_NO_FINISH)) ? 0 : kFinCap;
    args.fin_segs = cfg.fin_segs;
    // a call of the same shape as the last one starts the finishing kernel
    // where that call finished; any other call from round 0
    args.fin_from = (c->fin_hint_n == n && c->fin_hint_k == k && c->fin_hint_mode == mode) ? c->fin_hint : 0;
    const int grid = cfg.grid;
    // the finishing kernel: at most its resident count of workgroups (two per
    // CU), each finishing segments, or runs of small segments, one after the
    // other
    const int grid_fin = std::max(1, std::min(cfg.fin_segs, 2 * c->cus));
    args.fin_pts = args.fin_cap > 0 ? kFinUnitsPerBlock * kFinUnit * grid_fin : 0;
    // the split and the round after it at their own residency, scaled like
    // the round kernel's grid
    args.grid_split = (int32_t)std::max<int64_t>(1, (int64_t)c->grid_pre[mode][0] * grid / std::max(1, c->grid[mode]));
    args.grid_ro1 = (int32_t)std::max<int64_t>(1, (int64_t)c->grid_pre[mode][1] * grid / std::max(1, c->grid[mode]));
    int64_t syncs = 0;
    int r = 0;
    Timing tm{c, timing, {}};

    for (int attempt = 0;; ++attempt) {
        qh_status s = ensure(c, n, k);
        if (s != QH_OK) return s;
        const Ws2 &ws = c->ws;
        // few blocks: most rounds have few segment tiles, and every idle block
        // still costs two claims on the shared counters
        const int grid_seg = std::max(1, std::min((2 * c->scap + kSegBlock - 1) / kSegBlock, c->cus / 2));
        tm.kind.clear();
        // the launches of a batch: with prefix, the set-up and extremes first
        auto enqueue = [&](bool prefix, int r0, int len) -> hipError_t {
            hipError_t e = hipSuccess;
            auto ok = [&e](hipError_t x) { return (e = x) == hipSuccess; };
            if (prefix) {
                if (single_off && !ok(fill_single_offsets(single_off, n, st))) return e;
                if (!ok(tm.before(st, Timing::kSetup)) || !ok(launch_setup(ws, args, grid, st)) ||
                    !ok(tm.after(st)))
                    return e;
                if (!ok(tm.before(st, Timing::kExtremes)) || !ok(launch_extremes(ws, args, c->grid_ext, st)) ||
                    !ok(tm.after(st)))
                    return e;
            }
            for (int rr = r0; rr < r0 + len; ++rr) {
                if (!ok(tm.before(st, rr == 0 ? Timing::kSplit : Timing::kRound)) ||
                    !ok(launch_round(ws, args, mode, rr, grid, cfg.grid_multi, grid_fin, st)) || !ok(tm.after(st)))
                    return e;
                if (!ok(tm.before(st, Timing::kSegments)) || !ok(launch_segments(ws, args, rr, grid_seg, st)) ||
                    !ok(tm.after(st)))
                    return e;
            }
            return e;
        };
        // the same batch from a graph the context captured with the same
        // arguments (captured now if there is none)
        auto run_batch = [&](bool prefix, int r0, int len) -> hipError_t {
            if (!graph) return enqueue(prefix, r0, len);
            for (const QhGraph &g : c->graphs)
                if (g.prefix == (int)prefix && g.r0 == r0 && g.len == len) {
                    ++graph_launches;
                    return hipGraphLaunch(g.exec, st);
                }
            hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return e;
            e = enqueue(prefix, r0, len);
            hipGraph_t gr = nullptr;
            const hipError_t e2 = hipStreamEndCapture(st, &gr);
            if (e == hipSuccess) e = e2;
            hipGraphExec_t ex = nullptr;
            if (e == hipSuccess) e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
            if (gr) (void)hipGraphDestroy(gr);
            if (e != hipSuccess) return e;
            c->graphs.push_back({(int)prefix, r0, len, ex});
            ++graph_launches;
            return hipGraphLaunch(ex, st);
        };
        if (graph) {
            std::vector<unsigned char> key;
            key_add(key, args);
            key_add(key, ws);
            key_add(key, cfg);
            key_add(key, mode);
            key_add(key, grid_seg);
            key_add(key, st);
            key_add(key, single_off);
            if (key != c->gkey) {
                drop_graphs(c);
                c->gkey = key;
            }
        }
        r = 0;
        // the first batch: as many rounds as the previous call of this context
        // needed (no launches left over when the inputs are alike), else the
        // first split and 4 rounds; then 8 rounds per batch
        int batch = c->hint_rounds > 0 ? c->hint_rounds : 5;
        bool prefix = true;
        while (true) {
            QH_TRY(run_batch(prefix, r, batch));
            prefix = false;
            r += batch;
            QH_TRY(hipMemcpyAsync(c->ctl_host, ws.ctl, sizeof(Control), hipMemcpyDeviceToHost, st));
            QH_TRY(hipStreamSynchronize(st));
            ++syncs;
            const Control &hc = *c->ctl_host;
            if (hc.error) break;
            const RoundState &rs = hc.rs[r & 1];
            if (rs.s[0] + rs.s[1] == 0) break;
            batch = 8;
        }
        const int err = c->ctl_host->error;
        if (err & kErrOffsets) return QH_EINVAL;
        if (err & kErrRange) return QH_ERANGE;
        if (err & (kErrSegCap | kErrHullCap)) {
            if (attempt >= 8) return QH_ECAPACITY;
            if (err & kErrSegCap)
                c->want_scap = (int32_t)std::min<int64_t>((int64_t)c->scap * 4, INT32_MAX / 2);
            if (err & kErrHullCap)
                c->want_hcap = (int32_t)std::min<int64_t>((int64_t)c->hcap * 4, INT32_MAX / 2);
            continue;
        }
        if (err) return QH_EDEVICE;
        break;
    }
    const int32_t H = c->ctl_host->rs[r & 1].hbase;
    {
        const Control &hc = *c->ctl_host;
        const int need = hc.fin_round >= 0 ? hc.fin_round + 1 : (int)hc.rounds_with_work;
        c->hint_rounds = std::max(1, std::min(need, 64));
        c->fin_hint = hc.fin_round >= 0 ? hc.fin_round : 0;
        c->fin_hint_n = n;
        c->fin_hint_k = k;
        c->fin_hint_mode = mode;
    }
    QH_TRY(tm.before(st, Timing::kOutput));
    QH_TRY(launch_output(c->ws, args, H, st));
    QH_TRY(tm.after(st));
    QH_TRY(hipMemcpyAsync(c->ctl_host, c->ws.ctl, sizeof(Control), hipMemcpyDeviceToHost, st));
    QH_TRY(hipStreamSynchronize(st));
    ++syncs;
    const Control &h = *c->ctl_host;
    if (h.error) return QH_EDEVICE;
    if (h_total) *h_total = h.h_total;
    if (stats) {
        stats->rounds = (int64_t)h.rounds_with_work;
        stats->round_launches = r;
        stats->round_points_in = (int64_t)(h.second_in + h.points_in);
        stats->round_points_out = (int64_t)(h.second_out + h.points_out);
        stats->split_points_out = (int64_t)h.first_out;
        // the split reads 8 B per point and writes nothing; the round after it
        // reads the input again (8 B per point: the index is the position)
        // and writes 12 B per survivor; later rounds read and write 12 B
        const int64_t split_bytes = (int64_t)(8 * h.first_in);
        const int64_t later = (int64_t)(8 * h.second_in + 12 * h.second_out + 12 * h.points_in +
                                        12 * h.points_out);
        stats->round_kernel_bytes = split_bytes + later;
        stats->hull_bytes = 8 * n + split_bytes + later;
        if (timing) {
            double ms[Timing::kKinds];
            tm.totals(ms);
            stats->kernel_ms = ms[0] + ms[1] + ms[2] + ms[3] + ms[4] + ms[5];
            stats->round_kernel_ms = ms[Timing::kSplit] + ms[Timing::kRound];
            stats->split_ms = ms[Timing::kSplit];
            stats->extremes_ms = ms[Timing::kExtremes];
            stats->segment_ms = ms[Timing::kSegments];
        }
        unsigned long long fs[3] = {0, 0, 0};
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < kAccSlots; ++i) fs[j] += h.fstat[j][i];
        stats->filter_tests = (int64_t)fs[0];
        stats->filter_fallbacks = (int64_t)fs[1];
        stats->argmax_candidates = (int64_t)fs[2];
        stats->max_segments = h.max_segments;
        stats->grid_blocks = grid;
        stats->host_syncs = syncs;
        stats->finish_round = h.fin_round;
        stats->finish_runs = h.fin_round >= 0 ? h.fin_runs : 0;
        stats->multi_blocks = cfg.grid_multi;
        stats->finish_segments = args.fin_cap > 0 ? cfg.fin_segs : 0;
        stats->graph_launches = graph_launches;
        stats->tuned_configs = tuned_configs;
    }
    return QH_OK;
}

// An order-independent digest of a call's outputs (the hull indices and the
// hull offsets, each entry mixed with its position by SplitMix64's output
// function, Steele, Lea and Flood 2014, and summed): the autotuner checks
// that every configuration it times gives the same output.
__device__ __forceinline__ uint64_t out_mix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_out_digest(const int32_t *idx, int64_t h, const int64_t *hoff, int32_t k,
                                                    unsigned long long *acc) {
    __shared__ unsigned long long part[256 / kWave];
    unsigned long long v = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < h; i += (int64_t)gridDim.x * 256)
        v += out_mix(((uint64_t)i << 32) ^ (uint32_t)idx[i]);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i <= k; i += (int64_t)gridDim.x * 256)
        v += out_mix(~(((uint64_t)i << 40) ^ (uint64_t)hoff[i]));
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane_id() == 0) part[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < 256 / kWave; ++w) t += part[w];
        atomicAdd(acc, t);
    }
}

// the digest of the outputs of the last call (h hull entries, k + 1 offsets)
qh_status out_digest(qh_ctx *c, hipStream_t st, const int32_t *idx, int64_t h, const int64_t *hoff, int32_t k,
                     unsigned long long *out) {
    if (!c->digest && hipMalloc((void **)&c->digest, sizeof(unsigned long long)) != hipSuccess) {
        (void)hipGetLastError();
        c->digest = nullptr;
        return QH_ENOMEM;
    }
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(c->cus, (std::max<int64_t>(h, k + 1) + 255) / 256));
    if (hipMemsetAsync(c->digest, 0, sizeof(unsigned long long), st) != hipSuccess) return QH_EDEVICE;
    hipLaunchKernelGGL(k_out_digest, dim3(grid), dim3(256), 0, st, idx, h, hoff, k, c->digest);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(c->ctl_host, c->digest, sizeof(unsigned long long), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        return QH_EDEVICE;
    }
    memcpy(out, c->ctl_host, sizeof(unsigned long long));
    return QH_OK;
}

// The size class of a call: mode, and the point and instance counts rounded
// up to powers of two.
uint64_t size_class(int mode, int64_t n, int32_t k) {
    uint64_t ln = 0, lk = 0;
    while ((1ll << ln) < n) ++ln;
    while ((1ll << lk) < k) ++lk;
    return (uint64_t)mode | (ln << 8) | (lk << 16);
}

// A call with the context's launch configuration for its size class
// (QH_FLAG_AUTOTUNE), else the default one: the resident blocks of the round
// kernel, two blocks per CU for the multi-segment kernel and two segments
// per block of it for finishing.
qh_status run2d_tuned(qh_ctx *c, const int32_t *pts, int64_t n, const int64_t *offsets, int32_t k,
                      int32_t *hull_idx, int64_t *hull_offsets, int64_t *h_total,
                      int64_t *single_off, const qh_opts *o) {
    const int mode = o ? (int)o->mode : 0;
    if (mode != QH_EXACT_INT64 && mode != QH_FP32_FILTER) return QH_EINVAL;
    if (o && (o->flags & QH_FLAG_GRAPH) && !o->stream) return QH_EINVAL;
    const QhLaunch dflt = {c->grid[mode], 4 * c->cus, 16 * c->cus};
    if (!o || !(o->flags & QH_FLAG_AUTOTUNE))
        return run2d(c, pts, n, offsets, k, hull_idx, hull_offsets, h_total, single_off, o, dflt, 0);
    const uint64_t key = size_class(mode, n, k);
    for (const QhTuned &t : c->tuned)
        if (t.key == key)
            return run2d(c, pts, n, offsets, k, hull_idx, hull_offsets, h_total, single_off, o, t.cfg, 0);
    // time every candidate (the better of two calls) and keep the fastest;
    // every candidate must give the first one's output (checked by digest)
    hipStream_t st = (hipStream_t)o->stream;
    unsigned long long ref = 0;
    int64_t ref_h = -1;
    qh_opts quiet = *o;
    quiet.flags &= ~(uint32_t)(QH_FLAG_AUTOTUNE | QH_FLAG_TIMING | QH_FLAG_GRAPH);
    quiet.stats = nullptr;
    QhLaunch pick = dflt;
    double best = 1e300;
    int64_t tried = 0;
    for (int gm = 1; gm <= 2; ++gm)
        for (int mm = 2; mm <= 4; mm += 2)
            for (int fp = 1; fp <= 4; fp *= 2) {
                const QhLaunch cand = {c->grid[mode] * gm, mm * c->cus, fp * 4 * c->cus};
                for (int rep = 0; rep < 2; ++rep) {
                    const auto t0 = std::chrono::steady_clock::now();
                    qh_status s = run2d(c, pts, n, offsets, k, hull_idx, hull_offsets, h_total, single_off,
                                        &quiet, cand, 0);
                    const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                    if (s != QH_OK) return s;
                    if (t < best) {
                        best = t;
                        pick = cand;
                    }
                }
                const int64_t h = h_total ? *h_total : 0;
                unsigned long long dg = 0;
                qh_status s = out_digest(c, st, hull_idx, h, hull_offsets, k, &dg);
                if (s != QH_OK) return s;
                if (ref_h < 0) {
                    ref = dg;
                    ref_h = h;
                } else if (dg != ref || h != ref_h) {
                    return QH_EDEVICE;  // a launch configuration changed the output
                }
                ++tried;
            }
    c->tuned.push_back({key, pick});
    return run2d(c, pts, n, offsets, k, hull_idx, hull_offsets, h_total, single_off, o, pick, tried);
}

}  // namespace

namespace qhi {

qh_status get_ctx(const qh_opts *o, TempCtx &t) {
    if (o && o->ctx) {
        t.c = o->ctx;
        return QH_OK;
    }
    qh_ctx *c = new (std::nothrow) qh_ctx();
    if (!c) return QH_ENOMEM;
    t.c = c;
    t.owned = true;
    return ctx_init(c);
}

}  // namespace qhi

using qhi::TempCtx;
using qhi::get_ctx;

extern "C" {

qh_status qh_ctx_create(qh_ctx **out) {
    if (!out) return QH_EINVAL;
    *out = nullptr;
    qh_ctx *c = new (std::nothrow) qh_ctx();
    if (!c) return QH_ENOMEM;
    qh_status s = ctx_init(c);
    if (s != QH_OK) {
        ctx_free(c);
        return s;
    }
    *out = c;
    return QH_OK;
}

void qh_ctx_destroy(qh_ctx *ctx) { ctx_free(ctx); }

const char *qh_status_str(int status) {
    switch (status) {
        case QH_OK: return "ok";
        case QH_EINVAL: return "invalid argument";
        case QH_ERANGE: return "coordinate out of the exact range";
        case QH_ENOMEM: return "out of memory";
        case QH_EDEGENERATE: return "degenerate input";
        case QH_EDEVICE: return "HIP runtime error";
        case QH_ECAPACITY: return "internal capacity exceeded";
        default: return "unknown status";
    }
}

const char *qh_version(void) { return "qh 0.1 (gfx950)"; }

qh_status qh_hull2d(const int32_t *pts, int64_t n, int32_t *hull_idx, int64_t *h, const qh_opts *opts) {
    if (h) *h = 0;
    if (!h || n < 0 || n > (int64_t)INT32_MAX - 65536) return QH_EINVAL;
    if (n > 0 && (!pts || !hull_idx)) return QH_EINVAL;
    if (opts && (opts->flags & QH_FLAG_GRAPH) && !opts->stream) return QH_EINVAL;
    if (opts && opts->stats) memset(opts->stats, 0, sizeof(qh_stats));
    if (n == 0) return QH_OK;
    TempCtx t;
    qh_status s = get_ctx(opts, t);
    if (s != QH_OK) return s;
    int64_t ht = 0;
    s = run2d_tuned(t.c, pts, n, t.c->single_off, 1, hull_idx, t.c->single_hoff, &ht, t.c->single_off, opts);
    if (s != QH_OK) return s;
    *h = ht;
    return QH_OK;
}

qh_status qh_hull2d_batched(const int32_t *pts, int64_t n_total, const int64_t *offsets, int32_t k,
                            int32_t *hull_idx, int64_t *hull_offsets, int64_t *h_total,
                            const qh_opts *opts) {
    if (h_total) *h_total = 0;
    if (k < 1 || k > (1 << 24) || n_total < 0 || n_total > (int64_t)INT32_MAX - 65536) return QH_EINVAL;
    if (!offsets || !hull_offsets || (n_total > 0 && (!pts || !hull_idx))) return QH_EINVAL;
    if (opts && (opts->flags & QH_FLAG_GRAPH) && !opts->stream) return QH_EINVAL;
    if (opts && opts->stats) memset(opts->stats, 0, sizeof(qh_stats));
    TempCtx t;
    qh_status s = get_ctx(opts, t);
    if (s != QH_OK) return s;
    return run2d_tuned(t.c, pts, n_total, offsets, k, hull_idx, hull_offsets, h_total, nullptr, opts);
}

}  // extern "C"
