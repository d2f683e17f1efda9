// qh3d_host.hip -- the host driver of the 3D Quickhull (qh_hull3d).
//
// Rounds of the segmented Quickhull in 3D (Tzeng & Owens, Algorithm 1 and
// Section 4.3).  The points stay on the device; the facets of the current
// hull (corners, neighbours, planes, the range of their outside set in the
// point pool and their apex) are kept on the host (qh3d_topo.h).  One round:
//
//   1. topology (host threads): apexes whose visible regions do not touch
//      are accepted in facet id order and each region is replaced by its cone
//      (Topo::round);
//   2. classify (device, two passes): the points of every removed facet are
//      tested against the new facets of their region and counted, then
//      scattered into fresh ranges of the pool; the rest are dropped.
//   3. apex (device): the farthest point of every new facet's outside set.
//
// When no facet has outside points, the corners whose facets span at least
// three planes are the hull vertices; every face (edge-connected coplanar
// facets) is triangulated again as a fan from its lowest-index vertex over its
// vertices, counter-clockwise seen from outside, so the facet list is the
// canonical triangulation of the hull, a function of the point set alone.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <initializer_list>
#include <utility>
#include <memory>
#include <new>
#include <vector>

#include "../../include/qh.h"
#include "qh3d.h"
#include "qh3d_topo.h"
#include "qh_ctx.h"

namespace qh3 {

namespace {

// device buffer that only grows
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t want(size_t b) {
        if (b <= bytes) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        size_t nb = std::max<size_t>(b, 4096);
        nb = nb + nb / 4;
        hipError_t e = hipMalloc(&p, nb);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = nb;
        return hipSuccess;
    }
    template <typename T>
    T *as() const {
        return static_cast<T *>(p);
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

// pinned host buffer that only grows
struct HBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t want(size_t b) {
        if (b <= bytes) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        size_t nb = std::max<size_t>(b, 4096);
        nb = nb + nb / 4;
        hipError_t e = hipHostMalloc(&p, nb, hipHostMallocDefault);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = nb;
        return hipSuccess;
    }
    template <typename T>
    T *as() const {
        return static_cast<T *>(p);
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
};

}  // namespace

struct Ctx3 {
    DBuf pool[2];      // point pools: x, y, z, idx planes of pool_cap each
    int64_t pool_cap = 0;
    DBuf fac, src, seg, counts, cursor, range, tkeys, skeys, gdst, init, filt, ilist, scan;
    HBuf up, down;
    std::vector<hipEvent_t> ev;
    Topo topo;                         // facet table (kept for its capacity)
    std::unique_ptr<Workers> workers;  // host threads of the topology step
};

}  // namespace qh3

namespace qhi {
void ctx3_free(qh3::Ctx3 *c3) {
    if (!c3) return;
    for (auto &b : c3->pool) b.release();
    c3->fac.release();
    c3->src.release();
    c3->seg.release();
    c3->counts.release();
    c3->cursor.release();
    c3->range.release();
    c3->tkeys.release();
    c3->skeys.release();
    c3->gdst.release();
    c3->init.release();
    c3->filt.release();
    c3->ilist.release();
    c3->scan.release();
    c3->up.release();
    c3->down.release();
    for (hipEvent_t e : c3->ev) (void)hipEventDestroy(e);
    delete c3;
}
}  // namespace qhi

namespace qh3 {
namespace {

#define QH3_TRY(expr)                    \
    do {                                 \
        if ((expr) != hipSuccess) {      \
            (void)hipGetLastError();     \
            return QH_EDEVICE;           \
        }                                \
    } while (0)

FacetRec to_rec(const Topo &T, const Facet &f) {
    FacetRec r;
    memset(&r, 0, sizeof(r));
    const int32_t *a = T.coords(f.v[0]), *b = T.coords(f.v[1]), *c = T.coords(f.v[2]);
    r.nx = f.n[0];
    r.ny = f.n[1];
    r.nz = f.n[2];
    r.off = f.off;
    r.ax = a[0];
    r.ay = a[1];
    r.az = a[2];
    r.ebx = b[0] - a[0];
    r.eby = b[1] - a[1];
    r.ebz = b[2] - a[2];
    r.ecx = c[0] - a[0];
    r.ecy = c[1] - a[1];
    r.ecz = c[2] - a[2];
    return r;
}

struct Run {
    qh_ctx *c;
    Ctx3 *w;
    hipStream_t st;
    int mode;
    bool timing;
    const int32_t *x, *y, *z;
    int32_t n;
    Topo *T = nullptr;             // the facet table
    Workers *W = nullptr;          // host threads
    int cur = 0;                   // pool holding the live ranges
    int64_t top = 0;               // first free pool position
    // statistics
    int64_t rounds = 0, launches = 0, syncs = 0, pts_in = 0, pts_out = 0, apex_pts = 0;
    int64_t max_active = 0;
    double host_ms = 0, output_ms = 0;
    std::vector<std::pair<int, int>> evk;  // (kind, event pair index)

    Pool pool(int i) const {
        Pool p;
        int32_t *b = w->pool[i].as<int32_t>();
        p.x = b;
        p.y = b + w->pool_cap;
        p.z = b + 2 * w->pool_cap;
        p.idx = b + 3 * w->pool_cap;
        return p;
    }

    hipError_t ev_begin(int kind) {
        if (!timing) return hipSuccess;
        const size_t i = evk.size() * 2;
        while (w->ev.size() < i + 2) {
            hipEvent_t e;
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return err;
            w->ev.push_back(e);
        }
        evk.push_back({kind, (int)evk.size()});
        return hipEventRecord(w->ev[i], st);
    }
    hipError_t ev_end() {
        if (!timing) return hipSuccess;
        return hipEventRecord(w->ev[evk.size() * 2 - 1], st);
    }

    qh_status classify(const std::vector<SrcRec> &srcs, int from_input, int32_t first, int32_t nf);
    qh_status compact(const std::vector<SrcRec> &srcs_in, std::vector<SrcRec> &srcs_out);
};

// Classify the points of srcs against the new facets [first, first + nf)
// (the round's facet table, in order), fill the new facets' outside sets and
// apexes.
qh_status Run::classify(const std::vector<SrcRec> &srcs_in, int from_input, int32_t first,
                        int32_t nf) {
    std::vector<SrcRec> srcs = srcs_in;
    Topo &Tp = *T;
    int64_t total = 0;
    for (const SrcRec &s : srcs) total += s.len;
    if (!from_input && top + total > w->pool_cap) {
        std::vector<SrcRec> moved;
        qh_status s = compact(srcs, moved);
        if (s != QH_OK) return s;
        srcs.swap(moved);
    }
    int32_t tiles = 0;
    for (SrcRec &s : srcs) {
        s.tile0 = tiles;
        tiles += (s.len + kTile - 1) / kTile;
    }
    // the new outside sets never pass the pool's end: every classified point
    // is written at most once, after the live data
    if (top + total > w->pool_cap) return QH_ECAPACITY;
    // staging (pinned, written only after the previous round's last wait):
    // up = [facet records | sources], down = [counts | apex keys | totals]
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int64_t nseg_max = std::min<int64_t>(nf, total);
    const int64_t tiles_max = nseg_max + total / kTile;
    const int32_t nchunk = (nf + kScanChunk - 1) / kScanChunk;
    const size_t fb = sizeof(FacetRec) * (size_t)nf, sb = sizeof(SrcRec) * srcs.size();
    const size_t o_src = al(fb);
    QH3_TRY(w->up.want(o_src + al(sb)));
    const size_t o_key = al(sizeof(uint32_t) * (size_t)nf);
    const size_t o_tot = o_key + al(sizeof(ApexKey) * (size_t)nseg_max);
    QH3_TRY(w->down.want(o_tot + sizeof(ScanTot) + 256));
    QH3_TRY(w->fac.want(fb));
    QH3_TRY(w->src.want(sb));
    QH3_TRY(w->counts.want(sizeof(uint32_t) * (size_t)nf));
    QH3_TRY(w->cursor.want(sizeof(uint32_t) * (size_t)nf));
    QH3_TRY(w->range.want(sizeof(int64_t) * (size_t)nf));
    QH3_TRY(w->seg.want(sizeof(SegRec) * (size_t)std::max<int64_t>(1, nseg_max)));
    QH3_TRY(w->tkeys.want(sizeof(ApexKey) * (size_t)std::max<int64_t>(1, tiles_max)));
    QH3_TRY(w->skeys.want(sizeof(ApexKey) * (size_t)std::max<int64_t>(1, nseg_max)));
    const size_t o_stot = al(sizeof(uint32_t) * 3 * (size_t)std::max(1, nchunk));
    QH3_TRY(w->scan.want(o_stot + sizeof(ScanTot)));
    uint32_t *dpart = w->scan.as<uint32_t>();
    ScanTot *dtot = reinterpret_cast<ScanTot *>(w->scan.as<char>() + o_stot);
    FacetRec *hf = w->up.as<FacetRec>();
    W->run(nf, 4096, [&](int64_t lo, int64_t hi, int) {
        for (int64_t j = lo; j < hi; ++j) hf[j] = to_rec(Tp, Tp.F[first + j]);
    });
    SrcRec *hs = reinterpret_cast<SrcRec *>(w->up.as<char>() + o_src);
    std::copy(srcs.begin(), srcs.end(), hs);
    QH3_TRY(hipMemcpyAsync(w->fac.p, hf, fb, hipMemcpyHostToDevice, st));
    QH3_TRY(hipMemcpyAsync(w->src.p, hs, sb, hipMemcpyHostToDevice, st));
    QH3_TRY(hipMemsetAsync(w->counts.p, 0, sizeof(uint32_t) * (size_t)nf, st));
    const Pool in = pool(cur);
    // pass 1 counts per new facet; the scan makes the ranges and the apex
    // list on the device; pass 2 scatters; the apex step follows, and the
    // host waits once, for the counts, the apexes and the totals
    QH3_TRY(ev_begin(0));
    QH3_TRY(launch_classify(1, x, y, z, from_input, in, in, w->src.as<SrcRec>(), (int32_t)srcs.size(),
                            tiles, w->fac.as<FacetRec>(), w->counts.as<uint32_t>(),
                            w->cursor.as<uint32_t>(), w->range.as<int64_t>(), mode,
                            w->filt.as<unsigned long long>(), st));
    QH3_TRY(launch_scan(w->counts.as<uint32_t>(), nf, top, w->range.as<int64_t>(), w->seg.as<SegRec>(),
                        w->cursor.as<uint32_t>(), dpart, dtot, st));
    QH3_TRY(launch_classify(2, x, y, z, from_input, in, in, w->src.as<SrcRec>(), (int32_t)srcs.size(),
                            tiles, w->fac.as<FacetRec>(), w->counts.as<uint32_t>(),
                            w->cursor.as<uint32_t>(), w->range.as<int64_t>(), mode,
                            w->filt.as<unsigned long long>(), st));
    QH3_TRY(ev_end());
    launches += 5;
    QH3_TRY(ev_begin(1));
    QH3_TRY(launch_apex(in, w->seg.as<SegRec>(), (int32_t)nseg_max, (int32_t)tiles_max, dtot,
                        w->fac.as<FacetRec>(), w->tkeys.as<ApexKey>(), w->skeys.as<ApexKey>(), st));
    QH3_TRY(ev_end());
    if (nseg_max > 0) launches += 2;
    uint32_t *hc = w->down.as<uint32_t>();
    ApexKey *hk = reinterpret_cast<ApexKey *>(w->down.as<char>() + o_key);
    ScanTot *htot = reinterpret_cast<ScanTot *>(w->down.as<char>() + o_tot);
    QH3_TRY(hipMemcpyAsync(hc, w->counts.p, sizeof(uint32_t) * (size_t)nf, hipMemcpyDeviceToHost, st));
    if (nseg_max > 0)
        QH3_TRY(hipMemcpyAsync(hk, w->skeys.p, sizeof(ApexKey) * (size_t)nseg_max, hipMemcpyDeviceToHost, st));
    QH3_TRY(hipMemcpyAsync(htot, dtot, sizeof(ScanTot), hipMemcpyDeviceToHost, st));
    QH3_TRY(hipStreamSynchronize(st));
    ++syncs;
    pts_in += total;

    // the host's copy of the facet table: each new facet's range (the same
    // prefix sums, over chunks on the host threads) and the facets with
    // points in facet order, as the device listed them
    constexpr int32_t kChunk = 8192;
    const int32_t nhc = (nf + kChunk - 1) / kChunk;
    std::vector<int64_t> cpts((size_t)nhc + 1, 0);
    std::vector<int32_t> cseg((size_t)nhc + 1, 0);
    W->run(nhc, 1, [&](int64_t lo, int64_t hi, int) {
        for (int64_t c = lo; c < hi; ++c) {
            int64_t np = 0;
            int32_t ng = 0;
            for (int32_t j = (int32_t)c * kChunk; j < std::min<int32_t>(nf, (int32_t)(c + 1) * kChunk); ++j) {
                np += hc[j];
                ng += hc[j] ? 1 : 0;
            }
            cpts[c + 1] = np;
            cseg[c + 1] = ng;
        }
    });
    for (int32_t c = 0; c < nhc; ++c) {
        cpts[c + 1] += cpts[c];
        cseg[c + 1] += cseg[c];
    }
    const int64_t written = cpts[nhc];
    const int32_t ns = cseg[nhc];
    // (with no new facet the scan did not run and wrote no totals)
    const ScanTot dt = nf > 0 ? *htot : ScanTot{0, 0, 0};
    if (written != dt.written || ns != dt.nseg || written > total) return QH_EDEVICE;
    std::vector<int32_t> segf((size_t)ns);
    W->run(nhc, 1, [&](int64_t lo, int64_t hi, int) {
        for (int64_t c = lo; c < hi; ++c) {
            int64_t at = top + cpts[c];
            int32_t q = cseg[c];
            for (int32_t j = (int32_t)c * kChunk; j < std::min<int32_t>(nf, (int32_t)(c + 1) * kChunk); ++j) {
                const int32_t id = first + j;
                Tp.len[id] = (int32_t)hc[j];
                Tp.start[id] = at;
                if (hc[j]) segf[q++] = j;
                at += hc[j];
            }
        }
    });
    top += written;
    pts_out += written;
    apex_pts += written;

    // apex of every new facet with points
    if (ns) {
        std::atomic<int> bad{0};
        W->run(ns, 4096, [&](int64_t lo, int64_t hi, int) {
            for (int64_t s = lo; s < hi; ++s) {
                const ApexKey &k = hk[s];
                // an outside set holds only points above its facet
                if (k.idx < 0 || k.idx >= n || k.d <= 0)
                    bad.store(1);
                else
                    Tp.set_apex(first + segf[s], k.idx, k.x, k.y, k.z);
            }
        });
        if (bad.load()) return QH_EDEVICE;
    }
    for (int32_t j : segf) Tp.active.push_back(first + j);
    return QH_OK;
}

// Copy every live range (facets with points, and the sources of this round)
// to the other pool, front to back.
qh_status Run::compact(const std::vector<SrcRec> &srcs_in, std::vector<SrcRec> &srcs_out) {
    std::vector<SegRec> segs;
    std::vector<int64_t> dst;
    int64_t pos = 0;
    int32_t tiles = 0;
    auto add = [&](int64_t start, int32_t len) {
        SegRec s;
        s.start = start;
        s.len = len;
        s.facet = 0;
        s.tile0 = tiles;
        s.pad = 0;
        tiles += (len + kTile - 1) / kTile;
        segs.push_back(s);
        dst.push_back(pos);
        const int64_t d = pos;
        pos += len;
        return d;
    };
    for (int32_t id : T->active)
        if (T->gone[id] == 0 && T->len[id] > 0) T->start[id] = add(T->start[id], T->len[id]);
    srcs_out = srcs_in;
    for (SrcRec &s : srcs_out)
        if (s.len > 0) s.start = add(s.start, s.len);
    const size_t sb = sizeof(SegRec) * segs.size(), db = sizeof(int64_t) * dst.size();
    QH3_TRY(w->seg.want(sb));
    QH3_TRY(w->gdst.want(db));
    QH3_TRY(hipStreamSynchronize(st));
    QH3_TRY(w->up.want(sb + db + 256));
    memcpy(w->up.p, segs.data(), sb);
    char *hd = w->up.as<char>() + ((sb + 255) & ~(size_t)255);
    memcpy(hd, dst.data(), db);
    QH3_TRY(hipMemcpyAsync(w->seg.p, w->up.p, sb, hipMemcpyHostToDevice, st));
    QH3_TRY(hipMemcpyAsync(w->gdst.p, hd, db, hipMemcpyHostToDevice, st));
    QH3_TRY(ev_begin(2));
    QH3_TRY(launch_gather(pool(cur), pool(1 - cur), w->seg.as<SegRec>(), (int32_t)segs.size(), tiles,
                          w->gdst.as<int64_t>(), st));
    QH3_TRY(ev_end());
    ++launches;
    QH3_TRY(hipStreamSynchronize(st));
    ++syncs;
    cur = 1 - cur;
    top = pos;
    return QH_OK;
}

// Host data to device buffers through the pinned staging buffer (pieces of
// `bytes` each, copied in order), then a wait.
qh_status put_all(Ctx3 *w, hipStream_t st, std::initializer_list<std::pair<void *, std::pair<const void *, size_t>>> parts) {
    size_t total = 0;
    for (const auto &pt : parts) total += (pt.second.second + 255) & ~(size_t)255;
    QH3_TRY(w->up.want(total + 256));
    char *h = w->up.as<char>();
    size_t o = 0;
    for (const auto &pt : parts) {
        const size_t b = pt.second.second;
        if (b) {
            memcpy(h + o, pt.second.first, b);
            QH3_TRY(hipMemcpyAsync(pt.first, h + o, b, hipMemcpyHostToDevice, st));
        }
        o += (b + 255) & ~(size_t)255;
    }
    QH3_TRY(hipStreamSynchronize(st));
    return QH_OK;
}

// The hulls of the instances [off[i], off[i+1]) of the n points (one
// instance for qh_hull3d; every round serves the facets of all of them):
// the sorted index triples and the ascending vertices, in point ids of the
// whole array; degen[i] = 1 for an instance with fewer than four affinely
// independent points (it has no hull).
qh_status run3d(qh_ctx *c, const int32_t *pts, int64_t n, const std::vector<int64_t> &off,
                const int64_t *off_dev, std::vector<int32_t> &tri, std::vector<int32_t> &vlist,
                std::vector<uint8_t> &degen, const qh_opts *o) {
    using clk = std::chrono::steady_clock;
    if (!c->c3) {
        c->c3 = new (std::nothrow) Ctx3();
        if (!c->c3) return QH_ENOMEM;
    }
    Ctx3 *w = c->c3;
    Run R;
    R.c = c;
    R.w = w;
    R.st = o ? (hipStream_t)o->stream : nullptr;
    R.mode = o ? (int)o->mode : 0;
    R.timing = o && (o->flags & QH_FLAG_TIMING);
    R.x = pts;
    R.y = pts + n;
    R.z = pts + 2 * n;
    R.n = (int32_t)n;
    hipStream_t st = R.st;

    // pools: the live points never exceed n, and one round writes at most n
    const int64_t cap = 2 * n + kTile;
    if (w->pool_cap < cap) {
        w->pool[0].release();
        w->pool[1].release();
        w->pool_cap = 0;
        QH3_TRY(w->pool[0].want(sizeof(int32_t) * 4 * (size_t)cap));
        QH3_TRY(w->pool[1].want(sizeof(int32_t) * 4 * (size_t)cap));
        w->pool_cap = cap;
    }
    const int32_t k = (int32_t)off.size() - 1;
    auto grid_for = [&](int64_t m) { return std::max(1, std::min<int>(c->cus * 4, (int)((m + kBlock - 1) / kBlock))); };
    int gmax = 1;
    for (int32_t i = 0; i < k; ++i) gmax = std::max(gmax, grid_for(off[i + 1] - off[i]));
    const size_t res_at = (init_scratch_bytes(gmax) + 255) & ~(size_t)255;
    QH3_TRY(w->init.want(res_at + sizeof(InitRes) * (size_t)k + 512));
    QH3_TRY(w->filt.want(64));
    QH3_TRY(hipMemsetAsync(w->filt.p, 0, 16, st));
    InitRes *dres = reinterpret_cast<InitRes *>(w->init.as<char>() + res_at);
    // the first simplex of every instance: the large ones one after the
    // other over the whole device (the scratch is reused in turn), the small
    // ones (with the instance bounds on the device) one block each in one launch
    std::vector<int32_t> small;
    QH3_TRY(R.ev_begin(3));
    for (int32_t i = 0; i < k; ++i) {
        const int64_t ni = off[i + 1] - off[i];
        if (ni < 4) continue;
        if (off_dev && ni <= kInitSmall) {
            small.push_back(i);
            continue;
        }
        QH3_TRY(launch_init(R.x + off[i], R.y + off[i], R.z + off[i], (int32_t)ni, w->init.p, dres + i,
                            grid_for(ni), st));
        R.launches += 7;
    }
    if (!small.empty()) {
        const size_t lb = sizeof(int32_t) * small.size();
        QH3_TRY(w->ilist.want(lb));
        QH3_TRY(w->up.want(lb + 256));
        memcpy(w->up.p, small.data(), lb);
        QH3_TRY(hipMemcpyAsync(w->ilist.p, w->up.p, lb, hipMemcpyHostToDevice, st));
        QH3_TRY(launch_init_small(R.x, R.y, R.z, off_dev, w->ilist.as<int32_t>(), (int32_t)small.size(), dres, st));
        R.launches += 1;
    }
    QH3_TRY(R.ev_end());
    QH3_TRY(w->down.want(sizeof(InitRes) * (size_t)k + 256));
    InitRes *hres = w->down.as<InitRes>();
    QH3_TRY(hipMemcpyAsync(hres, dres, sizeof(InitRes) * (size_t)k, hipMemcpyDeviceToHost, st));
    QH3_TRY(hipStreamSynchronize(st));
    ++R.syncs;

    if (!w->workers) {
        w->workers.reset(new (std::nothrow) Workers());
        if (!w->workers) return QH_ENOMEM;
    }
    Topo &Tp = w->topo;
    R.T = &Tp;
    R.W = w->workers.get();
    Tp.reset((int32_t)n);
    degen.assign((size_t)k, 1);
    std::vector<SrcRec> srcs0;
    int64_t hulls = 0;
    for (int32_t i = 0; i < k; ++i) {
        const int64_t ni = off[i + 1] - off[i];
        if (ni < 4) continue;
        const InitRes &res = hres[i];
        if (res.error) return QH_ERANGE;
        if (res.a < 0 || res.c < 0 || res.d < 0) continue;
        // each facet turned away from the opposite corner
        const int32_t T4[4] = {(int32_t)(res.a + off[i]), (int32_t)(res.b + off[i]),
                               (int32_t)(res.c + off[i]), (int32_t)(res.d + off[i])};
        for (int q = 0; q < 4; ++q) {
            if (T4[q] < off[i] || T4[q] >= off[i + 1]) return QH_EDEVICE;
            Tp.set_point(T4[q], res.coords[q][0], res.coords[q][1], res.coords[q][2]);
        }
        if (!Tp.simplex(T4)) return QH_ENOMEM;
        SrcRec sr;
        sr.start = off[i];
        sr.len = (int32_t)ni;
        sr.gfirst = (int32_t)(4 * hulls);
        sr.gcount = 4;
        sr.tile0 = 0;
        srcs0.push_back(sr);
        degen[(size_t)i] = 0;
        ++hulls;
    }
    R.cur = 0;
    R.top = 0;
    if (hulls) {
        qh_status s = R.classify(srcs0, 1, 0, (int32_t)(4 * hulls));
        if (s != QH_OK) return s;
    }
    std::vector<TopoSrc> tsrcs;
    std::vector<SrcRec> srcs;
    while (!Tp.active.empty()) {
        R.max_active = std::max<int64_t>(R.max_active, (int64_t)Tp.active.size());
        // every round drops at least the accepted apexes from the live points
        if (R.rounds > n) return QH_EDEVICE;
        ++R.rounds;
        int32_t first = 0, count = 0;
        const auto t0 = clk::now();
        const int tr = Tp.round((int32_t)R.rounds, *R.W, tsrcs, first, count);
        R.host_ms += std::chrono::duration<double, std::milli>(clk::now() - t0).count();
        if (tr == kTopoNoMem) return QH_ENOMEM;
        if (tr != kTopoOk) return QH_EDEVICE;
        srcs.resize(tsrcs.size());
        for (size_t i = 0; i < tsrcs.size(); ++i) {
            srcs[i].start = tsrcs[i].start;
            srcs[i].len = tsrcs[i].len;
            srcs[i].gfirst = tsrcs[i].gfirst;
            srcs[i].gcount = tsrcs[i].gcount;
            srcs[i].tile0 = 0;
        }
        qh_status s = R.classify(srcs, 0, first, count);
        if (s != QH_OK) return s;
    }
    const auto t0 = clk::now();
    tri.clear();
    vlist.clear();
    if (hulls && !Tp.output(*R.W, tri, vlist, hulls)) return QH_EDEVICE;
    R.output_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    R.host_ms += R.output_ms;

    if (o && o->stats) {
        qh_stats *S = o->stats;
        unsigned long long fc[2] = {0, 0};
        QH3_TRY(hipMemcpyAsync(fc, w->filt.p, sizeof(fc), hipMemcpyDeviceToHost, R.st));
        QH3_TRY(hipStreamSynchronize(R.st));
        S->rounds = R.rounds;
        S->round_launches = R.launches;
        S->round_points_in = R.pts_in;
        S->round_points_out = R.pts_out;
        S->split_points_out = 0;
        // classify: pass 1 reads x, y, z (12 B), pass 2 reads 16 B and writes
        // 16 B per survivor; apex reads 16 B per point
        S->round_kernel_bytes = 28 * R.pts_in + 16 * R.pts_out + 16 * R.apex_pts;
        S->hull_bytes = 36 * n + S->round_kernel_bytes;
        S->filter_tests = (int64_t)fc[0];
        S->filter_fallbacks = (int64_t)fc[1];
        S->max_segments = R.max_active;
        S->host_syncs = R.syncs;
        S->host_ms = R.host_ms;
        S->host_output_ms = R.output_ms;
        S->degenerate_instances = 0;
        for (uint8_t d : degen) S->degenerate_instances += d;
        if (R.timing) {
            double ms[4] = {0, 0, 0, 0};
            for (size_t j = 0; j < R.evk.size(); ++j) {
                float t = 0;
                if (hipEventElapsedTime(&t, w->ev[2 * j], w->ev[2 * j + 1]) == hipSuccess)
                    ms[R.evk[j].first] += t;
            }
            S->round_kernel_ms = ms[0];
            S->segment_ms = ms[1];
            S->extremes_ms = ms[3];
            S->kernel_ms = ms[0] + ms[1] + ms[2] + ms[3];
        }
    }
    return QH_OK;
}

}  // namespace
}  // namespace qh3

extern "C" qh_status qh_hull3d(const int32_t *pts, int64_t n, int32_t *facets, int64_t *nfacets,
                               int32_t *verts, int64_t *nverts, const qh_opts *opts) {
    if (nfacets) *nfacets = 0;
    if (nverts) *nverts = 0;
    if (!nfacets || !nverts || n < 0 || n > (int64_t)INT32_MAX / 2 - 4096) return QH_EINVAL;
    if (opts && opts->stats) {
        memset(opts->stats, 0, sizeof(qh_stats));
        opts->stats->finish_round = -1;  // a 2D option
    }
    if (opts && opts->mode != QH_EXACT_INT64 && opts->mode != QH_FP32_FILTER) return QH_EINVAL;
    if (n < 4) return QH_EDEGENERATE;
    if (!pts || !facets || !verts) return QH_EINVAL;
    qhi::TempCtx t;
    qh_status s = qhi::get_ctx(opts, t);
    if (s != QH_OK) return s;
    const std::vector<int64_t> off = {0, n};
    std::vector<int32_t> tri, vl;
    std::vector<uint8_t> degen;
    s = qh3::run3d(t.c, pts, n, off, nullptr, tri, vl, degen, opts);
    if (s != QH_OK) return s;
    if (degen[0]) {
        if (opts && opts->stats) opts->stats->degenerate_instances = 0;
        return QH_EDEGENERATE;
    }
    hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
    s = qh3::put_all(t.c->c3, st, {{facets, {tri.data(), sizeof(int32_t) * tri.size()}},
                                    {verts, {vl.data(), sizeof(int32_t) * vl.size()}}});
    if (s != QH_OK) return s;
    if (opts && opts->stats) {
        opts->stats->host_syncs += 1;
        opts->stats->degenerate_instances = 0;
    }
    *nfacets = (int64_t)(tri.size() / 3);
    *nverts = (int64_t)vl.size();
    return QH_OK;
}

extern "C" qh_status qh_hull3d_batched(const int32_t *pts, int64_t n_total, const int64_t *offsets, int32_t k,
                                       int32_t *facets, int64_t *facet_offsets, int32_t *verts,
                                       int64_t *vert_offsets, const qh_opts *opts) {
    if (k < 1 || k > (1 << 20) || n_total < 0 || n_total > (int64_t)INT32_MAX / 2 - 4096) return QH_EINVAL;
    if (!offsets || !facet_offsets || !vert_offsets || (n_total > 0 && (!pts || !facets || !verts)))
        return QH_EINVAL;
    if (opts && opts->stats) {
        memset(opts->stats, 0, sizeof(qh_stats));
        opts->stats->finish_round = -1;  // a 2D option
    }
    if (opts && opts->mode != QH_EXACT_INT64 && opts->mode != QH_FP32_FILTER) return QH_EINVAL;
    qhi::TempCtx t;
    qh_status s = qhi::get_ctx(opts, t);
    if (s != QH_OK) return s;
    hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
    // the instance bounds, checked on the host
    std::vector<int64_t> off((size_t)k + 1);
    if (hipMemcpyAsync(off.data(), offsets, sizeof(int64_t) * off.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        return QH_EDEVICE;
    }
    if (off[0] != 0 || off[(size_t)k] != n_total) return QH_EINVAL;
    for (int32_t i = 0; i < k; ++i)
        if (off[(size_t)i + 1] < off[(size_t)i]) return QH_EINVAL;
    std::vector<int32_t> tri, vl;
    std::vector<uint8_t> degen((size_t)k, 1);
    if (n_total > 0) {
        s = qh3::run3d(t.c, pts, n_total, off, offsets, tri, vl, degen, opts);
        if (s != QH_OK) return s;
    } else if (opts && opts->stats) {
        opts->stats->degenerate_instances = k;
    }
    // every instance's triples and vertices, in its own point indices: the
    // vertices are sorted and so are the triples by their first vertex, so
    // each instance is one contiguous range of both
    std::vector<int64_t> foff((size_t)k + 1, 0), voff((size_t)k + 1, 0);
    const size_t nt = tri.size() / 3;
    size_t tpos = 0, vpos = 0;
    for (int32_t i = 0; i < k; ++i) {
        const int64_t lo = off[(size_t)i], hi = off[(size_t)i + 1];
        const size_t v0 = vpos, t0 = tpos;
        while (vpos < vl.size() && vl[vpos] < hi) {
            if (vl[vpos] < lo) return QH_EDEVICE;
            vl[vpos] = (int32_t)(vl[vpos] - lo);
            ++vpos;
        }
        while (tpos < nt && tri[3 * tpos] < hi) {
            for (int q = 0; q < 3; ++q) {
                int32_t &x = tri[3 * tpos + q];
                if (x < lo || x >= hi) return QH_EDEVICE;
                x = (int32_t)(x - lo);
            }
            ++tpos;
        }
        const int64_t nv = (int64_t)(vpos - v0), nti = (int64_t)(tpos - t0);
        if (degen[(size_t)i] ? (nv != 0 || nti != 0) : (nv < 4 || nti != 2 * nv - 4)) return QH_EDEVICE;
        foff[(size_t)i + 1] = (int64_t)tpos;
        voff[(size_t)i + 1] = (int64_t)vpos;
    }
    if (vpos != vl.size() || tpos != nt) return QH_EDEVICE;
    if (!t.c->c3) {
        t.c->c3 = new (std::nothrow) qh3::Ctx3();
        if (!t.c->c3) return QH_ENOMEM;
    }
    s = qh3::put_all(t.c->c3, st,
                     {{facets, {tri.data(), sizeof(int32_t) * tri.size()}},
                      {verts, {vl.data(), sizeof(int32_t) * vl.size()}},
                      {facet_offsets, {foff.data(), sizeof(int64_t) * foff.size()}},
                      {vert_offsets, {voff.data(), sizeof(int64_t) * voff.size()}}});
    if (s != QH_OK) return s;
    if (opts && opts->stats) opts->stats->host_syncs += 2;
    return QH_OK;
}
