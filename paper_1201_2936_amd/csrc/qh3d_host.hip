// qh3d_host.hip -- the host driver of the 3D Quickhull (qh_hull3d).
//
// Rounds of the segmented Quickhull in 3D (Tzeng & Owens, Algorithm 1 and
// Section 4.3).  The points stay on the device; the facets of the current
// hull (corners, neighbours, planes, the range of their outside set in the
// point pool and their apex) are kept here.  One round:
//
//   1. topology (host): the facets with outside points are taken in id order
//      as candidates.  For each, the facets its apex sees strictly (a walk
//      over neighbours from the facet) are the region the apex replaces.  A
//      candidate whose region meets a facet locked earlier in the round waits
//      for a later round; otherwise it is accepted and its region and the
//      region's neighbours are locked.  An accepted apex never sees another
//      accepted apex's new facets (each such facet lies between two planes
//      the other apex is on or below), so the accepted insertions give the
//      hull that inserting them one after the other would.
//      Every horizon edge of a region gets a new facet (edge, apex).
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
#include <chrono>
#include <new>
#include <thread>
#include <vector>

#include "../../include/qh.h"
#include "qh3d.h"
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
    DBuf fac, src, seg, counts, cursor, range, tkeys, skeys, gdst, init, filt;
    HBuf up, down;
    std::vector<hipEvent_t> ev;
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

struct HFacet {
    int32_t v[3];      // corners (input indices), counter-clockwise from outside
    int32_t nb[3];     // facet across v[i] -> v[i+1]
    int32_t c[3][3];   // corner coordinates
    int64_t n[3];      // outward normal (v1 - v0) x (v2 - v0)
    int64_t off;       // n . v0
    int64_t start;     // outside set: pool range
    int32_t len;
    int32_t apex;      // apex index (input), -1 = none
    int32_t ap[3];     // apex coordinates
    int32_t alive;
    int32_t lock;      // round stamp of the last lock
    int64_t seen;      // walk stamp
    int64_t vis;       // walk stamp at which it was found visible
};

int64_t side(const HFacet &f, const int32_t p[3]) {
    return f.n[0] * p[0] + f.n[1] * p[1] + f.n[2] * p[2] - f.off;
}

void set_plane(HFacet &f) {
    const int64_t ux = f.c[1][0] - f.c[0][0], uy = f.c[1][1] - f.c[0][1], uz = f.c[1][2] - f.c[0][2];
    const int64_t wx = f.c[2][0] - f.c[0][0], wy = f.c[2][1] - f.c[0][1], wz = f.c[2][2] - f.c[0][2];
    f.n[0] = uy * wz - uz * wy;
    f.n[1] = uz * wx - ux * wz;
    f.n[2] = ux * wy - uy * wx;
    f.off = f.n[0] * f.c[0][0] + f.n[1] * f.c[0][1] + f.n[2] * f.c[0][2];
}

HFacet make_facet(int32_t a, const int32_t *ca, int32_t b, const int32_t *cb, int32_t c,
                  const int32_t *cc) {
    HFacet f;
    memset(&f, 0, sizeof(f));
    f.v[0] = a;
    f.v[1] = b;
    f.v[2] = c;
    for (int k = 0; k < 3; ++k) {
        f.c[0][k] = ca[k];
        f.c[1][k] = cb[k];
        f.c[2][k] = cc[k];
    }
    f.nb[0] = f.nb[1] = f.nb[2] = -1;
    f.apex = -1;
    f.alive = 1;
    f.lock = -1;
    f.seen = -1;
    f.vis = -1;
    set_plane(f);
    return f;
}

FacetRec to_rec(const HFacet &f) {
    FacetRec r;
    memset(&r, 0, sizeof(r));
    r.nx = f.n[0];
    r.ny = f.n[1];
    r.nz = f.n[2];
    r.off = f.off;
    r.ax = f.c[0][0];
    r.ay = f.c[0][1];
    r.az = f.c[0][2];
    r.ebx = f.c[1][0] - f.c[0][0];
    r.eby = f.c[1][1] - f.c[0][1];
    r.ebz = f.c[1][2] - f.c[0][2];
    r.ecx = f.c[2][0] - f.c[0][0];
    r.ecy = f.c[2][1] - f.c[0][1];
    r.ecz = f.c[2][2] - f.c[0][2];
    return r;
}

// same plane (both through a common point): parallel normals, same direction
bool coplanar_dir(const int64_t a[3], const int64_t b[3]) {
    const __int128 cx = (__int128)a[1] * b[2] - (__int128)a[2] * b[1];
    const __int128 cy = (__int128)a[2] * b[0] - (__int128)a[0] * b[2];
    const __int128 cz = (__int128)a[0] * b[1] - (__int128)a[1] * b[0];
    if (cx != 0 || cy != 0 || cz != 0) return false;
    const __int128 d = (__int128)a[0] * b[0] + (__int128)a[1] * b[1] + (__int128)a[2] * b[2];
    return d > 0;
}

struct Run {
    qh_ctx *c;
    Ctx3 *w;
    hipStream_t st;
    int mode;
    bool timing;
    const int32_t *x, *y, *z;
    int32_t n;
    std::vector<HFacet> F;
    std::vector<int32_t> active;   // facets with outside points, ascending id
    int64_t walks = 0;             // visibility walks made (stamps)
    std::vector<int32_t> from;     // per point: the cone facet whose horizon edge starts there
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

    qh_status classify(const std::vector<SrcRec> &srcs, int from_input,
                       const std::vector<int32_t> &newf);
    qh_status compact(const std::vector<SrcRec> &srcs_in, std::vector<SrcRec> &srcs_out);
    qh_status topology(std::vector<SrcRec> &srcs, std::vector<int32_t> &newf);
    qh_status output(int32_t *facets, int64_t *nfacets, int32_t *verts, int64_t *nverts);
};

// Classify the points of srcs against the new facets newf (the round's
// facet table, in order), fill the new facets' outside sets and apexes.
qh_status Run::classify(const std::vector<SrcRec> &srcs_in, int from_input,
                        const std::vector<int32_t> &newf) {
    std::vector<SrcRec> srcs = srcs_in;
    const int32_t nf = (int32_t)newf.size();
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
    // staging (pinned, written only after the previous round's last wait):
    // up = [facet records | sources | ranges | apex segments],
    // down = [counts | apex keys]
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t fb = sizeof(FacetRec) * (size_t)nf, sb = sizeof(SrcRec) * srcs.size();
    const size_t rb = sizeof(int64_t) * (size_t)nf, gb = sizeof(SegRec) * (size_t)nf;
    const size_t o_src = al(fb), o_rng = o_src + al(sb), o_seg = o_rng + al(rb);
    QH3_TRY(w->up.want(o_seg + al(gb)));
    const size_t o_key = al(sizeof(uint32_t) * (size_t)nf);
    QH3_TRY(w->down.want(o_key + sizeof(ApexKey) * (size_t)nf + 256));
    QH3_TRY(w->fac.want(fb));
    QH3_TRY(w->src.want(sb));
    QH3_TRY(w->counts.want(sizeof(uint32_t) * (size_t)nf));
    QH3_TRY(w->cursor.want(sizeof(uint32_t) * (size_t)nf));
    QH3_TRY(w->range.want(rb));
    FacetRec *hf = w->up.as<FacetRec>();
    for (int32_t j = 0; j < nf; ++j) hf[j] = to_rec(F[newf[j]]);
    SrcRec *hs = reinterpret_cast<SrcRec *>(w->up.as<char>() + o_src);
    std::copy(srcs.begin(), srcs.end(), hs);
    QH3_TRY(hipMemcpyAsync(w->fac.p, hf, fb, hipMemcpyHostToDevice, st));
    QH3_TRY(hipMemcpyAsync(w->src.p, hs, sb, hipMemcpyHostToDevice, st));
    QH3_TRY(hipMemsetAsync(w->counts.p, 0, sizeof(uint32_t) * (size_t)nf, st));
    QH3_TRY(hipMemsetAsync(w->cursor.p, 0, sizeof(uint32_t) * (size_t)nf, st));
    const Pool in = pool(cur);
    QH3_TRY(ev_begin(0));
    QH3_TRY(launch_classify(1, x, y, z, from_input, in, in, w->src.as<SrcRec>(), (int32_t)srcs.size(),
                            tiles, w->fac.as<FacetRec>(), w->counts.as<uint32_t>(),
                            w->cursor.as<uint32_t>(), w->range.as<int64_t>(), mode,
                            w->filt.as<unsigned long long>(), st));
    QH3_TRY(ev_end());
    ++launches;
    uint32_t *hc = w->down.as<uint32_t>();
    QH3_TRY(hipMemcpyAsync(hc, w->counts.p, sizeof(uint32_t) * (size_t)nf, hipMemcpyDeviceToHost, st));
    QH3_TRY(hipStreamSynchronize(st));
    ++syncs;
    pts_in += total;

    // ranges of the new outside sets, after the live data
    int64_t *hr = reinterpret_cast<int64_t *>(w->up.as<char>() + o_rng);
    std::vector<SegRec> segs;
    int32_t seg_tiles = 0;
    int64_t written = 0;
    for (int32_t j = 0; j < nf; ++j) {
        HFacet &f = F[newf[j]];
        f.len = (int32_t)hc[j];
        f.start = top + written;
        hr[j] = f.start;
        written += hc[j];
        if (hc[j]) {
            SegRec sg;
            sg.start = f.start;
            sg.len = (int32_t)hc[j];
            sg.facet = j;
            sg.tile0 = seg_tiles;
            sg.pad = 0;
            seg_tiles += (sg.len + kTile - 1) / kTile;
            segs.push_back(sg);
        }
    }
    if (top + written > w->pool_cap) return QH_ECAPACITY;  // cannot happen after compaction
    QH3_TRY(hipMemcpyAsync(w->range.p, hr, sizeof(int64_t) * (size_t)nf, hipMemcpyHostToDevice, st));
    QH3_TRY(ev_begin(0));
    QH3_TRY(launch_classify(2, x, y, z, from_input, in, in, w->src.as<SrcRec>(), (int32_t)srcs.size(),
                            tiles, w->fac.as<FacetRec>(), w->counts.as<uint32_t>(),
                            w->cursor.as<uint32_t>(), w->range.as<int64_t>(), mode,
                            w->filt.as<unsigned long long>(), st));
    QH3_TRY(ev_end());
    ++launches;
    top += written;
    pts_out += written;

    // apex of every new facet with points
    const int32_t ns = (int32_t)segs.size();
    if (ns) {
        QH3_TRY(w->seg.want(sizeof(SegRec) * (size_t)ns));
        QH3_TRY(w->tkeys.want(sizeof(ApexKey) * (size_t)seg_tiles));
        QH3_TRY(w->skeys.want(sizeof(ApexKey) * (size_t)ns));
        SegRec *hsg = reinterpret_cast<SegRec *>(w->up.as<char>() + o_seg);
        std::copy(segs.begin(), segs.end(), hsg);
        QH3_TRY(hipMemcpyAsync(w->seg.p, hsg, sizeof(SegRec) * (size_t)ns, hipMemcpyHostToDevice, st));
        QH3_TRY(ev_begin(1));
        QH3_TRY(launch_apex(in, w->seg.as<SegRec>(), ns, seg_tiles, w->fac.as<FacetRec>(),
                            w->tkeys.as<ApexKey>(), w->skeys.as<ApexKey>(), st));
        QH3_TRY(ev_end());
        launches += 2;
        ApexKey *hk = reinterpret_cast<ApexKey *>(w->down.as<char>() + o_key);
        QH3_TRY(hipMemcpyAsync(hk, w->skeys.p, sizeof(ApexKey) * (size_t)ns, hipMemcpyDeviceToHost, st));
        QH3_TRY(hipStreamSynchronize(st));
        ++syncs;
        apex_pts += written;
        for (int32_t s = 0; s < ns; ++s) {
            HFacet &f = F[newf[segs[s].facet]];
            if (hk[s].idx < 0 || hk[s].d <= 0) return QH_EDEVICE;  // an outside set holds only points above
            f.apex = hk[s].idx;
            f.ap[0] = hk[s].x;
            f.ap[1] = hk[s].y;
            f.ap[2] = hk[s].z;
        }
    } else {
        QH3_TRY(hipStreamSynchronize(st));
    }
    for (int32_t j = 0; j < nf; ++j)
        if (F[newf[j]].len > 0) active.push_back(newf[j]);
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
    for (int32_t id : active) {
        HFacet &f = F[id];
        if (f.alive && f.len > 0) f.start = add(f.start, f.len);
    }
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

// Accept apexes with non-overlapping regions; build their cones.  Fills the
// sources (removed facets with points) and the new facets, in id order.
qh_status Run::topology(std::vector<SrcRec> &srcs, std::vector<int32_t> &newf) {
    const int32_t stamp = (int32_t)rounds;
    std::vector<int32_t> region, queue;
    struct Edge {
        int32_t u, w, g;
    };
    std::vector<Edge> horizon;
    if (from.size() < (size_t)n) from.assign((size_t)n, -1);  // horizon vertex -> cone facet starting there
    for (int32_t cand : active) {
        if (!F[cand].alive || F[cand].len == 0) continue;
        if (F[cand].lock == stamp) continue;
        const int32_t p[3] = {F[cand].ap[0], F[cand].ap[1], F[cand].ap[2]};
        const int32_t pid = F[cand].apex;
        // visible region: walk from cand over facets strictly below p
        const int64_t wstamp = ++walks;
        region.clear();
        queue.clear();
        bool clash = false;
        F[cand].seen = wstamp;
        F[cand].vis = wstamp;
        queue.push_back(cand);
        for (size_t h = 0; h < queue.size() && !clash; ++h) {
            const HFacet &f = F[queue[h]];
            for (int i = 0; i < 3; ++i) {
                const int32_t g = f.nb[i];
                if (F[g].seen == wstamp) continue;
                F[g].seen = wstamp;
                if (side(F[g], p) > 0) {
                    if (F[g].lock == stamp) {
                        clash = true;
                        break;
                    }
                    F[g].vis = wstamp;
                    queue.push_back(g);
                }
            }
        }
        if (clash) continue;
        region = queue;
        // lock the region and its neighbours
        for (int32_t f : region) {
            F[f].lock = stamp;
            for (int i = 0; i < 3; ++i) F[F[f].nb[i]].lock = stamp;
        }
        // horizon, in walk order
        horizon.clear();
        for (int32_t f : region)
            for (int i = 0; i < 3; ++i) {
                const int32_t g = F[f].nb[i];
                if (F[g].vis == wstamp) continue;
                horizon.push_back({F[f].v[i], F[f].v[(i + 1) % 3], g});
            }
        // the cone
        const int32_t gfirst = (int32_t)newf.size();
        const int32_t first_id = (int32_t)F.size();
        for (const Edge &e : horizon) {
            const HFacet &fg = F[e.g];
            // corner coordinates of u and w from the facet across the edge
            const int32_t *cu = nullptr, *cw = nullptr;
            for (int k = 0; k < 3; ++k) {
                if (fg.v[k] == e.u) cu = fg.c[k];
                if (fg.v[k] == e.w) cw = fg.c[k];
            }
            if (!cu || !cw) return QH_EDEVICE;
            HFacet nf = make_facet(e.u, cu, e.w, cw, pid, p);
            nf.nb[0] = e.g;
            const int32_t id = (int32_t)F.size();
            F.push_back(nf);
            HFacet &g = F[e.g];
            for (int k = 0; k < 3; ++k)
                if (g.v[k] == e.w && g.v[(k + 1) % 3] == e.u) g.nb[k] = id;
            from[e.u] = id;
            newf.push_back(id);
        }
        for (int32_t id = first_id; id < (int32_t)F.size(); ++id) {
            const int32_t nxt = from[F[id].v[1]];
            if (nxt < 0) return QH_EDEVICE;
            F[id].nb[1] = nxt;        // edge w -> p
            F[nxt].nb[2] = id;        // its edge p -> w
            F[id].lock = stamp;
        }
        for (int32_t id = first_id; id < (int32_t)F.size(); ++id) from[F[id].v[0]] = -1;
        const int32_t gcount = (int32_t)F.size() - first_id;
        // the region dies; its points go to the cone
        for (int32_t f : region) {
            F[f].alive = 0;
            if (F[f].len > 0) {
                SrcRec s;
                s.start = F[f].start;
                s.len = F[f].len;
                s.gfirst = gfirst;
                s.gcount = gcount;
                s.tile0 = 0;
                srcs.push_back(s);
            }
        }
    }
    // drop dead facets from the active list (new ones are added after the
    // classification)
    std::vector<int32_t> keep;
    keep.reserve(active.size());
    for (int32_t id : active)
        if (F[id].alive && F[id].len > 0) keep.push_back(id);
    active.swap(keep);
    return QH_OK;
}

// Run fn(lo, hi, t) over [0, n) on up to 16 host threads.
template <typename Fn>
void par_for(int64_t n, Fn fn) {
    int T = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
    if (n < 32768) T = 1;
    std::vector<std::thread> th;
    th.reserve(T);
    for (int t = 1; t < T; ++t) th.emplace_back([&fn, n, T, t] { fn(n * t / T, n * (t + 1) / T, t); });
    fn(0, n / T, 0);
    for (auto &x : th) x.join();
}

struct Tri {
    int32_t a, b, c;
};

bool tri_less(const Tri &p, const Tri &q) {
    if (p.a != q.a) return p.a < q.a;
    if (p.b != q.b) return p.b < q.b;
    return p.c < q.c;
}

// Hull vertices and the canonical triangulation.  Everything is indexed by
// point or facet id in flat arrays (no hashing) and the independent parts run
// on host threads: corners -> incident facets by counting, the vertex test per
// corner, faces by union-find over coplanar neighbours, each face's boundary
// cycle fanned from its lowest vertex, and the triples sorted.
qh_status Run::output(int32_t *facets, int64_t *nfacets, int32_t *verts, int64_t *nverts) {
    const int32_t nf = (int32_t)F.size();
    std::vector<int32_t> alive;
    {
        std::vector<std::vector<int32_t>> part(16);
        par_for(nf, [&](int64_t lo, int64_t hi, int t) {
            for (int64_t i = lo; i < hi; ++i)
                if (F[i].alive) part[t].push_back((int32_t)i);
        });
        for (auto &v : part) alive.insert(alive.end(), v.begin(), v.end());
    }
    const int64_t na = (int64_t)alive.size();
    // incident facets per corner (CSR over point ids)
    std::vector<int32_t> deg((size_t)n + 1, 0);
    for (int32_t f : alive)
        for (int k = 0; k < 3; ++k) deg[F[f].v[k] + 1]++;
    for (int32_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
    std::vector<int32_t> inc(deg[n]);
    {
        std::vector<int32_t> fill(deg.begin(), deg.end() - 1);
        for (int32_t f : alive)
            for (int k = 0; k < 3; ++k) inc[fill[F[f].v[k]]++] = f;
    }
    // the vertex test: at least three distinct planes around a corner
    std::vector<char> isv((size_t)n, 0);
    std::vector<int32_t> vlist;
    {
        std::vector<std::vector<int32_t>> part(16);
        par_for(n, [&](int64_t lo, int64_t hi, int t) {
            for (int64_t v = lo; v < hi; ++v) {
                const int32_t a0 = deg[v], a1 = deg[v + 1];
                if (a0 == a1) continue;
                int32_t planes[3];
                int np = 0;
                for (int32_t q = a0; q < a1 && np < 3; ++q) {
                    const int32_t f = inc[q];
                    bool dup = false;
                    for (int r = 0; r < np && !dup; ++r) dup = coplanar_dir(F[f].n, F[planes[r]].n);
                    if (!dup) planes[np++] = f;
                }
                if (np >= 3) {
                    isv[v] = 1;
                    part[t].push_back((int32_t)v);
                }
            }
        });
        for (auto &v : part) vlist.insert(vlist.end(), v.begin(), v.end());
    }
    // faces: coplanar neighbour pairs found in parallel, joined in order
    std::vector<uint8_t> cop((size_t)na, 0);
    par_for(na, [&](int64_t lo, int64_t hi, int) {
        for (int64_t i = lo; i < hi; ++i) {
            const int32_t f = alive[i];
            uint8_t m = 0;
            for (int k = 0; k < 3; ++k) {
                const int32_t g = F[f].nb[k];
                if (g > f && coplanar_dir(F[f].n, F[g].n)) m |= (uint8_t)(1u << k);
            }
            cop[i] = m;
        }
    });
    std::vector<int32_t> parent((size_t)nf);
    for (int32_t f : alive) parent[f] = f;
    auto root = [&](int32_t f) {
        while (parent[f] != f) {
            parent[f] = parent[parent[f]];
            f = parent[f];
        }
        return f;
    };
    for (int64_t i = 0; i < na; ++i) {
        if (!cop[i]) continue;
        const int32_t f = alive[i];
        for (int k = 0; k < 3; ++k)
            if (cop[i] & (1u << k)) {
                const int32_t a = root(f), b = root(F[f].nb[k]);
                if (a != b) parent[std::max(a, b)] = std::min(a, b);
            }
    }
    for (int32_t f : alive) parent[f] = root(f);
    // facets grouped by face (counting sort on the root id)
    std::vector<int32_t> fstart((size_t)nf + 1, 0);
    for (int32_t f : alive) fstart[parent[f] + 1]++;
    for (int32_t i = 0; i < nf; ++i) fstart[i + 1] += fstart[i];
    std::vector<int32_t> byface(alive.size());
    {
        std::vector<int32_t> fill(fstart.begin(), fstart.end() - 1);
        for (int32_t f : alive) byface[fill[parent[f]]++] = f;
    }
    // every face: boundary cycle over its vertices, fanned from the lowest
    std::vector<std::vector<Tri>> tparts(16);
    std::vector<int> tbad(16, 0);
    par_for(nf, [&](int64_t lo, int64_t hi, int t) {
        std::vector<std::pair<int32_t, int32_t>> edges;
        std::vector<int32_t> poly;
        std::vector<Tri> &out = tparts[t];
        for (int64_t r = lo; r < hi; ++r) {
            const int32_t a0 = fstart[r], a1 = fstart[r + 1];
            if (a0 == a1) continue;
            edges.clear();
            for (int32_t q = a0; q < a1; ++q) {
                const HFacet &f = F[byface[q]];
                for (int k = 0; k < 3; ++k)
                    if (parent[f.nb[k]] != r) edges.push_back({f.v[k], f.v[(k + 1) % 3]});
            }
            if (edges.size() < 3) { tbad[t] = 1; continue; }
            std::sort(edges.begin(), edges.end());
            poly.clear();
            const int32_t start = edges[0].first;
            int32_t u = start;
            size_t steps = 0;
            bool ok = true;
            do {
                if (isv[u]) poly.push_back(u);
                auto it = std::lower_bound(edges.begin(), edges.end(),
                                           std::pair<int32_t, int32_t>(u, INT32_MIN));
                if (it == edges.end() || it->first != u || ++steps > edges.size()) { ok = false; break; }
                u = it->second;
            } while (u != start);
            const size_t m = poly.size();
            if (!ok || m < 3) { tbad[t] = 1; continue; }
            const size_t l0 = std::min_element(poly.begin(), poly.end()) - poly.begin();
            for (size_t i = 1; i + 1 < m; ++i)
                out.push_back({poly[l0], poly[(l0 + i) % m], poly[(l0 + i + 1) % m]});
        }
        std::sort(out.begin(), out.end(), tri_less);
    });
    for (int b : tbad)
        if (b) return QH_EDEVICE;
    std::vector<Tri> tri;
    for (auto &v : tparts) {
        const size_t mid = tri.size();
        tri.insert(tri.end(), v.begin(), v.end());
        std::inplace_merge(tri.begin(), tri.begin() + mid, tri.end(), tri_less);
    }
    const size_t nt = tri.size();
    if (nt != 2 * vlist.size() - 4) return QH_EDEVICE;
    QH3_TRY(w->up.want(sizeof(int32_t) * (3 * nt + vlist.size()) + 512));
    int32_t *ht = w->up.as<int32_t>();
    memcpy(ht, tri.data(), sizeof(int32_t) * 3 * nt);
    int32_t *hv = ht + 3 * nt;
    std::copy(vlist.begin(), vlist.end(), hv);
    QH3_TRY(hipMemcpyAsync(facets, ht, sizeof(int32_t) * 3 * nt, hipMemcpyHostToDevice, st));
    QH3_TRY(hipMemcpyAsync(verts, hv, sizeof(int32_t) * vlist.size(), hipMemcpyHostToDevice, st));
    QH3_TRY(hipStreamSynchronize(st));
    ++syncs;
    *nfacets = (int64_t)nt;
    *nverts = (int64_t)vlist.size();
    return QH_OK;
}

qh_status run3d(qh_ctx *c, const int32_t *pts, int64_t n, int32_t *facets, int64_t *nfacets,
                int32_t *verts, int64_t *nverts, const qh_opts *o) {
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
    const int grid = std::max(1, std::min<int>(c->cus * 4, (int)((n + kBlock - 1) / kBlock)));
    QH3_TRY(w->init.want(init_scratch_bytes(grid) + sizeof(InitRes) + 512));
    QH3_TRY(w->filt.want(64));
    QH3_TRY(hipMemsetAsync(w->filt.p, 0, 16, st));
    InitRes *dres = reinterpret_cast<InitRes *>(w->init.as<char>() + ((init_scratch_bytes(grid) + 255) & ~(size_t)255));
    QH3_TRY(R.ev_begin(3));
    QH3_TRY(launch_init(R.x, R.y, R.z, (int32_t)n, w->init.p, dres, grid, st));
    QH3_TRY(R.ev_end());
    R.launches += 7;
    QH3_TRY(w->down.want(sizeof(InitRes) + 256));
    InitRes *hres = w->down.as<InitRes>();
    QH3_TRY(hipMemcpyAsync(hres, dres, sizeof(InitRes), hipMemcpyDeviceToHost, st));
    QH3_TRY(hipStreamSynchronize(st));
    ++R.syncs;
    if (hres->error) return QH_ERANGE;
    if (hres->a < 0 || hres->c < 0 || hres->d < 0) return QH_EDEGENERATE;
    const InitRes res = *hres;

    // the first simplex: each facet oriented away from the opposite corner
    const int32_t T[4] = {res.a, res.b, res.c, res.d};
    static const int tri[4][4] = {{0, 1, 2, 3}, {0, 1, 3, 2}, {0, 2, 3, 1}, {1, 2, 3, 0}};
    for (int k = 0; k < 4; ++k) {
        const int p = tri[k][0], q = tri[k][1], r = tri[k][2], s = tri[k][3];
        HFacet f = make_facet(T[p], res.coords[p], T[q], res.coords[q], T[r], res.coords[r]);
        if (side(f, res.coords[s]) > 0) f = make_facet(T[p], res.coords[p], T[r], res.coords[r], T[q], res.coords[q]);
        R.F.push_back(f);
    }
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 3; ++i) {
            const int32_t u = R.F[k].v[i], v = R.F[k].v[(i + 1) % 3];
            for (int g = 0; g < 4; ++g)
                for (int j = 0; j < 3; ++j)
                    if (g != k && R.F[g].v[j] == v && R.F[g].v[(j + 1) % 3] == u) R.F[k].nb[i] = g;
        }
    {
        std::vector<SrcRec> srcs(1);
        srcs[0].start = 0;
        srcs[0].len = (int32_t)n;
        srcs[0].gfirst = 0;
        srcs[0].gcount = 4;
        srcs[0].tile0 = 0;
        std::vector<int32_t> newf = {0, 1, 2, 3};
        R.cur = 0;
        R.top = 0;
        qh_status s = R.classify(srcs, 1, newf);
        if (s != QH_OK) return s;
    }
    while (!R.active.empty()) {
        R.max_active = std::max<int64_t>(R.max_active, (int64_t)R.active.size());
        // every round drops at least the accepted apexes from the live points
        if (R.rounds > n) return QH_EDEVICE;
        ++R.rounds;
        std::vector<SrcRec> srcs;
        std::vector<int32_t> newf;
        const auto t0 = clk::now();
        qh_status s = R.topology(srcs, newf);
        R.host_ms += std::chrono::duration<double, std::milli>(clk::now() - t0).count();
        if (s != QH_OK) return s;
        s = R.classify(srcs, 0, newf);
        if (s != QH_OK) return s;
    }
    const auto t0 = clk::now();
    qh_status s = R.output(facets, nfacets, verts, nverts);
    R.output_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    R.host_ms += R.output_ms;
    if (s != QH_OK) return s;

    if (o && o->stats) {
        qh_stats *S = o->stats;
        unsigned long long fc[2] = {0, 0};
        QH3_TRY(hipMemcpy(fc, w->filt.p, sizeof(fc), hipMemcpyDeviceToHost));
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
    return qh3::run3d(t.c, pts, n, facets, nfacets, verts, nverts, opts);
}
