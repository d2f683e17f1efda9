// qh3d_topo.h -- the host side of the 3D Quickhull rounds (Tzeng & Owens,
// Algorithm 1 and Section 4.3): the facet table, the topology step of a round
// and the canonical output.  Plain C++17 with no device code, so the step can
// be run and timed on its own.
//
// A round's topology step, for the facets with outside points (candidates) in
// id order:
//
//   A. (parallel) the visible region of every candidate's apex: the facets
//      reachable from the candidate over neighbours that lie strictly below
//      the apex, walked on the facet table as it was when the round began;
//   B. (in order) a candidate is accepted unless its region meets a facet
//      locked earlier in the round; an accepted candidate locks its region and
//      the region's neighbours.  An accepted apex never sees another accepted
//      apex's new facets (each such facet lies between two planes the other
//      apex is on or below), so the accepted insertions give the hull that
//      inserting them one after the other would.  A walk that started on the
//      round's table reaches a locked facet exactly when the same walk made
//      after the earlier insertions would, so computing the regions first
//      changes nothing;
//   C. (parallel) every horizon edge (u, w) of an accepted region, with g the
//      facet across it, gets a new facet (u, w, apex) whose neighbours are g
//      and the new facets on the edges that meet it at u and w.
//
// The regions of two accepted candidates are disjoint, and so are a region and
// the neighbours of another, so phase C's writes never meet.
#pragma once

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace qh3 {

// A persistent pool of host threads.  run(n, grain, fn) calls fn(lo, hi, t)
// on chunks of at most `grain` items that cover [0, n) (claimed from a
// counter, so uneven chunks balance), with t < threads() the calling thread's
// slot, and returns when every chunk is done.  The caller is slot 0.  Not for
// use by two callers at once.
class Workers {
  public:
    explicit Workers(int want = 0) {
        const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
        nthr_ = std::max(1, std::min(want > 0 ? want : hw, 16));
        for (int t = 1; t < nthr_; ++t) pool_.emplace_back([this, t] { loop(t); });
    }
    ~Workers() {
        {
            std::lock_guard<std::mutex> g(m_);
            stop_ = true;
            ++gen_;
        }
        cv_.notify_all();
        for (auto &th : pool_) th.join();
    }
    Workers(const Workers &) = delete;
    Workers &operator=(const Workers &) = delete;

    int threads() const { return nthr_; }

    void run(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t, int)> &fn) {
        if (n <= 0) return;
        grain = std::max<int64_t>(1, grain);
        if (nthr_ == 1 || n <= grain) {
            fn(0, n, 0);
            return;
        }
        {
            std::lock_guard<std::mutex> g(m_);
            fn_ = &fn;
            n_ = n;
            grain_ = grain;
            next_.store(0);
            busy_ = nthr_ - 1;
            ++gen_;
        }
        cv_.notify_all();
        work(0);
        std::unique_lock<std::mutex> l(m_);
        done_.wait(l, [this] { return busy_ == 0; });
        fn_ = nullptr;
    }

  private:
    void work(int t) {
        for (;;) {
            const int64_t lo = next_.fetch_add(grain_);
            if (lo >= n_) break;
            (*fn_)(lo, std::min(n_, lo + grain_), t);
        }
    }
    void loop(int t) {
        uint64_t seen = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> l(m_);
                cv_.wait(l, [&] { return gen_ != seen; });
                seen = gen_;
                if (stop_) return;
            }
            work(t);
            {
                std::lock_guard<std::mutex> g(m_);
                if (--busy_ == 0) done_.notify_one();
            }
        }
    }

    int nthr_ = 1;
    std::vector<std::thread> pool_;
    std::mutex m_;
    std::condition_variable cv_, done_;
    uint64_t gen_ = 0;
    bool stop_ = false;
    int busy_ = 0;
    const std::function<void(int64_t, int64_t, int)> *fn_ = nullptr;
    int64_t n_ = 0, grain_ = 1;
    std::atomic<int64_t> next_{0};
};

// A set of facet ids for one walk: open addressing, emptied in O(1) by a
// generation number kept in the upper half of every slot (0 = empty).
class IdSet {
  public:
    void clear() {
        if (++gen_ == 0) {
            std::fill(s_.begin(), s_.end(), 0);
            gen_ = 1;
        }
        count_ = 0;
    }
    // true if id was not in the set
    bool insert(int32_t id) {
        if (2 * (count_ + 1) > s_.size()) grow();
        return put((uint32_t)id);
    }

  private:
    bool put(uint32_t id) {
        const uint64_t tag = (uint64_t)gen_ << 32;
        size_t h = (size_t)((id * 0x9E3779B1u) >> 7) & mask_;
        for (;;) {
            const uint64_t e = s_[h];
            if ((uint32_t)(e >> 32) != gen_) {
                s_[h] = tag | id;
                ++count_;
                return true;
            }
            if ((uint32_t)e == id) return false;
            h = (h + 1) & mask_;
        }
    }
    void grow() {
        std::vector<uint64_t> old;
        old.swap(s_);
        s_.assign(std::max<size_t>(64, old.size() * 2), 0);
        mask_ = s_.size() - 1;
        const uint32_t g = gen_;
        gen_ = 1;
        count_ = 0;
        for (uint64_t e : old)
            if ((uint32_t)(e >> 32) == g) put((uint32_t)e);
    }

    std::vector<uint64_t> s_;
    size_t mask_ = 0, count_ = 0;
    uint32_t gen_ = 1;
};

// A growable array of plain records whose new elements are left
// uninitialised (every facet field is written when the facet is made).
template <class T>
class PodVec {
  public:
    PodVec() = default;
    PodVec(const PodVec &) = delete;
    PodVec &operator=(const PodVec &) = delete;
    ~PodVec() { free(p_); }
    size_t size() const { return n_; }
    T *data() { return p_; }
    const T *data() const { return p_; }
    T &operator[](size_t i) { return p_[i]; }
    const T &operator[](size_t i) const { return p_[i]; }
    void clear() { n_ = 0; }
    // false if memory ran out (the contents are kept)
    bool resize(size_t n) {
        if (n > cap_) {
            const size_t c = std::max(n, cap_ + cap_ / 2);
            T *q = static_cast<T *>(aligned_alloc(64, (c * sizeof(T) + 63) & ~(size_t)63));
            if (!q) return false;
            if (n_) memcpy(q, p_, n_ * sizeof(T));
            free(p_);
            p_ = q;
            cap_ = c;
        }
        n_ = n;
        return true;
    }

  private:
    T *p_ = nullptr;
    size_t n_ = 0, cap_ = 0;
};

// A facet of the current hull: the fields a walk touches, in one cache line.
struct alignas(64) Facet {
    int64_t n[3];   // outward normal (v1 - v0) x (v2 - v0)
    int64_t off;    // n . v0: a point p is strictly above iff n . p > off
    int32_t nb[3];  // the facet across the edge v[i] -> v[i+1]
    int32_t v[3];   // corners (point ids), counter-clockwise seen from outside
};
static_assert(sizeof(Facet) == 64, "a facet is one cache line");

// a[i] += a[i - 1] for i = 1 .. len - 1 (an inclusive prefix sum in place),
// in chunks on the host threads: chunk sums, their scan, then each chunk
inline void prefix_sum(Workers &W, int32_t *a, int64_t len) {
    const int64_t chunk = 1 << 16;
    const int64_t nc = (len + chunk - 1) / chunk;
    if (nc <= 1) {
        for (int64_t i = 1; i < len; ++i) a[i] += a[i - 1];
        return;
    }
    std::vector<int64_t> tot((size_t)nc, 0);
    W.run(nc, 1, [&](int64_t lo, int64_t hi, int) {
        for (int64_t c = lo; c < hi; ++c) {
            int32_t *p = a + c * chunk;
            const int64_t m = std::min(chunk, len - c * chunk);
            for (int64_t i = 1; i < m; ++i) p[i] += p[i - 1];
            tot[(size_t)c] = p[m - 1];
        }
    });
    for (int64_t c = 1; c < nc; ++c) tot[(size_t)c] += tot[(size_t)c - 1];
    W.run(nc - 1, 1, [&](int64_t lo, int64_t hi, int) {
        for (int64_t c = lo + 1; c < hi + 1; ++c) {
            int32_t *p = a + c * chunk;
            const int32_t add = (int32_t)tot[(size_t)c - 1];
            const int64_t m = std::min(chunk, len - c * chunk);
            for (int64_t i = 0; i < m; ++i) p[i] += add;
        }
    });
}

enum { kTopoOk = 0, kTopoBroken = 1, kTopoNoMem = 2 };

struct P3 {
    int32_t x, y, z;
};

// The outside set of a removed facet and the cone its points go to.
struct TopoSrc {
    int64_t start;   // pool position
    int32_t len;
    int32_t gfirst;  // first facet of the cone, counted from the round's first new facet
    int32_t gcount;  // facets in the cone
};

inline int64_t side(const Facet &f, const int32_t *p) {
    return f.n[0] * p[0] + f.n[1] * p[1] + f.n[2] * p[2] - f.off;
}

// same plane (both through a common point): parallel normals, same direction
inline bool coplanar_dir(const int64_t a[3], const int64_t b[3]) {
    const __int128 cx = (__int128)a[1] * b[2] - (__int128)a[2] * b[1];
    const __int128 cy = (__int128)a[2] * b[0] - (__int128)a[0] * b[2];
    const __int128 cz = (__int128)a[0] * b[1] - (__int128)a[1] * b[0];
    if (cx != 0 || cy != 0 || cz != 0) return false;
    const __int128 d = (__int128)a[0] * b[0] + (__int128)a[1] * b[1] + (__int128)a[2] * b[2];
    return d > 0;
}

struct Topo {
    int32_t n = 0;                // points
    PodVec<Facet> F;              // every facet made so far (removed ones stay)
    PodVec<uint16_t> lock;        // per facet: the round that last locked it, modulo 2^16 (an
                                  // older lock read as this round's only defers a candidate)
    PodVec<uint8_t> gone;         // per facet: 1 once removed from the hull
    PodVec<int64_t> start;        // per facet: its outside set's pool range
    PodVec<int32_t> len;
    PodVec<int32_t> apex;         // per facet: its farthest outside point, -1 = none
    PodVec<P3> apc;               // ... and that point's coordinates
    std::vector<int32_t> vc;      // x, y, z of every point that is a corner or an apex
    std::vector<int32_t> active;  // facets with outside points, ascending id

    const int32_t *coords(int32_t id) const { return &vc[3 * (size_t)id]; }
    void set_point(int32_t id, int32_t x, int32_t y, int32_t z) {
        int32_t *c = &vc[3 * (size_t)id];
        c[0] = x;
        c[1] = y;
        c[2] = z;
    }

    void reset(int32_t npts) {
        n = npts;
        F.clear();
        lock.clear();
        gone.clear();
        start.clear();
        len.clear();
        apex.clear();
        apc.clear();
        active.clear();
        if (vc.size() < 3 * (size_t)npts) vc.resize(3 * (size_t)npts);
    }

    // the apex of facet f (coordinates kept with the facet; they become a
    // corner's when the apex is inserted)
    void set_apex(int32_t f, int32_t id, int32_t x, int32_t y, int32_t z) {
        apex[f] = id;
        apc[f] = {x, y, z};
    }

    // the plane of facet f from its corners' coordinates
    void set_plane(Facet &f) const {
        const int32_t *a = coords(f.v[0]), *b = coords(f.v[1]), *c = coords(f.v[2]);
        const int64_t ux = (int64_t)b[0] - a[0], uy = (int64_t)b[1] - a[1], uz = (int64_t)b[2] - a[2];
        const int64_t wx = (int64_t)c[0] - a[0], wy = (int64_t)c[1] - a[1], wz = (int64_t)c[2] - a[2];
        f.n[0] = uy * wz - uz * wy;
        f.n[1] = uz * wx - ux * wz;
        f.n[2] = ux * wy - uy * wx;
        f.off = f.n[0] * a[0] + f.n[1] * a[1] + f.n[2] * a[2];
    }

    void init_facet(int32_t id, int32_t a, int32_t b, int32_t c, int32_t stamp) {
        Facet &f = F[id];
        f.v[0] = a;
        f.v[1] = b;
        f.v[2] = c;
        f.nb[0] = f.nb[1] = f.nb[2] = -1;
        set_plane(f);
        lock[id] = (uint16_t)stamp;
        gone[id] = 0;
        start[id] = 0;
        len[id] = 0;
        apex[id] = -1;
    }

    // A first simplex on the points T (coordinates already set), appended
    // to the table: four facets, each turned away from the opposite corner,
    // with neighbours among themselves (one per instance of a batch).
    bool simplex(const int32_t T[4]) {
        static const int tri[4][4] = {{0, 1, 2, 3}, {0, 1, 3, 2}, {0, 2, 3, 1}, {1, 2, 3, 0}};
        const int32_t b = (int32_t)F.size();
        if (!grow((size_t)b + 4)) return false;
        for (int k = 0; k < 4; ++k) {
            const int p = tri[k][0], q = tri[k][1], r = tri[k][2], s = tri[k][3];
            init_facet(b + k, T[p], T[q], T[r], 0);
            if (side(F[b + k], coords(T[s])) > 0) init_facet(b + k, T[p], T[r], T[q], 0);
        }
        for (int k = 0; k < 4; ++k)
            for (int i = 0; i < 3; ++i) {
                const int32_t u = F[b + k].v[i], v = F[b + k].v[(i + 1) % 3];
                for (int g = 0; g < 4; ++g)
                    for (int j = 0; j < 3; ++j)
                        if (g != k && F[b + g].v[j] == v && F[b + g].v[(j + 1) % 3] == u) F[b + k].nb[i] = b + g;
            }
        return true;
    }

    // One round's topology step (phases A-C above).  The new facets are
    // [first, first + count); srcs lists, in order, the outside sets of the
    // removed facets with the cone of each.  Returns kTopoOk, kTopoNoMem, or
    // kTopoBroken if the facet table broke an invariant (a corrupted input
    // from the device).
    int round(int32_t stamp, Workers &W, std::vector<TopoSrc> &srcs, int32_t &first, int32_t &count) {
        const int T = W.threads();
        const int64_t m = (int64_t)active.size();
        if ((int)loc_.size() < T) loc_.resize(T);
        for (int t = 0; t < T; ++t) {
            loc_[t].reg.clear();
            loc_[t].hor.clear();
        }
        rthr_.resize(m);
        roff_.resize(m);
        rcnt_.resize(m);
        rall_.resize(m);
        // A: visible regions, in walk order, on the round's table; after each
        // region, the neighbours of the region that are not in it
        W.run(m, 64, [&](int64_t lo, int64_t hi, int t) {
            std::vector<int32_t> &buf = loc_[t].reg;
            std::vector<int32_t> &rim = loc_[t].rim;
            IdSet &seen = loc_[t].seen;
            for (int64_t i = lo; i < hi; ++i) {
                const int32_t c = active[i];
                const int32_t *p = &apc[c].x;
                const size_t o = buf.size();
                seen.clear();
                seen.insert(c);
                rim.clear();
                buf.push_back(c);
                for (size_t h = o; h < buf.size(); ++h) {
                    const Facet &f = F[buf[h]];
                    for (int k = 0; k < 3; ++k) {
                        const int32_t g = f.nb[k];
                        if (!seen.insert(g)) continue;
                        if (side(F[g], p) > 0)
                            buf.push_back(g);
                        else
                            rim.push_back(g);
                    }
                }
                rthr_[i] = (int16_t)t;
                roff_[i] = (int64_t)o;
                rcnt_[i] = (int32_t)(buf.size() - o);
                buf.insert(buf.end(), rim.begin(), rim.end());
                rall_[i] = (int32_t)(buf.size() - o);
            }
        });
        // B: accept in id order
        acc_.clear();
        uint16_t *lk = lock.data();
        const uint16_t st16 = (uint16_t)stamp;
        // (the regions' addresses first: a flat array, read in order)
        rptr_.resize(m);
        for (int64_t i = 0; i < m; ++i) rptr_[i] = region(i);
        constexpr int64_t kAhead = 8;  // candidates whose locks are fetched ahead
        for (int64_t i = 0; i < m; ++i) {
            if (i + kAhead < m) {
                const int32_t *Rq = rptr_[i + kAhead];
                __builtin_prefetch(&lk[Rq[0]]);
                __builtin_prefetch(&lk[Rq[rcnt_[i + kAhead] > 1 ? 1 : 0]]);
            }
            if (lk[active[i]] == st16) continue;
            const int32_t *R = rptr_[i];
            const int32_t k = rcnt_[i];
            bool clash = false;
            for (int32_t j = 0; j < k && !clash; ++j) clash = lk[R[j]] == st16;
            if (clash) continue;
            acc_.push_back(i);
            for (int32_t j = 0; j < k; ++j) gone[R[j]] = 1;
            for (int32_t j = 0; j < rall_[i]; ++j) lk[R[j]] = st16;
        }
        const int64_t na = (int64_t)acc_.size();
        // C1: horizon edges of every accepted region (walk order)
        hthr_.resize(na);
        hoff_.resize(na);
        hcnt_.resize(na);
        scnt_.resize(na);
        W.run(na, 32, [&](int64_t lo, int64_t hi, int t) {
            std::vector<Edge> &hb = loc_[t].hor;
            for (int64_t a = lo; a < hi; ++a) {
                const int64_t i = acc_[a];
                const int32_t *R = region(i);
                const size_t o = hb.size();
                int32_t ns = 0;
                for (int32_t j = 0; j < rcnt_[i]; ++j) {
                    ns += len[R[j]] > 0;
                    const Facet &f = F[R[j]];
                    for (int e = 0; e < 3; ++e) {
                        const int32_t g = f.nb[e];
                        if (gone[g] == 0) hb.push_back({f.v[e], f.v[(e + 1) % 3], g});
                    }
                }
                hthr_[a] = (int16_t)t;
                hoff_[a] = (int64_t)o;
                hcnt_[a] = (int32_t)(hb.size() - o);
                scnt_[a] = ns;
            }
        });
        // ids of the cones, in acceptance order
        first = (int32_t)F.size();
        base_.resize(na);
        sbase_.resize(na);
        int64_t total = 0, stotal = 0;
        for (int64_t a = 0; a < na; ++a) {
            base_[a] = first + (int32_t)total;
            total += hcnt_[a];
            sbase_[a] = stotal;
            stotal += scnt_[a];
        }
        srcs.resize((size_t)stotal);
        if (!grow((size_t)first + (size_t)total)) return kTopoNoMem;
        count = (int32_t)total;
        // C2: the cones
        std::atomic<int> bad{0};
        W.run(na, 32, [&](int64_t lo, int64_t hi, int t) {
            std::vector<std::pair<int32_t, int32_t>> &by_u = loc_[t].by_u;
            for (int64_t a = lo; a < hi; ++a) {
                const Edge *H = loc_[hthr_[a]].hor.data() + hoff_[a];
                const int32_t k = hcnt_[a], b0 = base_[a];
                const int32_t pid = apex[active[acc_[a]]];
                {
                    const P3 &q = apc[active[acc_[a]]];
                    set_point(pid, q.x, q.y, q.z);
                }
                {
                    // the outside sets of the region, in walk order
                    const int32_t *R = region(acc_[a]);
                    int64_t q = sbase_[a];
                    for (int32_t j = 0; j < rcnt_[acc_[a]]; ++j)
                        if (len[R[j]] > 0) srcs[q++] = {start[R[j]], len[R[j]], b0 - first, k};
                }
                for (int32_t j = 0; j < k; ++j) {
                    const int32_t id = b0 + j;
                    init_facet(id, H[j].u, H[j].w, pid, stamp);
                    F[id].nb[0] = H[j].g;
                    Facet &g = F[H[j].g];
                    int hit = 0;
                    for (int e = 0; e < 3; ++e)
                        if (g.v[e] == H[j].w && g.v[(e + 1) % 3] == H[j].u) {
                            g.nb[e] = id;
                            hit = 1;
                        }
                    if (!hit) bad.store(1);
                }
                // the edge w -> apex of a cone facet is the edge apex -> u of
                // the cone facet whose horizon edge starts at w
                auto link = [&](int32_t j, int32_t jj) {
                    F[b0 + j].nb[1] = b0 + jj;
                    F[b0 + jj].nb[2] = b0 + j;
                };
                if (k <= 16) {
                    for (int32_t j = 0; j < k; ++j) {
                        int32_t jj = 0;
                        while (jj < k && H[jj].u != H[j].w) ++jj;
                        if (jj == k) {
                            bad.store(1);
                            break;
                        }
                        link(j, jj);
                    }
                } else {
                    by_u.clear();
                    for (int32_t j = 0; j < k; ++j) by_u.push_back({H[j].u, j});
                    std::sort(by_u.begin(), by_u.end());
                    for (int32_t j = 0; j < k; ++j) {
                        auto it = std::lower_bound(by_u.begin(), by_u.end(),
                                                   std::pair<int32_t, int32_t>(H[j].w, INT32_MIN));
                        if (it == by_u.end() || it->first != H[j].w) {
                            bad.store(1);
                            break;
                        }
                        link(j, it->second);
                    }
                }
            }
        });
        // the candidates left
        live_.resize(m);
        W.run(m, 4096, [&](int64_t lo, int64_t hi, int) {
            for (int64_t i = lo; i < hi; ++i) live_[i] = gone[active[i]] == 0;
        });
        size_t keep = 0;
        for (int64_t i = 0; i < m; ++i)
            if (live_[i]) active[keep++] = active[i];
        active.resize(keep);
        return bad.load() == 0 ? kTopoOk : kTopoBroken;
    }

    // Hull vertices (ascending) and the canonical triangulation (sorted index
    // triples): the corners whose facets span at least three planes are the
    // vertices; every face (edge-connected coplanar facets) is fanned from its
    // lowest vertex over its vertices, counter-clockwise seen from outside.
    // The table may hold several hulls (disjoint point sets); false if a
    // face's boundary is not one cycle or the triangles do not number
    // 2 V - 4 per hull.
    bool output(Workers &W, std::vector<int32_t> &tri, std::vector<int32_t> &verts, int64_t hulls = 1) {
        const int T = W.threads();
        if ((int)loc_.size() < T) loc_.resize(T);
        const int32_t nf = (int32_t)F.size();
        // the live facets (their order does not matter below: the vertex test
        // and the faces do not depend on it, and the triples are sorted)
        for (int t = 0; t < T; ++t) loc_[t].part.clear();
        W.run(nf, 1 << 16, [&](int64_t lo, int64_t hi, int t) {
            for (int64_t i = lo; i < hi; ++i)
                if (gone[i] == 0) loc_[t].part.push_back((int32_t)i);
        });
        std::vector<int32_t> alive;
        for (int t = 0; t < T; ++t) alive.insert(alive.end(), loc_[t].part.begin(), loc_[t].part.end());
        const int64_t na = (int64_t)alive.size();
        // incident facets per corner (CSR over point ids, filled in parallel)
        std::vector<int32_t> deg((size_t)n + 1, 0);
        W.run(na, 1 << 14, [&](int64_t lo, int64_t hi, int) {
            for (int64_t i = lo; i < hi; ++i)
                for (int k = 0; k < 3; ++k) __atomic_fetch_add(&deg[F[alive[i]].v[k] + 1], 1, __ATOMIC_RELAXED);
        });
        prefix_sum(W, deg.data(), (int64_t)n + 1);
        std::vector<int32_t> inc(deg[n]);
        {
            std::vector<int32_t> fill(deg.begin(), deg.end() - 1);
            W.run(na, 1 << 14, [&](int64_t lo, int64_t hi, int) {
                for (int64_t i = lo; i < hi; ++i)
                    for (int k = 0; k < 3; ++k)
                        inc[__atomic_fetch_add(&fill[F[alive[i]].v[k]], 1, __ATOMIC_RELAXED)] = alive[i];
            });
        }
        // the vertex test: at least three distinct planes around a corner
        std::vector<char> isv((size_t)n, 0);
        W.run(n, 1 << 16, [&](int64_t lo, int64_t hi, int) {
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
                isv[v] = np >= 3;
            }
        });
        {
            // the vertices in ascending order: per-chunk counts, then fills
            const int64_t ch = 1 << 16, nc = ((int64_t)n + ch - 1) / ch;
            std::vector<int32_t> vc((size_t)nc + 1, 0);
            W.run(nc, 1, [&](int64_t lo, int64_t hi, int) {
                for (int64_t c = lo; c < hi; ++c) {
                    int32_t k = 0;
                    for (int64_t v = c * ch; v < std::min<int64_t>(n, (c + 1) * ch); ++v) k += isv[v];
                    vc[(size_t)c + 1] = k;
                }
            });
            for (int64_t c = 0; c < nc; ++c) vc[(size_t)c + 1] += vc[(size_t)c];
            verts.resize((size_t)vc[(size_t)nc]);
            W.run(nc, 1, [&](int64_t lo, int64_t hi, int) {
                for (int64_t c = lo; c < hi; ++c) {
                    int32_t o = vc[(size_t)c];
                    for (int64_t v = c * ch; v < std::min<int64_t>(n, (c + 1) * ch); ++v)
                        if (isv[v]) verts[(size_t)o++] = (int32_t)v;
                }
            });
        }
        // faces: coplanar neighbour pairs (found in parallel) are joined by
        // union-find; a facet with no coplanar neighbour is a face by itself
        std::vector<uint8_t> cop((size_t)na, 0);
        W.run(na, 1 << 15, [&](int64_t lo, int64_t hi, int) {
            for (int64_t i = lo; i < hi; ++i) {
                const int32_t f = alive[i];
                uint8_t msk = 0;
                for (int k = 0; k < 3; ++k) {
                    const int32_t g = F[f].nb[k];
                    if (g > f && coplanar_dir(F[f].n, F[g].n)) msk = (uint8_t)(msk | (1u << k));
                }
                cop[i] = msk;
            }
        });
        std::vector<int32_t> multi;  // facets of faces with two or more facets
        for (int64_t i = 0; i < na; ++i)
            if (cop[i])
                for (int k = 0; k < 3; ++k)
                    if (cop[i] & (1u << k)) {
                        multi.push_back(alive[i]);
                        multi.push_back(F[alive[i]].nb[k]);
                    }
        std::sort(multi.begin(), multi.end());
        multi.erase(std::unique(multi.begin(), multi.end()), multi.end());
        std::vector<int32_t> parent(multi.size());
        auto slot = [&](int32_t f) {
            return (int32_t)(std::lower_bound(multi.begin(), multi.end(), f) - multi.begin());
        };
        for (size_t j = 0; j < multi.size(); ++j) parent[j] = (int32_t)j;
        auto root = [&](int32_t j) {
            while (parent[j] != j) {
                parent[j] = parent[parent[j]];
                j = parent[j];
            }
            return j;
        };
        for (int64_t i = 0; i < na; ++i)
            if (cop[i])
                for (int k = 0; k < 3; ++k)
                    if (cop[i] & (1u << k)) {
                        const int32_t a = root(slot(alive[i])), b = root(slot(F[alive[i]].nb[k]));
                        if (a != b) parent[std::max(a, b)] = std::min(a, b);
                    }
        for (size_t j = 0; j < multi.size(); ++j) parent[j] = root((int32_t)j);
        // the faces of several facets: members grouped by root slot
        std::vector<int32_t> fstart(multi.size() + 1, 0), byface(multi.size());
        for (size_t j = 0; j < multi.size(); ++j) fstart[parent[j] + 1]++;
        for (size_t j = 0; j < multi.size(); ++j) fstart[j + 1] += fstart[j];
        {
            std::vector<int32_t> fill(fstart.begin(), fstart.end() - 1);
            for (size_t j = 0; j < multi.size(); ++j) byface[fill[parent[j]]++] = (int32_t)j;
        }
        // every face: its boundary cycle over its vertices, fanned from the
        // lowest; a one-facet face is its own fan
        std::atomic<int> bad{0};
        for (int t = 0; t < T; ++t) loc_[t].part.clear();
        W.run(na, 1 << 14, [&](int64_t lo, int64_t hi, int t) {
            std::vector<int32_t> &out = loc_[t].part;
            for (int64_t i = lo; i < hi; ++i) {
                const Facet &f = F[alive[i]];
                if (cop[i] || std::binary_search(multi.begin(), multi.end(), alive[i])) continue;
                if (!isv[f.v[0]] || !isv[f.v[1]] || !isv[f.v[2]]) {
                    bad.store(1);
                    continue;
                }
                int l = 0;
                if (f.v[1] < f.v[l]) l = 1;
                if (f.v[2] < f.v[l]) l = 2;
                out.push_back(f.v[l]);
                out.push_back(f.v[(l + 1) % 3]);
                out.push_back(f.v[(l + 2) % 3]);
            }
        });
        W.run((int64_t)multi.size(), 256, [&](int64_t lo, int64_t hi, int t) {
            std::vector<int32_t> &out = loc_[t].part;
            std::vector<std::pair<int32_t, int32_t>> &edges = loc_[t].by_u;
            std::vector<int32_t> &poly = loc_[t].rim;
            for (int64_t r = lo; r < hi; ++r) {
                const int32_t a0 = fstart[r], a1 = fstart[r + 1];
                if (a0 == a1) continue;
                edges.clear();
                for (int32_t q = a0; q < a1; ++q) {
                    const Facet &f = F[multi[byface[q]]];
                    for (int k = 0; k < 3; ++k) {
                        const int32_t g = f.nb[k];
                        const bool inside = std::binary_search(multi.begin(), multi.end(), g) &&
                                            parent[slot(g)] == (int32_t)r;
                        if (!inside) edges.push_back({f.v[k], f.v[(k + 1) % 3]});
                    }
                }
                if (edges.size() < 3) {
                    bad.store(1);
                    continue;
                }
                std::sort(edges.begin(), edges.end());
                poly.clear();
                const int32_t s0 = edges[0].first;
                int32_t u = s0;
                size_t steps = 0;
                bool ok = true;
                do {
                    if (isv[u]) poly.push_back(u);
                    auto it = std::lower_bound(edges.begin(), edges.end(),
                                               std::pair<int32_t, int32_t>(u, INT32_MIN));
                    if (it == edges.end() || it->first != u || ++steps > edges.size()) {
                        ok = false;
                        break;
                    }
                    u = it->second;
                } while (u != s0);
                const size_t mm = poly.size();
                if (!ok || mm < 3) {
                    bad.store(1);
                    continue;
                }
                const size_t l0 = std::min_element(poly.begin(), poly.end()) - poly.begin();
                for (size_t i = 1; i + 1 < mm; ++i) {
                    out.push_back(poly[l0]);
                    out.push_back(poly[(l0 + i) % mm]);
                    out.push_back(poly[(l0 + i + 1) % mm]);
                }
            }
        });
        if (bad.load()) return false;
        // sorted triples: counting sort on the first vertex, then (b, c)
        // inside each first vertex (a vertex starts few fans)
        std::vector<int32_t> cnt((size_t)n + 1, 0);
        size_t nt = 0;
        for (int t = 0; t < T; ++t) nt += loc_[t].part.size() / 3;
        W.run(T, 1, [&](int64_t lo, int64_t hi, int) {
            for (int64_t t = lo; t < hi; ++t) {
                const std::vector<int32_t> &v = loc_[t].part;
                for (size_t i = 0; i < v.size(); i += 3) __atomic_fetch_add(&cnt[v[i] + 1], 1, __ATOMIC_RELAXED);
            }
        });
        prefix_sum(W, cnt.data(), (int64_t)n + 1);
        tri.resize(3 * nt);
        {
            std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
            W.run(T, 1, [&](int64_t lo, int64_t hi, int) {
                for (int64_t t = lo; t < hi; ++t) {
                    const std::vector<int32_t> &v = loc_[t].part;
                    for (size_t i = 0; i < v.size(); i += 3) {
                        const size_t o = 3 * (size_t)__atomic_fetch_add(&fill[v[i]], 1, __ATOMIC_RELAXED);
                        tri[o] = v[i];
                        tri[o + 1] = v[i + 1];
                        tri[o + 2] = v[i + 2];
                    }
                }
            });
        }
        W.run(n, 1 << 16, [&](int64_t lo, int64_t hi, int) {
            for (int64_t a = lo; a < hi; ++a) {
                const int32_t t0 = cnt[a], t1 = cnt[a + 1];
                for (int32_t i = t0 + 1; i < t1; ++i) {
                    const int32_t b = tri[3 * (size_t)i + 1], c = tri[3 * (size_t)i + 2];
                    int32_t j = i - 1;
                    while (j >= t0 && (tri[3 * (size_t)j + 1] > b ||
                                       (tri[3 * (size_t)j + 1] == b && tri[3 * (size_t)j + 2] > c))) {
                        tri[3 * (size_t)(j + 1) + 1] = tri[3 * (size_t)j + 1];
                        tri[3 * (size_t)(j + 1) + 2] = tri[3 * (size_t)j + 2];
                        --j;
                    }
                    tri[3 * (size_t)(j + 1) + 1] = b;
                    tri[3 * (size_t)(j + 1) + 2] = c;
                }
            }
        });
        return (int64_t)verts.size() >= 4 * hulls && (int64_t)nt == 2 * (int64_t)verts.size() - 4 * hulls;
    }

  private:
    struct Edge {
        int32_t u, w, g;
    };

    bool grow(size_t nf) {
        return F.resize(nf) && lock.resize(nf) && gone.resize(nf) && start.resize(nf) &&
               len.resize(nf) && apex.resize(nf) && apc.resize(nf);
    }

    // per-thread scratch, one cache line apart (kept for its capacity)
    struct alignas(64) Local {
        std::vector<int32_t> reg;   // regions (and their rims), in walk order
        std::vector<int32_t> rim;
        std::vector<Edge> hor;      // horizon edges of accepted regions
        std::vector<std::pair<int32_t, int32_t>> by_u;
        std::vector<int32_t> part;  // output: per-thread lists
        IdSet seen;
    };
    std::vector<Local> loc_;
    const int32_t *region(int64_t i) const { return loc_[rthr_[i]].reg.data() + roff_[i]; }
    std::vector<int16_t> rthr_, hthr_;
    std::vector<int64_t> roff_, hoff_;
    std::vector<int32_t> rcnt_, rall_, hcnt_, scnt_, base_;
    std::vector<int64_t> sbase_;
    std::vector<uint8_t> live_;
    std::vector<int64_t> acc_;
    std::vector<const int32_t *> rptr_;
};

}  // namespace qh3
