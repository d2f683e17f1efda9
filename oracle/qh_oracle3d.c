/*
 * oracle/qh_oracle3d.c -- plain, slow, obviously correct CPU Quickhull in 3D.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the HIP 3D path is
 * compared against.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it; the library never does.  It shares no code,
 * header, table or helper with the HIP path.
 *
 * What it computes (Tzeng & Owens, Section 3.2 and Algorithm 1 in three
 * dimensions, with the facet-by-facet bookkeeping of Barber, Dobkin and
 * Huhdanpaa's Quickhull, which the paper cites for its CPU comparison):
 *
 *   Start: a = lexicographic minimum of (x, y, z), b = lexicographic maximum
 *   (lowest index among exact duplicates).  c = the point farthest from the
 *   line ab, d = the point farthest from the plane abc (either side).  The
 *   tetrahedron abcd has four facets, each oriented so that the opposite
 *   corner is strictly below it.  Every point goes to the outside set of the
 *   first facet (lowest id) it is strictly above; the others are dropped.
 *
 *   Step, for the alive facet F of lowest id with a non-empty outside set:
 *   the apex p = the point of F's outside set farthest above F.  The facets
 *   p is strictly above (found by a walk over facet neighbours from F) are
 *   removed; every edge between a removed and a kept facet (the horizon) gets
 *   a new facet (edge, p).  The points of the removed facets' outside sets go
 *   to the first new facet they are strictly above, or are dropped (they lie
 *   in the hull of the old hull and p).
 *
 *   Output: the surface that is left can hold corners that are not extreme
 *   points (a later apex coplanar with a face leaves it in place).  A corner is
 *   a hull vertex iff its facets span at least three distinct planes.  Each
 *   face (a maximal edge-connected set of coplanar facets) is then
 *   triangulated again as a fan from its lowest-index vertex, counter-clockwise
 *   seen from outside, over its vertices only.  So the facet list is a
 *   function of the point set alone: the canonical triangulation.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *  - the first split is a tetrahedron: a flat double-sided triangle would drop
 *    an extreme point coplanar with it but outside it;
 *  - the recursion removes every facet the apex sees and adds one facet per
 *    horizon edge: a facet-by-facet simplex split is only correct when the
 *    apex sees its own facet alone;
 *  - a point exactly on a facet plane is not above it;
 *  - c maximises |(b - a) x (p - a)|^2, then minimises (p - a).(b - a), then
 *    the index; d maximises |n_abc . (p - a)|, then minimises (p - a).(b - a),
 *    then (p - a).(c - a), then the index; the apex of facet (a, b, c)
 *    maximises n . (p - a), then minimises (p - a).(b - a), then
 *    (p - a).(c - a), then the index.  Each rule selects an extreme point of
 *    its tie set, and the lowest index among exact duplicates.
 *
 * Every predicate is taken in 128-bit integers, so every decision is exact
 * for any int32 coordinates.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

enum { QHO_OK = 0, QHO_ENOMEM = -1, QHO_EDEGENERATE = -4 };

typedef struct {
    const int32_t *x, *y, *z;
} pts3;

typedef struct {
    int32_t v[3];   /* corners, counter-clockwise seen from outside */
    int32_t nb[3];  /* facet across the edge v[i] -> v[i+1] */
    int alive;
    i128 n[3];      /* outward normal (v1 - v0) x (v2 - v0) */
    int64_t *out;   /* outside set (point indices) */
    int64_t nout, capout;
} facet3;

typedef struct {
    facet3 *f;
    int64_t n, cap;
} facets3;

static void sub3(const pts3 *P, int64_t p, int64_t q, i128 r[3])
{
    r[0] = (i128)P->x[p] - P->x[q];
    r[1] = (i128)P->y[p] - P->y[q];
    r[2] = (i128)P->z[p] - P->z[q];
}

static void cross3(const i128 a[3], const i128 b[3], i128 r[3])
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

static i128 dot3(const i128 a[3], const i128 b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static int lexcmp3(const pts3 *P, int64_t i, int64_t j)
{
    if (P->x[i] != P->x[j]) return P->x[i] < P->x[j] ? -1 : 1;
    if (P->y[i] != P->y[j]) return P->y[i] < P->y[j] ? -1 : 1;
    if (P->z[i] != P->z[j]) return P->z[i] < P->z[j] ? -1 : 1;
    return 0;
}

/* signed distance of p above facet f (times |n|) */
static i128 above(const pts3 *P, const facet3 *f, int64_t p)
{
    i128 d[3];
    sub3(P, p, f->v[0], d);
    return dot3(f->n, d);
}

static int add_out(facet3 *f, int64_t p)
{
    if (f->nout == f->capout) {
        int64_t nc = f->capout ? 2 * f->capout : 8;
        int64_t *no = (int64_t *)realloc(f->out, (size_t)nc * sizeof(int64_t));
        if (!no) return -1;
        f->out = no;
        f->capout = nc;
    }
    f->out[f->nout++] = p;
    return 0;
}

/* append facet (a, b, c); returns its id or -1 */
static int64_t new_facet(facets3 *F, const pts3 *P, int32_t a, int32_t b, int32_t c)
{
    if (F->n == F->cap) {
        int64_t nc = F->cap ? 2 * F->cap : 64;
        facet3 *nf = (facet3 *)realloc(F->f, (size_t)nc * sizeof(facet3));
        if (!nf) return -1;
        F->f = nf;
        F->cap = nc;
    }
    facet3 *f = &F->f[F->n];
    memset(f, 0, sizeof(*f));
    f->v[0] = a;
    f->v[1] = b;
    f->v[2] = c;
    f->nb[0] = f->nb[1] = f->nb[2] = -1;
    f->alive = 1;
    i128 e1[3], e2[3];
    sub3(P, b, a, e1);
    sub3(P, c, a, e2);
    cross3(e1, e2, f->n);
    return F->n++;
}

/* is the key of p better than the key of q for the apex of facet f?
 * key: (n.(p - a) descending, (p - a).(b - a) ascending,
 *       (p - a).(c - a) ascending, index ascending) */
static int apex_better(const pts3 *P, const facet3 *f, int64_t p, int64_t q)
{
    i128 dp = above(P, f, p), dq = above(P, f, q);
    if (dp != dq) return dp > dq;
    i128 eb[3], ec[3], rp[3], rq[3];
    sub3(P, f->v[1], f->v[0], eb);
    sub3(P, f->v[2], f->v[0], ec);
    sub3(P, p, f->v[0], rp);
    sub3(P, q, f->v[0], rq);
    i128 tp = dot3(rp, eb), tq = dot3(rq, eb);
    if (tp != tq) return tp < tq;
    tp = dot3(rp, ec);
    tq = dot3(rq, ec);
    if (tp != tq) return tp < tq;
    return p < q;
}

static int same_plane(const facet3 *f, const facet3 *g)
{
    i128 c[3];
    cross3(f->n, g->n, c);
    return c[0] == 0 && c[1] == 0 && c[2] == 0 && dot3(f->n, g->n) > 0;
}

static int64_t uf_find(int64_t *par, int64_t i)
{
    while (par[i] != i) {
        par[i] = par[par[i]];
        i = par[i];
    }
    return i;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int cmp_tri(const void *a, const void *b)
{
    const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
    for (int i = 0; i < 3; ++i)
        if (x[i] != y[i]) return x[i] < y[i] ? -1 : 1;
    return 0;
}

/*
 * Hull of (x[i], y[i], z[i]), i in [0, n).
 * facets: capacity 3 * max(2n - 4, 4) int32; receives the canonical
 *   triangulation (triples sorted lexicographically), *nfacets triples.
 * verts: capacity n; receives the hull vertex indices in ascending order.
 * Returns 0, -1 (out of memory) or -4 (fewer than four affinely independent
 * points; the outputs are then empty).
 */
int qho_hull3d(const int32_t *x, const int32_t *y, const int32_t *z, int64_t n,
               int32_t *facets, int64_t *nfacets, int32_t *verts, int64_t *nverts)
{
    *nfacets = 0;
    *nverts = 0;
    if (n < 4) return QHO_EDEGENERATE;
    pts3 P = {x, y, z};

    /* a, b: lexicographic extremes, lowest index among duplicates */
    int64_t a = 0, b = 0;
    for (int64_t i = 1; i < n; ++i) {
        if (lexcmp3(&P, i, a) < 0) a = i;
        if (lexcmp3(&P, i, b) > 0) b = i;
    }
    if (lexcmp3(&P, a, b) == 0) return QHO_EDEGENERATE;

    /* c: farthest from the line ab */
    i128 ab[3];
    sub3(&P, b, a, ab);
    int64_t c = -1;
    i128 cq = 0, ct = 0;
    for (int64_t i = 0; i < n; ++i) {
        i128 r[3], w[3];
        sub3(&P, i, a, r);
        cross3(ab, r, w);
        i128 q = dot3(w, w), t = dot3(r, ab);
        if (q == 0) continue;
        if (c < 0 || q > cq || (q == cq && (t < ct || (t == ct && i < c)))) {
            c = i;
            cq = q;
            ct = t;
        }
    }
    if (c < 0) return QHO_EDEGENERATE;

    /* d: farthest from the plane abc, either side */
    i128 ac[3], nabc[3];
    sub3(&P, c, a, ac);
    cross3(ab, ac, nabc);
    int64_t d = -1;
    i128 dd = 0, dt = 0, du = 0;
    for (int64_t i = 0; i < n; ++i) {
        i128 r[3];
        sub3(&P, i, a, r);
        i128 s = dot3(nabc, r);
        if (s < 0) s = -s;
        if (s == 0) continue;
        i128 t = dot3(r, ab), u = dot3(r, ac);
        if (d < 0 || s > dd || (s == dd && (t < dt || (t == dt && (u < du || (u == du && i < d)))))) {
            d = i;
            dd = s;
            dt = t;
            du = u;
        }
    }
    if (d < 0) return QHO_EDEGENERATE;

    facets3 F = {0};
    int rc = QHO_OK;
    int32_t *cone_from = NULL, *stamp = NULL, *bfs = NULL, *hz = NULL;
    int64_t stamp_cap = 0, bfs_cap = 0;

    /* the tetrahedron: each facet oriented away from the opposite corner */
    {
        int32_t T[4] = {(int32_t)a, (int32_t)b, (int32_t)c, (int32_t)d};
        static const int tri[4][4] = {{0, 1, 2, 3}, {0, 1, 3, 2}, {0, 2, 3, 1}, {1, 2, 3, 0}};
        for (int k = 0; k < 4; ++k) {
            int32_t p = T[tri[k][0]], q = T[tri[k][1]], r = T[tri[k][2]], s = T[tri[k][3]];
            int64_t id = new_facet(&F, &P, p, q, r);
            if (id < 0) { rc = QHO_ENOMEM; goto done; }
            if (above(&P, &F.f[id], s) > 0) {
                F.n--;
                id = new_facet(&F, &P, p, r, q);
            }
        }
        /* neighbours: the facet holding the reversed edge */
        for (int k = 0; k < 4; ++k)
            for (int i = 0; i < 3; ++i) {
                int32_t u = F.f[k].v[i], w = F.f[k].v[(i + 1) % 3];
                for (int g = 0; g < 4; ++g)
                    for (int j = 0; j < 3; ++j)
                        if (g != k && F.f[g].v[j] == w && F.f[g].v[(j + 1) % 3] == u) F.f[k].nb[i] = g;
            }
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < 4; ++k)
                if (above(&P, &F.f[k], i) > 0) {
                    if (add_out(&F.f[k], i)) { rc = QHO_ENOMEM; goto done; }
                    break;
                }
    }

    cone_from = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!cone_from) { rc = QHO_ENOMEM; goto done; }
    for (int64_t i = 0; i < n; ++i) cone_from[i] = -1;

    /* facets are processed in id order; a facet's outside set is fixed when
     * it is made, and new facets get higher ids, so one pass suffices */
    for (int64_t cur = 0; cur < F.n; ++cur) {
        if (!F.f[cur].alive || F.f[cur].nout == 0) continue;
        facet3 *f0 = &F.f[cur];
        int64_t p = f0->out[0];
        for (int64_t k = 1; k < f0->nout; ++k)
            if (apex_better(&P, f0, f0->out[k], p)) p = f0->out[k];

        /* visible facets: walk from cur over neighbours strictly below p */
        if (stamp_cap < F.n) {
            int64_t nc = 2 * F.n + 64;
            int32_t *ns = (int32_t *)realloc(stamp, (size_t)nc * sizeof(int32_t));
            if (!ns) { rc = QHO_ENOMEM; goto done; }
            for (int64_t i = stamp_cap; i < nc; ++i) ns[i] = 0;
            stamp = ns;
            stamp_cap = nc;
        }
        if (bfs_cap < F.n) {
            int64_t nc = 2 * F.n + 64;
            int32_t *nq = (int32_t *)realloc(bfs, (size_t)nc * sizeof(int32_t));
            int32_t *nh = (int32_t *)realloc(hz, (size_t)nc * 3 * sizeof(int32_t));
            if (nq) bfs = nq;
            if (nh) hz = nh;
            if (!nq || !nh) { rc = QHO_ENOMEM; goto done; }
            bfs_cap = nc;
        }
        /* stamp: 1 = visible, 2 = seen and not visible (reset afterwards) */
        int64_t nv = 0, head = 0;
        bfs[nv++] = (int32_t)cur;
        stamp[cur] = 1;
        int64_t nseen = 0;
        while (head < nv) {
            facet3 *f = &F.f[bfs[head++]];
            for (int i = 0; i < 3; ++i) {
                int32_t g = f->nb[i];
                if (stamp[g]) continue;
                if (above(&P, &F.f[g], p) > 0) {
                    stamp[g] = 1;
                    bfs[nv++] = g;
                } else {
                    stamp[g] = 2;
                    hz[3 * nseen] = g;  /* remembered only to reset the stamp */
                    nseen++;
                }
            }
        }
        for (int64_t k = 0; k < nseen; ++k) stamp[hz[3 * k]] = 0;

        /* horizon edges in walk order: (u, w) of a visible facet whose
         * neighbour across it is not visible */
        int64_t nh = 0;
        for (int64_t k = 0; k < nv; ++k) {
            facet3 *f = &F.f[bfs[k]];
            for (int i = 0; i < 3; ++i) {
                int32_t g = f->nb[i];
                if (stamp[g] == 1) continue;
                hz[3 * nh + 0] = f->v[i];
                hz[3 * nh + 1] = f->v[(i + 1) % 3];
                hz[3 * nh + 2] = g;
                nh++;
            }
        }
        /* the cone */
        int64_t first = F.n;
        for (int64_t k = 0; k < nh; ++k) {
            int32_t u = hz[3 * k], w = hz[3 * k + 1], g = hz[3 * k + 2];
            int64_t id = new_facet(&F, &P, u, w, (int32_t)p);
            if (id < 0) { rc = QHO_ENOMEM; goto done; }
            F.f[id].nb[0] = g;
            for (int j = 0; j < 3; ++j)
                if (F.f[g].v[j] == w && F.f[g].v[(j + 1) % 3] == u) F.f[g].nb[j] = (int32_t)id;
            cone_from[u] = (int32_t)id;
        }
        for (int64_t id = first; id < F.n; ++id) {
            facet3 *f = &F.f[id];
            int32_t u = f->v[0], w = f->v[1];
            f->nb[1] = cone_from[w];           /* the cone facet starting at w holds p -> w */
            F.f[cone_from[w]].nb[2] = (int32_t)id;  /* ... and its edge p -> w is our w -> p */
            (void)u;
        }
        /* the visible facets die; their points move to the cone or drop */
        for (int64_t k = 0; k < nv; ++k) {
            facet3 *f = &F.f[bfs[k]];
            f->alive = 0;
            stamp[bfs[k]] = 0;
            for (int64_t m = 0; m < f->nout; ++m) {
                int64_t q = f->out[m];
                if (q == p) continue;
                for (int64_t id = first; id < F.n; ++id)
                    if (above(&P, &F.f[id], q) > 0) {
                        if (add_out(&F.f[id], q)) { rc = QHO_ENOMEM; goto done; }
                        break;
                    }
            }
            free(f->out);
            f->out = NULL;
            f->nout = f->capout = 0;
        }
        for (int64_t id = first; id < F.n; ++id) cone_from[F.f[id].v[0]] = -1;
    }

    /* hull vertices: corners whose facets span at least three planes */
    {
        int64_t nf = F.n;
        int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
        if (!deg) { rc = QHO_ENOMEM; goto done; }
        for (int64_t k = 0; k < nf; ++k)
            if (F.f[k].alive)
                for (int i = 0; i < 3; ++i) deg[F.f[k].v[i] + 1]++;
        for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
        int64_t *inc = (int64_t *)malloc((size_t)(deg[n] + 1) * sizeof(int64_t));
        int64_t *fill = (int64_t *)calloc((size_t)n, sizeof(int64_t));
        char *isv = (char *)calloc((size_t)n, 1);
        int64_t *par = (int64_t *)malloc((size_t)(nf + 1) * sizeof(int64_t));
        int32_t *nxt = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        if (!inc || !fill || !isv || !par || !nxt) {
            free(deg); free(inc); free(fill); free(isv); free(par); free(nxt);
            rc = QHO_ENOMEM;
            goto done;
        }
        for (int64_t k = 0; k < nf; ++k)
            if (F.f[k].alive)
                for (int i = 0; i < 3; ++i) {
                    int32_t v = F.f[k].v[i];
                    inc[deg[v] + fill[v]++] = k;
                }
        int64_t nvert = 0;
        for (int64_t v = 0; v < n; ++v) {
            int64_t lo = deg[v], hi = deg[v + 1];
            if (hi == lo) continue;
            /* distinct planes among the incident facets (stop at three) */
            int64_t rep[3];
            int nrep = 0;
            for (int64_t k = lo; k < hi && nrep < 3; ++k) {
                int fresh = 1;
                for (int r = 0; r < nrep; ++r)
                    if (same_plane(&F.f[inc[k]], &F.f[rep[r]])) { fresh = 0; break; }
                if (fresh) rep[nrep++] = inc[k];
            }
            if (nrep >= 3) {
                isv[v] = 1;
                verts[nvert++] = (int32_t)v;
            }
        }
        *nverts = nvert;

        /* faces: facets joined across edges lying in one plane */
        for (int64_t k = 0; k < nf; ++k) par[k] = k;
        for (int64_t k = 0; k < nf; ++k) {
            if (!F.f[k].alive) continue;
            for (int i = 0; i < 3; ++i) {
                int32_t g = F.f[k].nb[i];
                if (same_plane(&F.f[k], &F.f[g])) {
                    int64_t r1 = uf_find(par, k), r2 = uf_find(par, g);
                    if (r1 != r2) par[r1 < r2 ? r2 : r1] = r1 < r2 ? r1 : r2;
                }
            }
        }
        /* each face: its boundary cycle, counter-clockwise from outside, kept
         * to its vertices, fanned from the lowest index.  Faces are handled
         * one at a time through the facets sorted by face root. */
        int64_t *ord = (int64_t *)malloc((size_t)(nf + 1) * sizeof(int64_t));
        int64_t *cnt = (int64_t *)calloc((size_t)nf + 1, sizeof(int64_t));
        int32_t *poly = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        if (!ord || !cnt || !poly) {
            free(deg); free(inc); free(fill); free(isv); free(par); free(nxt);
            free(ord); free(cnt); free(poly);
            rc = QHO_ENOMEM;
            goto done;
        }
        for (int64_t k = 0; k < nf; ++k)
            if (F.f[k].alive) cnt[uf_find(par, k) + 1]++;
        for (int64_t k = 0; k < nf; ++k) cnt[k + 1] += cnt[k];
        for (int64_t k = 0; k < nf; ++k)
            if (F.f[k].alive) {
                int64_t r = uf_find(par, k);
                ord[cnt[r]++] = k;
            }
        /* cnt[r] is now the end of face r; the start is the previous end */
        for (int64_t i = 0; i < n; ++i) nxt[i] = -1;
        int64_t nt = 0, pos = 0;
        while (pos < deg[n] / 3) {
            int64_t r = uf_find(par, ord[pos]);
            int64_t end = pos;
            while (end < deg[n] / 3 && uf_find(par, ord[end]) == r) end++;
            int32_t start = -1;
            for (int64_t q = pos; q < end; ++q) {
                facet3 *f = &F.f[ord[q]];
                for (int i = 0; i < 3; ++i) {
                    int32_t g = f->nb[i];
                    if (uf_find(par, g) == r) continue;
                    int32_t u = f->v[i], w = f->v[(i + 1) % 3];
                    nxt[u] = w;
                    if (start < 0 || u < start) start = u;
                }
            }
            int64_t m = 0;
            int32_t u = start;
            do {
                if (isv[u]) poly[m++] = u;
                int32_t w = nxt[u];
                nxt[u] = -1;
                u = w;
            } while (u != start && u >= 0 && m <= n);
            /* rotate to the lowest index, keeping the cyclic order */
            int64_t lo = 0;
            for (int64_t i = 1; i < m; ++i)
                if (poly[i] < poly[lo]) lo = i;
            for (int64_t i = 1; i + 1 < m; ++i) {
                facets[3 * nt + 0] = poly[lo];
                facets[3 * nt + 1] = poly[(lo + i) % m];
                facets[3 * nt + 2] = poly[(lo + i + 1) % m];
                nt++;
            }
            pos = end;
        }
        qsort(facets, (size_t)nt, 3 * sizeof(int32_t), cmp_tri);
        qsort(verts, (size_t)nvert, sizeof(int32_t), cmp_i32);
        *nfacets = nt;
        free(deg); free(inc); free(fill); free(isv); free(par); free(nxt);
        free(ord); free(cnt); free(poly);
    }

done:
    for (int64_t k = 0; k < F.n; ++k) free(F.f[k].out);
    free(F.f);
    free(cone_from);
    free(stamp);
    free(bfs);
    free(hz);
    return rc;
}
