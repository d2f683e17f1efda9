/*
 * oracle/qh_oracle.c -- plain, slow, obviously correct CPU Quickhull.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the HIP path is
 * compared against.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it; the library never does.  It shares no code,
 * header, table or helper with the HIP path.
 *
 * What it computes (Tzeng & Owens, "Finding Convex Hulls Using Quickhull on
 * the GPU", Section 3.2 and Algorithm 1; the 2D driver of Algorithm 4):
 *
 *   First split: a = lexicographic minimum of (x, y), b = lexicographic
 *   maximum (lowest index among exact duplicates for both).  Points strictly
 *   to one side of the line ab form one set, points strictly to the other side
 *   the other set; points on the line are dropped.
 *
 *   Recursive step, for a set S outside the directed edge u->v: the point f
 *   of S farthest from the line uv is a hull vertex.  Points of S inside or on
 *   the triangle (u, f, v) are dropped; the others go to the set of the one
 *   new edge (u->f or f->v) they are strictly outside of.
 *
 * Distances are the unnormalised cross products (the Euclidean distance to a
 * fixed line times the fixed edge length, so the argmax is the same), taken
 * in 128-bit integers, so every decision is exact.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *  - "extrema along x" is the lexicographic (x, y) order, ties by lowest index;
 *  - a point exactly on an edge line is not outside it (only strictly convex
 *    vertices are reported);
 *  - the farthest point is the maximum of the key
 *      (distance descending, t = (p - u).(v - u) ascending, index ascending),
 *    which selects an endpoint of any set of equally far collinear points and
 *    the lowest index among exact duplicates;
 *  - the output is the list of hull vertex indices in counter-clockwise order
 *    starting at a.
 *
 * The recursion is run with an explicit stack, so its depth is not bounded by
 * the C stack.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

/* signed area test: (p - u) x (v - u).  > 0 means p lies strictly to the
 * right of the directed line u -> v, i.e. strictly outside a counter-clockwise
 * hull edge u -> v. */
static i128 side2(const int32_t *x, const int32_t *y, int64_t u, int64_t v, int64_t p)
{
    i128 dx = (i128)x[p] - x[u], dy = (i128)y[p] - y[u];
    i128 ex = (i128)x[v] - x[u], ey = (i128)y[v] - y[u];
    return dx * ey - dy * ex;
}

static i128 along2(const int32_t *x, const int32_t *y, int64_t u, int64_t v, int64_t p)
{
    i128 dx = (i128)x[p] - x[u], dy = (i128)y[p] - y[u];
    i128 ex = (i128)x[v] - x[u], ey = (i128)y[v] - y[u];
    return dx * ex + dy * ey;
}

/* lexicographic comparison of points i and j by (x, y); 0 if equal */
static int lexcmp2(const int32_t *x, const int32_t *y, int64_t i, int64_t j)
{
    if (x[i] != x[j]) return x[i] < x[j] ? -1 : 1;
    if (y[i] != y[j]) return y[i] < y[j] ? -1 : 1;
    return 0;
}

/* one pending piece of work of the recursion */
typedef struct {
    int kind;        /* 0 = hull edge u->v with its outside set, 1 = emit vertex u */
    int64_t u, v;
    int64_t *set;    /* owned; NULL when empty */
    int64_t nset;
} frame2;

typedef struct {
    frame2 *f;
    int64_t n, cap;
} stack2;

static int push2(stack2 *s, frame2 fr)
{
    if (s->n == s->cap) {
        int64_t nc = s->cap ? 2 * s->cap : 64;
        frame2 *nf = (frame2 *)realloc(s->f, (size_t)nc * sizeof(frame2));
        if (!nf) return -1;
        s->f = nf;
        s->cap = nc;
    }
    s->f[s->n++] = fr;
    return 0;
}

/*
 * Convex hull of the points (x[i], y[i]), i in [0, n).
 * Writes the hull vertex indices in counter-clockwise order starting at the
 * lexicographic minimum to out[] (capacity n) and returns their number, or
 * -1 when memory runs out.
 */
int64_t qho_hull2d(const int32_t *x, const int32_t *y, int64_t n, int32_t *out)
{
    if (n <= 0) return 0;

    /* first split: extrema */
    int64_t a = 0, b = 0;
    for (int64_t i = 1; i < n; ++i) {
        if (lexcmp2(x, y, i, a) < 0) a = i;
        if (lexcmp2(x, y, i, b) > 0) b = i;
    }
    if (lexcmp2(x, y, a, b) == 0) {
        out[0] = (int32_t)a;
        return 1;
    }

    /* the two sides of the line ab */
    int64_t *below = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *above = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!below || !above) { free(below); free(above); return -1; }
    int64_t nb = 0, na = 0;
    for (int64_t i = 0; i < n; ++i) {
        i128 d = side2(x, y, a, b, i);
        if (d > 0) below[nb++] = i;       /* outside edge a->b */
        else if (d < 0) above[na++] = i;  /* outside edge b->a */
    }

    stack2 st = {0};
    int64_t h = 0;
    int bad = 0;
    /* pushed in reverse: a, (edge a->b), b, (edge b->a) */
    frame2 f4 = {0, b, a, above, na};
    frame2 f3 = {1, b, b, NULL, 0};
    frame2 f2 = {0, a, b, below, nb};
    frame2 f1 = {1, a, a, NULL, 0};
    if (push2(&st, f4) || push2(&st, f3) || push2(&st, f2) || push2(&st, f1)) bad = 1;

    while (!bad && st.n > 0) {
        frame2 fr = st.f[--st.n];
        if (fr.kind == 1) {
            out[h++] = (int32_t)fr.u;
            continue;
        }
        if (fr.nset == 0) {
            free(fr.set);
            continue;
        }
        int64_t u = fr.u, v = fr.v;
        /* farthest point: max of (distance, -t, -index) */
        int64_t f = fr.set[0];
        i128 fd = side2(x, y, u, v, f), ft = along2(x, y, u, v, f);
        for (int64_t k = 1; k < fr.nset; ++k) {
            int64_t p = fr.set[k];
            i128 d = side2(x, y, u, v, p);
            if (d < fd) continue;
            i128 t = along2(x, y, u, v, p);
            if (d > fd || t < ft || (t == ft && p < f)) {
                f = p;
                fd = d;
                ft = t;
            }
        }
        /* split the set by the two new edges u->f and f->v */
        int64_t *s0 = (int64_t *)malloc((size_t)fr.nset * sizeof(int64_t));
        int64_t *s1 = (int64_t *)malloc((size_t)fr.nset * sizeof(int64_t));
        if (!s0 || !s1) { free(s0); free(s1); free(fr.set); bad = 1; break; }
        int64_t n0 = 0, n1 = 0;
        for (int64_t k = 0; k < fr.nset; ++k) {
            int64_t p = fr.set[k];
            if (side2(x, y, u, f, p) > 0) s0[n0++] = p;
            else if (side2(x, y, f, v, p) > 0) s1[n1++] = p;
            /* else: inside or on the triangle (u, f, v): dropped */
        }
        free(fr.set);
        frame2 c1 = {0, f, v, s1, n1};
        frame2 cf = {1, f, f, NULL, 0};
        frame2 c0 = {0, u, f, s0, n0};
        if (push2(&st, c1) || push2(&st, cf) || push2(&st, c0)) { bad = 1; break; }
    }
    for (int64_t k = 0; k < st.n; ++k) free(st.f[k].set);
    free(st.f);
    return bad ? -1 : h;
}

/*
 * Many independent hulls: instance i is the index range
 * [offsets[i], offsets[i+1]).  Its hull (indices local to the instance) goes
 * to out[out_offsets[i] .. out_offsets[i+1]); out_offsets[0] = 0.
 */
int64_t qho_hull2d_batched(const int32_t *x, const int32_t *y, const int64_t *offsets,
                           int64_t k, int32_t *out, int64_t *out_offsets)
{
    out_offsets[0] = 0;
    for (int64_t i = 0; i < k; ++i) {
        int64_t lo = offsets[i], hi = offsets[i + 1];
        int64_t h = qho_hull2d(x + lo, y + lo, hi - lo, out + out_offsets[i]);
        if (h < 0) return -1;
        out_offsets[i + 1] = out_offsets[i] + h;
    }
    return out_offsets[k];
}
