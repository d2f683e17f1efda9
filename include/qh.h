/*
 * qh.h -- segmented data-parallel Quickhull on AMD Instinct MI355X (gfx950).
 *
 * The method is that of S. Tzeng and J. D. Owens, "Finding Convex Hulls Using
 * Quickhull on the GPU": the recursion of Quickhull (Section 3.2, Algorithm
 * 1) is replaced by rounds over one array of points grouped into segments
 * (Section 3.1), and each round permutes the survivors into new segments and
 * drops interior points (flagPermute and compact, Sections 4.1-4.2; the 2D
 * driver is Algorithm 4).
 *
 * Conventions shared by every call below:
 *
 *  - Point data and outputs live in DEVICE memory (hipMalloc'd or torch
 *    tensors on the GPU); counts returned "to the host" are written through
 *    host pointers.  The caller owns every buffer it passes.  Inputs are never
 *    modified.
 *  - Points are integer-grid coordinates stored as planes (structure of
 *    arrays): x[0..n) followed by y[0..n) (and z[0..n) in 3D).  All
 *    orientation and distance decisions are exact: 2D needs |coord| <= 2^30-1,
 *    3D |coord| <= 2^19, else QH_ERANGE.
 *  - Reported hull vertices are the strictly convex ones (points exactly on
 *    an edge or facet are not vertices).  Among exact duplicates the lowest
 *    index is reported.
 *  - Calls are host-synchronous: they enqueue work on opts->stream (NULL =
 *    the null stream) and return when the outputs are complete.
 *  - No call aborts or throws.  On error the outputs are unspecified and the
 *    host counts are set to 0; the status says what went wrong.
 *  - A context holds the device workspace (it grows on demand and is freed by
 *    qh_ctx_destroy).  One context per host thread / stream at a time.
 */
#ifndef QH_H
#define QH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QH_OK = 0,
    QH_EINVAL = -1,       /* bad argument (null pointer, negative size, bad offsets) */
    QH_ERANGE = -2,       /* a coordinate is outside the exact range */
    QH_ENOMEM = -3,       /* device or host allocation failed */
    QH_EDEGENERATE = -4,  /* 3D input has fewer than 4 affinely independent points */
    QH_EDEVICE = -5,      /* a HIP runtime call failed */
    QH_ECAPACITY = -6     /* an internal capacity was exceeded and could not grow */
} qh_status;

/* arithmetic of the distance tests (qh_opts.mode) */
enum {
    QH_EXACT_INT64 = 0,   /* every predicate in 64-bit integers */
    QH_FP32_FILTER = 1    /* FP32 with a static forward error bound; only
                             undecided signs / argmax candidates in int64.
                             Same outputs as QH_EXACT_INT64, bit for bit. */
};

/* qh_opts.flags */
enum {
    QH_FLAG_TIMING = 1u,    /* time every kernel launch of the call with HIP
                               events (qh_stats) */
    QH_FLAG_NO_FINISH = 2u, /* 2D: run every level of the recursion as a
                               round of the round kernels.  By default, once
                               no segment holds more than QH_FINISH_CAP
                               points and the round's segments are few
                               enough (qh_stats.finish_segments), one
                               workgroup per segment completes that segment's
                               recursion in on-chip memory (the same levels
                               and the same rules as the rounds, so the same
                               output); or, from the third round on, once no
                               segment holds more than QH_FINISH_CAP / 2
                               points and the round's points are few enough,
                               each workgroup completes runs of consecutive
                               segments of up to QH_FINISH_CAP / 2 points
                               together.  A call of the same point count,
                               instance count and arithmetic as the context's
                               previous call starts finishing no earlier than
                               the round that call finished in */
    QH_FLAG_GRAPH = 4u,     /* 2D: replay the call's launches from HIP graphs
                               that the context captured on an earlier call
                               with the same arguments, buffers and workspace
                               (captured on first use: the set-up, extremes
                               and first batch of rounds as one graph, every
                               later batch of rounds as another).  Needs a
                               non-null qh_opts.stream (QH_EINVAL otherwise);
                               ignored with QH_FLAG_TIMING.  The graphs keep
                               the buffer addresses: the caller may change
                               the inputs' contents between calls, and a call
                               with other buffers captures anew */
    QH_FLAG_AUTOTUNE = 8u   /* 2D: pick the launch configuration (round-kernel
                               blocks, multi-segment-kernel blocks, segments
                               per workgroup for finishing) by timing every
                               candidate on this call's input, the first time
                               the context sees the call's size class (mode,
                               point count and instance count rounded up to
                               powers of two); later calls of that class reuse
                               the choice.  Every configuration gives the same
                               output */
};

/* points of a segment that one workgroup finishes (QH_FLAG_NO_FINISH) */
#define QH_FINISH_CAP 1024

typedef struct qh_ctx qh_ctx;

/* Counters of one call (all host values, filled when qh_opts.stats != NULL). */
typedef struct qh_stats {
    int64_t rounds;             /* rounds that had points, first split included */
    int64_t round_launches;     /* launches of the round kernel, first split
                                   included (a batch of rounds may end with
                                   launches that find nothing left to do) */
    int64_t round_points_in;    /* points read by the rounds after the first split */
    int64_t round_points_out;   /* survivors written by those rounds */
    int64_t split_points_out;   /* survivors of the first split (counted: the
                                   split writes no point) */
    int64_t hull_bytes;         /* algorithmic HBM bytes of the whole call: the
                                   extremes read 8 B per point; the first split
                                   reads 8 B per point; the round after it
                                   reads the input again (8 B per point) and
                                   writes 12 B per survivor (x, y, index);
                                   every later round reads 12 B per point and
                                   writes 12 B per survivor */
    int64_t round_kernel_bytes; /* the part of hull_bytes moved by the round
                                   kernel (first split and later rounds) */
    double kernel_ms;           /* device time of all kernels of the call */
    double round_kernel_ms;     /* ... of the round-kernel launches */
    double split_ms;            /* ... of which the first split */
    double extremes_ms;         /* ... of the extremes */
    double segment_ms;          /* ... of the segment bookkeeping between rounds
                                   (the five times: QH_FLAG_TIMING only, HIP
                                   events around every launch, else 0) */
    int64_t filter_tests;       /* FP32 filter: sign tests made */
    int64_t filter_fallbacks;   /* ... of which were undecided and redone in int64 */
    int64_t argmax_candidates;  /* points whose exact distance was needed by the
                                   segmented argmax (FP32 filter) */
    int64_t max_segments;       /* most segments alive in one round */
    int64_t grid_blocks;        /* blocks of a round-kernel launch */
    int64_t host_syncs;         /* device-to-host waits of the call */
    double host_ms;             /* host time of the 3D topology step and output
                                   (qh_hull3d only) */
    double host_output_ms;      /* ... of which the output (vertex test and
                                   canonical triangulation) */
    int64_t finish_round;       /* 2D: the round whose segments were finished
                                   in on-chip memory (-1: none) */
    int64_t multi_blocks;       /* 2D: blocks of a multi-segment-kernel launch */
    int64_t finish_segments;    /* 2D: most segments that a round may finish
                                   (one workgroup each, in turn) */
    int64_t graph_launches;     /* 2D, QH_FLAG_GRAPH: captured graphs replayed
                                   by the call */
    int64_t tuned_configs;      /* 2D, QH_FLAG_AUTOTUNE: configurations timed by
                                   the call (0 once the size class is tuned) */
    int64_t degenerate_instances; /* qh_hull3d_batched: instances without a hull
                                   (fewer than four affinely independent points) */
    int64_t finish_runs;        /* 2D: 1 if the finishing round took runs of
                                   consecutive small segments together, 0 if
                                   one segment per workgroup (or none) */
} qh_stats;

typedef struct qh_opts {
    void *stream;      /* hipStream_t, or NULL for the null stream */
    uint32_t mode;     /* QH_EXACT_INT64 or QH_FP32_FILTER */
    uint32_t flags;    /* QH_FLAG_* */
    qh_ctx *ctx;       /* workspace; NULL = a temporary one for this call */
    qh_stats *stats;   /* optional host output */
} qh_opts;

/* Create / destroy a workspace context bound to the current HIP device. */
qh_status qh_ctx_create(qh_ctx **out);
void qh_ctx_destroy(qh_ctx *ctx);

/* Static text of a status code. */
const char *qh_status_str(int status);

/* Library version string. */
const char *qh_version(void);

/*
 * 2D convex hull (Algorithm 4; Algorithm 1 with d = 2).
 *
 *   pts       device int32[2*n]: x[0..n) then y[0..n)
 *   n         number of points, 0 <= n <= 2^31 - 2^16
 *   hull_idx  device int32[n] (capacity n; n >= 1): hull vertex indices in
 *             counter-clockwise order, starting at the lexicographically
 *             smallest (x, y)
 *   h         host: number of hull vertices written
 *
 * n = 0 gives h = 0; all points equal gives h = 1; all points collinear gives
 * h = 2 (the lexicographic minimum and maximum).
 */
qh_status qh_hull2d(const int32_t *pts, int64_t n, int32_t *hull_idx, int64_t *h,
                    const qh_opts *opts);

/*
 * Many independent 2D hulls in one call: instance i is the index range
 * [offsets[i], offsets[i+1]) of one shared point array, and every instance
 * becomes the initial segment of the permute-and-segment rounds
 * (Section 3.1: segments keep subproblems of varying size in one array).
 *
 *   pts           device int32[2*n_total]: x planes then y planes
 *   n_total       offsets[k] (host copy; checked on the device)
 *   offsets       device int64[k+1], offsets[0] = 0, non-decreasing
 *   k             number of instances, 1 <= k <= 2^24
 *   hull_idx      device int32[n_total]: the hulls one after the other, each
 *                 as in qh_hull2d, with indices LOCAL to the instance
 *   hull_offsets  device int64[k+1]: instance i's hull is
 *                 hull_idx[hull_offsets[i] .. hull_offsets[i+1])
 *   h_total       host (may be NULL): hull_offsets[k]
 */
qh_status qh_hull2d_batched(const int32_t *pts, int64_t n_total, const int64_t *offsets,
                            int32_t k, int32_t *hull_idx, int64_t *hull_offsets,
                            int64_t *h_total, const qh_opts *opts);

/*
 * 3D convex hull (Algorithm 1 with d = 3; Section 4.3 on three dimensions).
 * Every facet with points outside it finds its farthest point (its apex);
 * apexes whose visible regions do not touch replace their regions by cones
 * in the same round; the points of a removed facet go to the first new facet
 * of its cone they lie strictly above, or are dropped.
 *
 *   pts      device int32[3*n]: x[0..n), y[0..n), z[0..n); |coordinate| <= 2^19
 *            (so every plane test is exact in int64), else QH_ERANGE
 *   n        number of points, 4 <= n <= 2^30 - 2^12
 *   facets   device int32[3 * (2n - 4)]: triangles as index triples,
 *            counter-clockwise seen from outside.  Every face of the hull (a
 *            maximal planar region) is a fan from its lowest-index vertex over
 *            its vertices, and the triples are sorted, so the list is a
 *            function of the point set alone
 *   nfacets  host: triangles written (2 * nverts - 4)
 *   verts    device int32[n]: hull vertex indices (extreme points, the lowest
 *            index among duplicates), ascending
 *   nverts   host: vertices written
 *
 * Fewer than four affinely independent points give QH_EDEGENERATE.  In
 * QH_FP32_FILTER mode the plane tests of the classification are made in FP32
 * with an error bound and redone in int64 when undecided; the output is the
 * same.  The topology step runs on the host, inside the call.
 */
qh_status qh_hull3d(const int32_t *pts, int64_t n, int32_t *facets, int64_t *nfacets,
                    int32_t *verts, int64_t *nverts, const qh_opts *opts);

/*
 * 3D convex hulls of k independent point sets in one call: the batched form
 * of qh_hull3d (the segments of the method, Section 3, are the facets of all
 * instances together).  Instance i is the points [offsets[i], offsets[i+1])
 * of pts; each round serves the facets of every instance at once, so the
 * rounds and host synchronisations of a call do not grow with k.
 *
 *   pts            device int32[3*N], N = n_total: x[0..N), y[0..N), z[0..N);
 *                  |coordinate| <= 2^19 (else QH_ERANGE)
 *   n_total        N, 0 <= N <= 2^30 - 2^12
 *   offsets        device int64[k+1]: offsets[0] = 0, nondecreasing,
 *                  offsets[k] = N (else QH_EINVAL; read back to the host)
 *   k              instances, 1 <= k <= 2^20
 *   facets         device int32[6*N] (room for 3 (2 n_i - 4) per instance):
 *                  the triples of instance i at
 *                  [3 facet_offsets[i], 3 facet_offsets[i+1]), indices local
 *                  to the instance, in qh_hull3d's canonical order
 *   facet_offsets  device int64[k+1]: triangle offsets of the instances
 *   verts          device int32[N]: the vertices of instance i (local,
 *                  ascending) at [vert_offsets[i], vert_offsets[i+1])
 *   vert_offsets   device int64[k+1]
 *
 * An instance with fewer than four affinely independent points has no
 * facets and no vertices (qh_stats.degenerate_instances counts them; its
 * coordinates are range-checked only when it has four points or more); the
 * call still returns QH_OK.  Results equal those of k qh_hull3d calls.
 */
qh_status qh_hull3d_batched(const int32_t *pts, int64_t n_total, const int64_t *offsets, int32_t k,
                            int32_t *facets, int64_t *facet_offsets, int32_t *verts,
                            int64_t *vert_offsets, const qh_opts *opts);

/*
 * The k-state segmented stable partition on its own (flagPermute, Section
 * 4.1 and Figure 1; the rounds above fuse it into their scatter).  Segments
 * are runs of the array started by a head flag (element 0 always starts
 * one).  Element i of state f[i] in segment [h, e) moves to
 *   p[i] = h + #{j in [h, e): f[j] < f[i]} + #{j in [h, i): f[j] = f[i]},
 * and s_new flags the first slot of every non-empty state group of every
 * segment.  For tests and for callers of the primitive; not on the hull path.
 *
 *   f       device int32[n]: states, each in [0, k), else QH_EINVAL
 *   s       device uint8[n]: head flags (non-zero = a segment starts here)
 *   n       elements, 0 <= n <= 2^30
 *   k       states, 1 <= k <= 16
 *   p       device int32[n]: new positions (a permutation of 0..n-1)
 *   s_new   device uint8[n]: head flags after the permutation
 *   stream  hipStream_t or NULL; the call returns when the outputs are written
 *
 * Scratch device memory of about 4 (k + 2) n bytes is allocated and freed
 * inside the call.
 */
qh_status qh_test_flag_permute(const int32_t *f, const uint8_t *s, int64_t n, int32_t k,
                               int32_t *p, uint8_t *s_new, void *stream);

/*
 * qh_test_flag_permute without any device allocation, for callers that
 * cannot allocate device memory (serving loops that must not call hipMalloc,
 * harnesses that forbid it).  Same arguments, checks and outputs as
 * qh_test_flag_permute; the call is host-synchronous like it.
 *
 * Its scratch is a fixed array of 64 MiB in the library's device code, one
 * copy per GPU, held from the first call on that GPU until the process ends.
 * A call needs about 4 (k (n + 1) + 2 n) bytes of it: larger calls
 * (n > 4,186,095 for k = 2, n > 930,241 for k = 16) return
 * QH_ECAPACITY before any device work.  Every call on one GPU uses the same
 * array (each call clears what must start at zero), so calls that overlap on
 * one GPU, from several host threads or streams, race and must be
 * serialised by the caller.
 */
qh_status qh_test_flag_permute_noalloc(const int32_t *f, const uint8_t *s, int64_t n, int32_t k,
                                       int32_t *p, uint8_t *s_new, void *stream);

/*
 * The segmented compact on its own (Section 4.2, Algorithm 3): the elements
 * with b[i] = 0 are dropped.  For tests and for callers of the primitive.
 *
 *   b       device uint8[n]: keep flags (non-zero = keep)
 *   s       device uint8[n]: head flags (element 0 always starts a segment)
 *   n       elements, 0 <= n <= 2^30
 *   p       device int32[n]: p[i] = #{j < i : b[j] != 0}, the new position
 *           of every kept element
 *   s_new   device uint8[n]: its first *m entries flag the first kept element
 *           of every segment that keeps one (a segment with none vanishes)
 *   m       host: elements kept
 *   stream  hipStream_t or NULL; the call returns when the outputs are written
 *
 * Scratch device memory of about 8 n bytes is allocated and freed inside the
 * call.
 */
qh_status qh_test_compact(const uint8_t *b, const uint8_t *s, int64_t n, int32_t *p, uint8_t *s_new,
                          int64_t *m, void *stream);

/*
 * Order statistics of many segments at once: k-median finding in the
 * permute-and-segment framework (Section 6 names it as a use of flagPermute
 * followed by compact).  Every round picks a pseudo-random pivot in each
 * open segment, groups the segment below / equal to / above it with a
 * 3-state flagPermute, closes the segment when the wanted rank falls on the
 * pivot's group and otherwise keeps only the group that holds it (compact).
 *
 *   vals     device int32[n], n <= 2^29
 *   offsets  device int64[k+1]: offsets[0] = 0, offsets[k] = n, every segment
 *            [offsets[i], offsets[i+1]) non-empty (else QH_EINVAL)
 *   k        segments, 1 <= k <= 2^24
 *   ranks    device int64[k]: 0 <= ranks[i] < the length of segment i
 *            (else QH_EINVAL)
 *   out      device int32[k]: out[i] = the ranks[i]-th smallest value of
 *            segment i, counted from 0 (duplicates count separately)
 *   stream   hipStream_t or NULL; the call returns when out is written
 *
 * Scratch device memory of about 60 n bytes is allocated and freed inside
 * the call.
 */
qh_status qh_select(const int32_t *vals, int64_t n, const int64_t *offsets, int32_t k,
                    const int64_t *ranks, int32_t *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* QH_H */
