/*
 * hfcr.h -- C ABI of the MI355X (gfx950) history-free collision response
 * library (libhfcr.so).
 *
 * The library separates two penetrating triangle meshes, at least one of
 * which is oriented, following J. Ye, "History-free Collision Response for
 * Deformable Surfaces" (arXiv 1409.2081):
 *
 *   1. discrete collision detection finds every edge-face (E-F) intersection
 *      between the edges of one mesh and the triangles of the oriented one
 *      (Section 3; Section 4, decomposition of F-F into E-F penetrations);
 *   2. each intersecting edge yields a penetration stencil {x0; x1, x2, x3}:
 *      its endpoint x0 behind the oriented face and the face's three
 *      vertices; equal stencils are merged (Section 4, Fig. 3);
 *   3. every stencil is the constraint D(x) = n . [x0 - (x1 + x2 + x3)/3]
 *      with the face's unit normal n (Eq. 1) and gradient
 *      (n, -n/3, -n/3, -n/3) (Eq. 2);
 *   4. stencils that share vertices form impact zones; each zone solves
 *      grad(D) M^-1 grad(D)^T lambda = grad(D) x - d (Eq. 7, Eq. 8) and moves
 *      its vertices by x' = x - M^-1 grad(D)^T lambda (Eq. 5), the minimum
 *      mass-weighted displacement that puts every x0 at distance d in front
 *      of its face (Eq. 3);
 *   5. detection and response repeat until no E-F intersection is left
 *      (Section 3).
 *
 * Conventions shared by every entry point
 *   Orientation   a triangle (a, b, c) is oriented counter-clockwise seen
 *                 from its front: the right-hand normal (b - a) x (c - a)
 *                 points to the legal side.
 *   Directions    direction 0 tests the edges of mesh A against the faces of
 *                 mesh B (B oriented); direction 1 tests the edges of B
 *                 against the faces of A (A oriented).  HFCR_ORIENT_B uses
 *                 direction 0, HFCR_ORIENT_A direction 1, HFCR_ORIENT_BOTH
 *                 both (by default alternating between rounds, Section 4:
 *                 both oriented meshes take the oriented role in turn).
 *   Hit test      edge {p, q} hits triangle (a, b, c) iff p and q lie
 *                 strictly on opposite sides of the triangle's plane and
 *                 the line pq passes through the closed triangle; the sign
 *                 of every orientation determinant is decided exactly.
 *   Memory        every array argument marked "device" is a device pointer
 *                 on the context's GPU, owned by the caller, which must keep
 *                 it alive until the call's stream work completes.  Inputs
 *                 are read-only.  Host-side structs are read during the
 *                 call only.  The library owns only its internal workspace.
 *   Streams       `stream` is a hipStream_t (NULL = the default stream).
 *                 Work is ordered on that stream; the calls below return
 *                 after the results are written (they synchronise the
 *                 stream because the repair loop's length depends on the
 *                 data).
 *   Errors        every entry point returns an hfcr_status; nothing is
 *                 thrown across the ABI.  hfcr_last_error() gives a message.
 *   Threads       a context may be used by one host thread at a time.
 */
#ifndef HFCR_H
#define HFCR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HFCR_OK = 0,
  HFCR_NOT_CONVERGED = 1, /* max_rounds responses made, hits remain        */
  HFCR_PENDING = 2,       /* hfcr_server_wait: not finished within the wait  */
  HFCR_E_INVALID = -1,    /* bad argument, index out of range, non-finite
                             or out-of-domain coordinate                    */
  HFCR_E_CAPACITY = -2,   /* a caller output list was too short; stats hold
                             the required counts, positions are valid       */
  HFCR_E_OOM = -3,        /* device allocation failed                       */
  HFCR_E_DEVICE = -4,     /* a HIP runtime call failed                      */
  HFCR_E_ZONE_LIMIT = -5, /* an impact zone exceeded HFCR_MAX_ZONE stencils;
                             positions hold the state before that round     */
  HFCR_E_REJECTED = -6    /* a request larger than the server's memory
                             budget, or a server that is shutting down     */
} hfcr_status;

typedef enum { HFCR_F32 = 0, HFCR_F64 = 1 } hfcr_dtype;

typedef enum {
  HFCR_ORIENT_B = 0,   /* only mesh B is oriented                           */
  HFCR_ORIENT_A = 1,   /* only mesh A is oriented                           */
  HFCR_ORIENT_BOTH = 2 /* both meshes are oriented                          */
} hfcr_orientation;

typedef enum {
  HFCR_BOTH_ALTERNATE = 0,   /* round r uses direction (r + round_offset) % 2;
                                if it has no hit, the other direction       */
  HFCR_BOTH_SIMULTANEOUS = 1 /* every round uses both directions            */
} hfcr_both_mode;

/* Largest impact zone (stencil count) the dense zone solver accepts. */
#define HFCR_MAX_ZONE 4096

/* opts.flags */
#define HFCR_FLAG_TIMING 1u /* record per-stage GPU times in stats.stage_ms */

typedef struct {
  int32_t dtype;       /* hfcr_dtype of pos                                  */
  int32_t nv;          /* vertex count, >= 0                                 */
  int32_t nt;          /* triangle count, >= 0                               */
  int32_t reserved;
  const void *pos;     /* device, [nv][3] row-major x, y, z in dtype.
                          Coordinates must be finite and be 0 or of
                          magnitude in [2^-200, 2^200] (every finite float32
                          qualifies).                                         */
  const int32_t *tri;  /* device, [nt][3] vertex indices in [0, nv)          */
} hfcr_mesh;

typedef struct {
  int32_t max_rounds;     /* responses at most (>= 0); default 256            */
  int32_t both_mode;      /* hfcr_both_mode; default ALTERNATE                */
  int32_t predicate_tier; /* 0: float32 filter, then float64 filter, then
                             exact (needs float32 storage; with float64
                             storage it acts as 1).  1: float64 filter, then
                             exact.  Both give the same decisions.            */
  int32_t round_offset;   /* alternation parity of the first round            */
  const double *inv_mass_a; /* device [nv_a] inverse masses w >= 0, or NULL
                               for all 1 (equal masses, Section 4)           */
  const double *inv_mass_b; /* device [nv_b] or NULL                         */
  uint32_t flags;           /* HFCR_FLAG_*                                   */
  int32_t reserved;
} hfcr_opts;

#define HFCR_STAT_ROUNDS 64
#define HFCR_STAGES 8 /* stage_ms: 0 setup+topology, 1 refit, 2 traverse,
                         3 narrow phase (filters and exact tier),
                         4 stencils and constraints (and the round-0 hit
                         sort), 5 zones (a round with at most 1024 active
                         hits builds its stencils, constraints and zones in
                         one launch, timed here), 6 solve, 7 update       */

typedef struct {
  int32_t rounds;            /* responses performed                          */
  int32_t converged;         /* 1 when the last detection found no hit       */
  int64_t residual_hits;     /* hits left in the oriented direction(s)       */
  int64_t hits0;             /* round-0 E-F hits (all oriented directions)   */
  int64_t stencils0;         /* round-0 stencils                             */
  int64_t candidates;        /* narrow-phase E-F tests, all detections (a
                                pass redone after a buffer grew counts once) */
  int64_t exact_tests;       /* tests settled by the exact tier              */
  int64_t f32_ambiguous;     /* tests the float32 filter could not settle    */
  int32_t max_zone;          /* largest impact zone seen (stencils)          */
  int32_t rank_deficient;    /* zones solved in the least-squares sense      */
  int64_t node_visits;       /* BVH nodes fetched by the traversals          */
  int32_t pivoted_zones;     /* zones solved by the pivoted fallback (a zone
                                whose unpivoted pivots fell below 1e-6 of
                                its largest diagonal entry)                 */
  int32_t max_query_path;    /* most traversal steps of any wavefront       */
  double stage_ms[HFCR_STAGES];     /* with HFCR_FLAG_TIMING, else 0        */
  int32_t stage_calls[HFCR_STAGES]; /* timed intervals per stage            */
  int32_t round_hits[HFCR_STAT_ROUNDS];
  int32_t round_stencils[HFCR_STAT_ROUNDS];
  int32_t round_zones[HFCR_STAT_ROUNDS];
  int32_t round_max_zone[HFCR_STAT_ROUNDS];
} hfcr_stats;

typedef struct {
  void *pos_a_out;       /* device [nv_a][3] in A's dtype, or NULL            */
  void *pos_b_out;       /* device [nv_b][3] in B's dtype, or NULL            */
  int32_t *hits;         /* device [hit_cap][5] round-0 hits
                            (dir, u, v, f, x0), sorted; or NULL.  u < v are
                            the edge's vertices, f the face, x0 the endpoint
                            behind the face; indices are local to their mesh */
  int64_t hit_cap;
  int32_t *stencils;     /* device [stencil_cap][3] round-0 stencils
                            (dir, x0, f), sorted and unique; or NULL          */
  int64_t stencil_cap;
  hfcr_stats *stats;     /* host, or NULL                                    */
} hfcr_result;

typedef struct hfcr_ctx hfcr_ctx;

/* Launch schedule of a context (results never depend on it). */
typedef struct {
  int32_t trav_block;    /* traversal workgroup size: 64, 128 or 256 (64)   */
  int32_t trav_warm;     /* 1: warm the L2 with the face BVH first (0)      */
  int32_t batch_workers; /* pairs in flight at once in the batch calls,
                            each on its own stream, 1..64 (12)              */
  int32_t reserved;
} hfcr_tuning;

/* One mesh pair of a batch call.  Inputs as for hfcr_resolve; `status` and
 * the buffers of `res` receive this pair's results. */
typedef struct {
  hfcr_mesh a;
  hfcr_mesh b;
  int32_t orientation;       /* hfcr_orientation of this pair                 */
  int32_t status;            /* out: this pair's hfcr_status                  */
  double d;                  /* post-response distance (Eq. 8), finite, >= 0  */
  const double *inv_mass_a;  /* device [a.nv] inverse masses, or NULL for 1  */
  const double *inv_mass_b;  /* device [b.nv] or NULL                        */
  hfcr_result res;           /* this pair's outputs and stats, as for
                                hfcr_resolve                                */
} hfcr_pair;

/* Largest number of pairs in one batch call. */
#define HFCR_MAX_BATCH 65536

/* Fill *opts with the defaults above. */
void hfcr_default_opts(hfcr_opts *opts);

/* Create a context on HIP device `device`.  The context owns a growable
 * device workspace; it is released by hfcr_destroy. */
hfcr_status hfcr_create(hfcr_ctx **out, int device);
void hfcr_destroy(hfcr_ctx *ctx);

/* Message describing the last non-OK status returned on this context. */
const char *hfcr_last_error(const hfcr_ctx *ctx);

/* One DCD pass (Section 3, first step) at the given positions over every
 * oriented direction: writes the sorted hit list and the stencils built from
 * it (Section 4); moves nothing.  Returns HFCR_E_CAPACITY if a list was
 * truncated (stats hold the full counts). */
hfcr_status hfcr_detect(hfcr_ctx *ctx, const hfcr_mesh *a, const hfcr_mesh *b,
                        int32_t orientation, const hfcr_opts *opts,
                        hfcr_result *res, void *stream);

/* The repair loop (Section 3): detect, build stencils, solve every impact
 * zone (Eq. 7/8) and relocate (Eq. 5), until no hit remains in the oriented
 * direction(s) or opts->max_rounds responses were made.  d >= 0 is the
 * post-response distance (Eq. 8).  Writes the final positions (float32
 * storage is rounded to nearest after every round), the round-0 hits and
 * stencils, and stats.  Returns HFCR_OK, HFCR_NOT_CONVERGED, or an error. */
hfcr_status hfcr_resolve(hfcr_ctx *ctx, const hfcr_mesh *a, const hfcr_mesh *b,
                         int32_t orientation, double d, const hfcr_opts *opts,
                         hfcr_result *res, void *stream);

/* The repair loop of hfcr_resolve (Section 3) for npairs independent mesh
 * pairs in one call.  Pairs are resolved concurrently: up to
 * tuning.batch_workers pairs are in flight at once, each on an internal
 * stream of its own, so the launches and waits of different pairs overlap.
 * Every pair runs the single-pair path, so its positions, lists and stats are
 * bit-identical to hfcr_resolve on that pair alone with the same opts
 * (opts->inv_mass_a/b are ignored: masses come from the pairs).  A pair that
 * fails (invalid input, zone limit, short output list) gets that status and
 * does not stop the others.  batch_stats (host, or NULL) receives the sums
 * over the pairs of every counter, the maxima of rounds, max_zone,
 * max_query_path and round_max_zone, converged = 1 if all converged, and
 * stage_ms summed over pairs (stages of different pairs overlap in time).
 * The call waits for `stream` first (inputs written on it are complete) and
 * returns after every pair's results are written.  Returns a negative status
 * if the call as a whole failed (bad arguments, workers could not be
 * created); else HFCR_OK if every pair's status is HFCR_OK, otherwise the
 * status of the first pair whose status is not. */
hfcr_status hfcr_resolve_batch(hfcr_ctx *ctx, hfcr_pair *pairs, int32_t npairs,
                               const hfcr_opts *opts, hfcr_stats *batch_stats,
                               void *stream);

/* hfcr_detect for every pair of a batch, run as hfcr_resolve_batch runs its
 * pairs (d, the inverse masses and pos_*_out are unused). */
hfcr_status hfcr_detect_batch(hfcr_ctx *ctx, hfcr_pair *pairs, int32_t npairs,
                              const hfcr_opts *opts, hfcr_stats *batch_stats,
                              void *stream);

/* ------------------------------------------------------------ serving
 * A request server for a stream of independent resolves of uneven sizes.
 * Requests are admitted in arrival order while a slot is free and the sum
 * of the admitted requests' estimated device footprints stays within
 * pool_bytes; each slot is a worker with its own context (its device
 * workspace stays allocated between requests) and its own stream, so the
 * work of admitted requests overlaps on the GPU.  Every request runs the
 * single-pair path of hfcr_resolve, so its results are bit-identical to a
 * call of hfcr_resolve on the same pair alone.
 *
 * Footprint estimate of a request (bytes): 512 per vertex and 1024 per
 * triangle of the two meshes, plus 1 MiB; it bounds the workspace a
 * resolve of that pair allocates, with a zone-solver slot budget sized for
 * the common case.  The caller's own input and output buffers are not
 * counted. */
typedef struct hfcr_server hfcr_server;

typedef struct {
  int32_t slots;       /* requests on the device at once, 1..64 (default 8)   */
  int32_t reserved;
  int64_t pool_bytes;  /* budget for the admitted footprints; 0 = unlimited */
} hfcr_server_cfg;

/* Create a server on HIP device `device` (cfg NULL = defaults). */
hfcr_status hfcr_server_create(hfcr_server **out, int device, const hfcr_server_cfg *cfg);

/* Stop admitting, finish every admitted and queued request, release the
 * workers. */
void hfcr_server_destroy(hfcr_server *srv);

/* Queue one resolve (the fields of *pair as for hfcr_resolve_batch, opts as
 * for hfcr_resolve; opts->inv_mass_a/b are ignored).  Returns at once with
 * a ticket.  *pair and every buffer it names must stay valid until
 * hfcr_server_wait has returned a final status for the ticket; the result is
 * written to pair->status and pair->res.  Inputs must be complete on the
 * device (synchronised) before the call.  Returns HFCR_E_REJECTED for a
 * request whose footprint exceeds pool_bytes. */
hfcr_status hfcr_server_submit(hfcr_server *srv, hfcr_pair *pair, const hfcr_opts *opts,
                               uint64_t *ticket);

/* Wait up to timeout_us microseconds (< 0: without limit) for a ticket.
 * Returns the request's status once it has finished (then the ticket is
 * released), or HFCR_PENDING.  *latency_ms (may be NULL) receives the time
 * from submission to completion.  An unknown ticket gives HFCR_E_INVALID. */
hfcr_status hfcr_server_wait(hfcr_server *srv, uint64_t ticket, int64_t timeout_us,
                             double *latency_ms);

/* Counters of a server: requests queued, running, completed, and the
 * footprint currently admitted (bytes); any pointer may be NULL. */
void hfcr_server_counts(const hfcr_server *srv, int64_t *queued, int64_t *running,
                        int64_t *completed, int64_t *admitted_bytes);

/* Read or replace the context's launch schedule (hfcr_tuning).  Every
 * schedule gives identical results; only speed differs.  Returns
 * HFCR_E_INVALID for an unsupported value. */
hfcr_status hfcr_get_tuning(const hfcr_ctx *ctx, hfcr_tuning *tuning);
hfcr_status hfcr_set_tuning(hfcr_ctx *ctx, const hfcr_tuning *tuning);

/* Diagnostic: signs of orient(a,b,c,p) for n point quadruples pts (device,
 * [n][4][3] float64: a, b, c, p) into out (device, [n] int32).  tier 0: the
 * float32 filter on the points rounded to float32 (2 = unsure); tier 1: the
 * float64 filter (2 = unsure); tier 2: exact.  Used to test the predicate
 * tiers against exact rational arithmetic. */
hfcr_status hfcr_test_orient(hfcr_ctx *ctx, const double *pts, int64_t n,
                             int32_t tier, int32_t *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HFCR_H */
