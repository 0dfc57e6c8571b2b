/*
 * spoly.h -- C ABI of the MI355X (gfx950) specular-polynomial solver.
 *
 * Method: Fan et al., "Specular Polynomials", ACM TOG 43(4), 2024.  For every
 * candidate (separator x0, separator x_{k+1}, triangle or triangle tuple) the
 * library finds all admissible specular chains: the vertex constraints
 * (Sec. 4.2-4.3) and, for two vertices, the rational coordinate mapping
 * (Sec. 4.4, Eq. eq_rct) give a bivariate system a(u,v) = b(u,v) = 0 in the
 * barycentrics (u,v) of the first vertex (Sec. 4.5); the hidden-variable Bezout
 * resultant (Sec. 5.1, Eq. eq_bezout) reduces it to the zeros of det R(v);
 * those are found by Laplace expansion plus recursive root isolation (one
 * vertex) or by a piecewise sign scan with bisection (two vertices) (Sec. 5.2);
 * u follows from a(u)|_v and each candidate is polished in FP64 and kept only
 * if it lies inside its triangle(s) and satisfies h x n = 0 (Eq. eq_ch)
 * (Sec. 5.3).
 *
 * Conventions (all entry points):
 *  - Array pointers are DEVICE pointers unless marked [host].  The caller owns
 *    every buffer; the library allocates device memory only inside a
 *    spoly_ctx (per-triangle tables, stage buffers), and frees it in
 *    spoly_ctx_destroy.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t, or NULL for
 *    the null stream).  Results are valid after the stream is synchronised.
 *  - Argument errors (null pointers, negative sizes, eta <= 0, out-of-range
 *    enums) are detected on the host before any launch and return
 *    SPOLY_E_INVALID_ARG; nothing is enqueued then.
 *  - Capacity: *out_count receives the total number of solutions found, which
 *    may exceed out_capacity; only the first out_capacity records are written
 *    (in unspecified order).  A caller that sees *out_count > out_capacity
 *    re-runs with a larger buffer.  This can only be seen after the stream
 *    synchronises, so the call itself returns SPOLY_OK.
 *  - Degenerate instances (zero-length normals, NaN/Inf input, identically
 *    vanishing resultant) yield no solution and bump counters[2] if
 *    `counters` is given.
 *  - Index inputs (vertex ids in the mesh, query ids) must be in range; the
 *    kernels do not re-check them.
 *  - Calls on one ctx must not overlap on different streams.
 */
#ifndef SPOLY_H
#define SPOLY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPOLY_OK = 0,
    SPOLY_E_INVALID_ARG = 1,
    SPOLY_E_CAPACITY = 2,
    SPOLY_E_DEVICE = 3,
    SPOLY_E_UNSUPPORTED = 4
} spoly_status;

/* scattering event at a specular vertex (Sec. 4.5: R = reflection, T = refraction) */
typedef enum { SPOLY_R = 0, SPOLY_T = 1 } spoly_event;

/* arithmetic of the bulk stages; the final polish and validation are always FP64 */
typedef enum {
    SPOLY_FP64 = 0,          /* every stage in double precision                           */
    SPOLY_FP32_POLISH64 = 1  /* R: coefficients, elimination and root isolation in float; */
                             /* root polish, path phase and validation in double.  T and  */
                             /* TT run every stage in double under either value.          */
} spoly_precision;

/* Triangle mesh, structure of arrays.  px..pz: vertex positions, nx..nz: vertex
 * normals (need not be unit length; the interpolated normal N u of Eq. eq_ni
 * is used un-normalised), all double [n_vertices].  tri: int32 [3*n_tris],
 * the vertex ids of triangle t are tri[3t], tri[3t+1], tri[3t+2]; e1 = p1 - p0,
 * e2 = p2 - p0 (Table 1). */
typedef struct {
    const double *px, *py, *pz;
    const double *nx, *ny, *nz;
    const int32_t *tri;
    int32_t n_vertices, n_tris;
} spoly_mesh;

/* separator points (shading points, receivers, lights): double [n] each */
typedef struct {
    const double *x, *y, *z;
    int32_t n;
} spoly_points;

/* Solver parameters [host].  spoly_default_params() fills the values used
 * throughout (pieces = 100 and bisect_iters = 10 from Sec. 5.2, iso_eps = 1e-9
 * from Sec. 5.2, tau = 1e-6 on |h^ x n^|). */
typedef struct {
    int32_t pieces;        /* uniform pieces of [0,1] for the >= 2-vertex sign scan      */
    int32_t bisect_iters;  /* bisection steps per sign change                            */
    double iso_eps;        /* one-vertex isolation stops below this interval length      */
    double tau;            /* path-space tolerance on |h^ x n^| at every vertex          */
    double u_margin;       /* u is searched on [-m, 1-v+m] before the polish             */
    double dedup;          /* candidates closer than this in (u,v) are one solution      */
    int32_t polish_iters;  /* maximum FP64 Newton steps of the polish                    */
    uint32_t flags;        /* SPOLY_FLAG_* bits; other bits must be 0                    */
} spoly_params;

/* spoly_params.flags */
#define SPOLY_FLAG_FORCE_FP64   (1u << 1)  /* run every stage in double precision whatever */
                                           /* the precision argument says                  */
#define SPOLY_FLAG_STAGE_TIMES  (1u << 2)  /* one-vertex solve: record timing events       */
                                           /* around its kernels (spoly_stage_times)       */
#define SPOLY_FLAG_DETERMINISTIC_ORDER (1u << 3)  /* sort the records written by (query,   */
                                           /* v[0], u[0]) on the device after the solve,   */
                                           /* so one input gives one output order (the     */
                                           /* solves reserve output slots with atomics);   */
                                           /* the context grows an ~80 B-per-record        */
                                           /* workspace; not for the no-allocation entry   */
                                           /* point (E_UNSUPPORTED) nor the mixed solve    */

/* One admissible chain.  For one vertex tri[1] = -1 and u[1] = v[1] = 0. */
typedef struct {
    int32_t query;         /* index into the query arrays                                */
    int32_t tri[2];        /* triangle ids of x1 (and x2)                                */
    uint32_t flags;        /* reserved                                                   */
    double u[2], v[2];     /* barycentrics of x1 (and x2), Eq. eq_xi                     */
    float residual;        /* max over the chain of |h^ x n^| after polish               */
    float edge;            /* min over the chain of min(u, v, 1-u-v)                     */
} spoly_solution;

typedef struct spoly_ctx spoly_ctx;

/* Create a context on HIP device `device` (also made current).  *ctx receives
 * the handle.  SPOLY_E_DEVICE if the device cannot be used. */
spoly_status spoly_ctx_create(spoly_ctx **ctx, int device);
/* Free the context and all device memory it owns.  NULL is ignored. */
void spoly_ctx_destroy(spoly_ctx *ctx);

/* Fill *p [host] with the default parameters (one-vertex u margin 1e-4). */
void spoly_default_params(spoly_params *p);
/* The same defaults with the two-vertex u margin 0.05: the first vertex's u
 * range is widened because the sqrt approximation of Eq. eq_refr_rational
 * moves the approximate roots before the FP64 polish. */
void spoly_tt_default_params(spoly_params *p);

/* Durations in milliseconds of the kernels of the last spoly_solve_1bounce
 * call on ctx that had SPOLY_FLAG_STAGE_TIMES set: reflection front, back,
 * full list (3 values); refraction coefficients, isolation, back, full list
 * (4 values).  ms [host, cap]; returns the number written, 0 if no such call
 * was made, -1 on an argument or device error.  Waits for that call to finish.
 * For measurement; the events are the context's own (hipEventCreate). */
int32_t spoly_stage_times(spoly_ctx *ctx, float *ms, int32_t cap);

/* Human-readable name of a status code (static storage). */
const char *spoly_status_str(spoly_status s);

/*
 * Conservative normal-cone cull for one specular vertex.
 * For every (x0 in x0s, x2 in x2s, triangle) triple, keep it unless no
 * generalised half vector h = eta0 w0 + eta1 w2 (w0, w2 unit directions from a
 * point of the triangle to x0 and x2) can be parallel to an interpolated normal
 * N u: with direction cones from the triangle's bounding sphere to x0 and x2
 * and the cone of the three vertex normals, the triple is rejected iff the
 * angle between the normal-cone axis line and the centre half vector exceeds
 * the normal-cone half angle plus the half-vector spread plus `margin`
 * radians.  Evaluated in float with the outward margin, so every triple with
 * an admissible chain is kept (h x n = 0 of Eq. eq_ch holds only if h is
 * parallel to the normal).
 * Output: kept triples as three int32 arrays out_x0, out_x2, out_tri
 * [out_capacity]; *out_count (device, uint64) receives the total kept, which
 * may exceed the capacity (the excess is not written).  *out_count must be
 * zeroed by the caller before the call (the kernel accumulates into it).
 * Order of the output is unspecified.
 */
spoly_status spoly_cull_1bounce(spoly_ctx *ctx, const spoly_mesh *mesh,
                                const spoly_points *x0s, const spoly_points *x2s,
                                double eta0, double eta1, double margin,
                                int32_t *out_x0, int32_t *out_x2, int32_t *out_tri,
                                int64_t out_capacity, unsigned long long *out_count, void *stream);

/*
 * Full solve (coefficients, elimination, isolation, polish, validation) for
 * one specular vertex (Sec. 4.5 systems R and T).
 * Query q solves the chain x0s[q_x0[q]] -> triangle q_tri[q] -> x2s[q_x2[q]].
 * eta0: IOR of the medium of x0, eta1: IOR of the medium of x2 (Eq. eq_ch;
 * reflection uses eta0 = eta1).  R requires both endpoints on the same side of
 * the normal, T opposite sides.
 * out [out_capacity] receives solution records; *out_count (device uint64,
 * zeroed by the caller) the total number found.
 * counters (optional, device uint64 [4], accumulated): [0] real roots of r(v)
 * found in [0,1], [1] (u,v) candidates polished, [2] degenerate instances,
 * [3] valid solutions dropped because an instance had more than four (each
 * instance keeps at most four; nonzero means some instance lost solutions).
 * diag_q (optional, device int32 [2*n_queries]): per query the number of roots
 * of r(v) in [0,1] and the number of solutions.
 * Runs in two phases: the front finds the roots of r(v) and lists the
 * candidates that have any in a workspace owned by ctx (28 bytes per query,
 * for refraction 112 more; grown on demand, and growing synchronises the
 * device); the back solves, polishes and validates the listed candidates.  Calls that share a
 * context must therefore be issued on one stream.  E_DEVICE if the workspace
 * cannot be allocated.  With SPOLY_FP32_POLISH64, candidates with more than two
 * roots, or with a float root whose u misses the triangle by less than 0.005,
 * are solved again from scratch in double precision.
 */
spoly_status spoly_solve_1bounce(spoly_ctx *ctx, const spoly_mesh *mesh,
                                 const spoly_points *x0s, const spoly_points *x2s,
                                 const int32_t *q_x0, const int32_t *q_x2, const int32_t *q_tri,
                                 int64_t n_queries, spoly_event ev, double eta0, double eta1,
                                 spoly_precision prec, const spoly_params *params,
                                 spoly_solution *out, int64_t out_capacity,
                                 unsigned long long *out_count, unsigned long long *counters,
                                 int32_t *diag_q, void *stream);

/*
 * spoly_solve_1bounce without any device allocation, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * and harnesses that forbid hipMalloc.  Same arguments, semantics and results
 * as spoly_solve_1bounce, minus the context: the work runs on the device that
 * is current, and the two-phase workspace is a file-scope device array of
 * SPOLY_NOALLOC_SCRATCH_BYTES that every device the library runs on holds
 * until the process ends (its device address is looked up on the first call
 * on each device; no memory is allocated then either).  The workspace's
 * counters are cleared by a kernel at the start of every call.
 * Limits: n_queries <= SPOLY_NOALLOC_MAX_QUERIES_R (reflection) or
 * SPOLY_NOALLOC_MAX_QUERIES_T (refraction); larger calls return
 * SPOLY_E_CAPACITY and enqueue nothing.  Calls on one device share the one
 * array: calls that overlap on one device (other streams, other threads) race
 * and give undefined results; issue them on one stream.
 */
#define SPOLY_NOALLOC_SCRATCH_BYTES (64ll << 20)
#define SPOLY_NOALLOC_MAX_QUERIES_R 2000000
#define SPOLY_NOALLOC_MAX_QUERIES_T 450000
spoly_status spoly_solve_1bounce_noalloc(const spoly_mesh *mesh,
                                         const spoly_points *x0s, const spoly_points *x2s,
                                         const int32_t *q_x0, const int32_t *q_x2, const int32_t *q_tri,
                                         int64_t n_queries, spoly_event ev, double eta0, double eta1,
                                         spoly_precision prec, const spoly_params *params,
                                         spoly_solution *out, int64_t out_capacity,
                                         unsigned long long *out_count, unsigned long long *counters,
                                         int32_t *diag_q, void *stream);

/*
 * Normal-cone cull for two specular vertices (chain x0 -> T1 -> T2 -> x3).
 * For every x0 in x0s, x3 in x3s and ordered pair of distinct triangles, keep
 * the tuple unless one vertex fails the half-vector / normal-cone test of
 * spoly_cull_1bounce: at x1 the half vector combines the direction to x0
 * (eta[0]) with the direction cone from T1's bounding sphere to T2's (eta[1]);
 * at x2 the cone from T2 to T1 (eta[1]) with the direction to x3 (eta[2]).
 * The test at x2 does not depend on x0: it is evaluated once per (light, T1,
 * T2) into a pair list held in the context, then every x0 is tested against
 * the listed pairs.  eta [host, 3].  Output: int32 arrays out_x0, out_x3,
 * out_t1, out_t2 [out_capacity]; *out_count (device uint64, zeroed by the
 * caller) receives the total kept.  Synchronises `stream` once per light
 * (to size the second pass).
 */
spoly_status spoly_cull_2bounce(spoly_ctx *ctx, const spoly_mesh *mesh,
                                const spoly_points *x0s, const spoly_points *x3s,
                                const double *eta, double margin,
                                int32_t *out_x0, int32_t *out_x3, int32_t *out_t1, int32_t *out_t2,
                                int64_t out_capacity, unsigned long long *out_count, void *stream);

/*
 * Full solve for k = 2 specular vertices (Sec. 4.4-4.5, Sec. 5.2): chain [host, k]
 * = the event at T1 then at T2, each SPOLY_R or SPOLY_T (chains RR, RT, TR,
 * TT); eta [host, k+1] = IORs of the segments x0x1, x1x2, x2x3 (Eq. eq_ch); a
 * reflection needs equal IORs on its two segments (else E_INVALID_ARG).
 * Query q solves x0s[q_x0[q]] -> triangle q_tris[2q] -> triangle q_tris[2q+1]
 * -> x3s[q_x3[q]].
 * A reflected direction at x1 is exact (Eq. eq_431_di scaled by |n|^2); a
 * refracted one uses the piecewise (1,1)-rational square root of Sec. 4.4:
 * sqrt_table [host, optional] = 7 piece ends then (c0, c1, d0, d1) for each
 * of the 6 pieces; NULL selects the library's minimax table.  The sign of
 * det R(v) is sampled at v = j/pieces (1 <= pieces <= 4095) and each sign
 * change is refined by bisect_iters (<= 40) bisection steps; near-double root
 * pairs of a(., v), and roots where the mapped ray from x1 runs within 1e-4 rad
 * of T2's plane (x2 at infinity), are left out of the sign's product.  Every candidate is polished
 * in FP64 on the exact constraints (the approximation only brackets roots).
 * prec must be SPOLY_FP64.  Records carry tri[0..1] and (u,v) of both vertices.
 * counters / diag_q as for spoly_solve_1bounce ([0] counts sign changes).
 */
spoly_status spoly_solve_nbounce(spoly_ctx *ctx, const spoly_mesh *mesh, int32_t k,
                                 const spoly_event *chain, const double *eta,
                                 const spoly_points *x0s, const spoly_points *x3s,
                                 const int32_t *q_x0, const int32_t *q_x3, const int32_t *q_tris,
                                 int64_t n_queries, spoly_precision prec, const spoly_params *params,
                                 const double *sqrt_table,
                                 spoly_solution *out, int64_t out_capacity, unsigned long long *out_count,
                                 unsigned long long *counters, int32_t *diag_q, void *stream);

/*
 * Learned pruner of two-vertex tuples (callers who want to skip tuples
 * that cannot hold a path before spoly_solve_nbounce).  An MLP with 42 inputs
 * (x0/2, x3/2, the positions of T1 and T2 divided by 2, the vertex normals of
 * T1 and T2), three hidden layers of 128 ReLU units and a sigmoid output.
 * params: device float [SPOLY_PRUNER_NPARAMS]: W1 [42 x 128] (row = input),
 * b1 [128], W2 [128 x 128], b2 [128], W3 [128 x 128], b3 [128], W4 [128], b4 [1].
 * Dense layers run on the matrix cores with bf16 operands and fp32
 * accumulation; master parameters, gradients and optimizer state are fp32.
 * Tuples are given as for spoly_solve_nbounce (q_x0, q_x3, q_tris[2q..2q+1]).
 */
#define SPOLY_PRUNER_NPARAMS 38657

/* Scores in [0,1] (scores [n], optional) and the indices q of the tuples with
 * score >= threshold (keep_idx [keep_capacity], order unspecified);
 * *keep_count (device uint64, zeroed by the caller) receives the total kept. */
spoly_status spoly_prune_score(spoly_ctx *ctx, const spoly_mesh *mesh, const spoly_points *x0s,
                               const spoly_points *x3s, const int32_t *q_x0, const int32_t *q_x3,
                               const int32_t *q_tris, int64_t n, const float *params, float threshold,
                               float *scores, int32_t *keep_idx, int64_t keep_capacity,
                               unsigned long long *keep_count, void *stream);

/* Forward and backward pass of one batch under the class-weighted binary cross
 * entropy  mean_q [ -w y_q log p_q - (1 - y_q) log(1 - p_q) ],  w = pos_weight
 * for positives.  labels [n] in {0,1}; grads [SPOLY_PRUNER_NPARAMS] (written);
 * *loss (device float) accumulates the batch loss.  n <= 65536. */
spoly_status spoly_pruner_fwd_bwd(spoly_ctx *ctx, const spoly_mesh *mesh, const spoly_points *x0s,
                                  const spoly_points *x3s, const int32_t *q_x0, const int32_t *q_x3,
                                  const int32_t *q_tris, int64_t n, const float *labels, float pos_weight,
                                  const float *params, float *grads, float *loss, void *stream);

/* Adam step (step >= 1, bias-corrected) on params with grads and moment
 * buffers adam_m, adam_v [SPOLY_PRUNER_NPARAMS] (zero-initialised by the caller). */
spoly_status spoly_pruner_step(spoly_ctx *ctx, float *params, const float *grads, float *adam_m, float *adam_v,
                               int64_t step, float lr, float beta1, float beta2, float eps, void *stream);

/* Features of n tuples as fp32 [n x 48] (42 used, 6 zero), the network input. */
spoly_status spoly_pruner_features(spoly_ctx *ctx, const spoly_mesh *mesh, const spoly_points *x0s,
                                   const spoly_points *x3s, const int32_t *q_x0, const int32_t *q_x3,
                                   const int32_t *q_tris, int64_t n, float *features, void *stream);

/*
 * Mixed batches in one persistent launch.  Work items are tiles of
 * `r_tile` one-vertex instances (problem 1, as spoly_solve_1bounce) and single
 * two-vertex tuples (problem 2, as spoly_solve_nbounce with chain TT); waves
 * take items from the device counter *queue (zeroed by the caller) until it
 * passes the last item.  Output records of problem 1 carry query q, those of
 * problem 2 carry n1 + q.  prec applies to problem 1's R bulk (T and TT run in
 * FP64).  params->u_margin applies to problem 1; problem 2 searches u on
 * [-0.05, 1-v+0.05], the margin spoly_tt_default_params sets.  Shapes come
 * from spoly_mixed_shape (an autotuner may choose them).  Errors as
 * spoly_solve_1bounce; a shape outside the stated ranges is E_INVALID_ARG.
 */
typedef struct {
    int32_t workgroups_per_cu;  /* persistent grid = compute units x this (1..32)          */
    int32_t r_tile;             /* one-vertex instances per work item (64..4096, x64)       */
    int32_t order;              /* 0: two-vertex items first, 1: one-vertex first, 2: mixed */
    int32_t pad;
} spoly_mixed_shape;

spoly_status spoly_solve_mixed(spoly_ctx *ctx,
                               const spoly_mesh *mesh1, const spoly_points *x0s1, const spoly_points *x2s1,
                               const int32_t *q1_x0, const int32_t *q1_x2, const int32_t *q1_tri, int64_t n1,
                               spoly_event ev1, double eta0, double eta1,
                               const spoly_mesh *mesh2, const spoly_points *x0s2, const spoly_points *x3s2,
                               const int32_t *q2_x0, const int32_t *q2_x3, const int32_t *q2_tris, int64_t n2,
                               const double *eta2, spoly_precision prec, const spoly_params *params,
                               const spoly_mixed_shape *shape, unsigned long long *queue,
                               spoly_solution *out, int64_t out_capacity, unsigned long long *out_count,
                               void *stream);

/*
 * Path-phase tail (Sec. 5.3, "The whole pipeline"): after the path-space
 * check a chain is dropped when the segment from any of its vertices to the
 * next (x0 -> x1 -> ... -> x_k -> light) is blocked by the mesh; every chain
 * that stays contributes to its endpoint x0, and several chains between the
 * same endpoints add up.
 *
 * spoly_bvh_build: bounding volume hierarchy over the mesh's triangles (a
 * linear hierarchy over Morton-sorted centroids), built on ctx's device on
 * `stream` and waited for.  Allocates device memory owned by *out until
 * spoly_bvh_destroy (NULL is ignored).  The mesh arrays must not change
 * while the hierarchy is in use.  E_INVALID_ARG on a bad mesh, E_DEVICE on a
 * HIP error (nothing is left allocated).
 */
typedef struct spoly_bvh spoly_bvh;
spoly_status spoly_bvh_build(spoly_ctx *ctx, const spoly_mesh *mesh, spoly_bvh **out, void *stream);
void spoly_bvh_destroy(spoly_bvh *bvh);

/* Tail parameters [host]; spoly_tail_default_params fills I = 1, rho = 1,
 * t_eps = 1e-6 and a zero receiver normal. */
typedef struct {
    double intensity;      /* radiant intensity of the isotropic point light at x_{k+1}       */
    double reflectance;    /* rho, the factor of every reflection vertex                       */
    double t_eps;          /* hits within t_eps (segment parameter) of either end do not block */
    double rcv_normal[3];  /* image weight |w0 . n| (w0 the unit direction x0 -> x1); all      */
                           /* zero: weight 1 (irradiance on the plane normal to the ray)       */
} spoly_tail_params;
void spoly_tail_default_params(spoly_tail_params *p);

/*
 * Visibility and contribution of validated chains (records `sols` from
 * spoly_solve_1bounce (k = 1) or spoly_solve_nbounce (k = 2) over the same
 * query arrays q_x0 / q_xl and endpoint sets; device memory).  chain [host, k]
 * and eta [host, k+1] as for the solve (eta[i] the index between x_i and
 * x_{i+1}; a reflection needs equal indices on both sides).  Per record p:
 *  mask[p]    (device int32, optional): bit i set when x_i -> x_{i+1} is
 *             blocked: some triangle other than those carrying its two ends
 *             meets it at closed barycentrics and a segment parameter in
 *             [t_eps, 1 - t_eps] (double-precision Moller-Trumbore);
 *             bit 30 set when the constraint Jacobian is singular (a caustic
 *             point: contribution undefined, reported as 0); bit 29 set if a
 *             traversal hit its stack or visit bound (not reachable for a
 *             hierarchy from spoly_bvh_build);
 *  contrib[p] (device double, optional): E = I * prod F_i * dw/dA, the
 *             irradiance at x0 on the plane normal to the arriving ray, before
 *             visibility; F_i is the unpolarised Fresnel transmittance at a
 *             refraction (interpolated shading normal) and rho at a
 *             reflection; dw/dA the light's solid angle per unit of that area,
 *             by implicit differentiation of the vertex constraints of Eq. eq_ch;
 *  image[q_x0[query]] (device double [x0s->n], optional): += E * weight
 *             (rcv_normal) for each record with mask 0, by atomic adds (the
 *             caller zeroes it; the order of the adds is unspecified).
 * sol_count (device, optional): only min(*sol_count, n_sols) records are read,
 * so a solve's out_count can be passed without a host round trip.  Asynchronous
 * on `stream`.  E_INVALID_ARG on bad arguments or a hierarchy of another mesh
 * or device; E_UNSUPPORTED for k outside 1..2.
 */
spoly_status spoly_path_tail(spoly_ctx *ctx, const spoly_mesh *mesh, const spoly_bvh *bvh, int32_t k,
                             const spoly_event *chain, const double *eta,
                             const spoly_points *x0s, const spoly_points *xls,
                             const int32_t *q_x0, const int32_t *q_xl,
                             const spoly_solution *sols, int64_t n_sols, const unsigned long long *sol_count,
                             const spoly_tail_params *params, int32_t *mask, double *contrib, double *image,
                             void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SPOLY_H */
