/*
 * vp.h -- C ABI of libvp, a gfx950 (MI355X) evaluator of the 2-D volume
 * potential
 *
 *     u(x) = (1/2pi) int_Omega log|x - y| f(y) dA_y
 *
 * over an unstructured mesh of straight triangles, after Shen & Serkh,
 * "Accelerating potential evaluation over unstructured meshes in two
 * dimensions" (problem statement: Sec. 1 and Sec. 3.6; method: Sec. 3-4).
 *
 * The density is given by its values at the interpolation nodes of every
 * triangle (vp_ref_nodes); per triangle it is represented by the degree-p
 * interpolant f_h (Sec. 2.2 interpolation matrix, Sec. 3.5).  The library
 * returns, at every target x_t,
 *
 *   u(x_t) = (1/2pi) sum_Delta sum_j w_j |J_Delta| f_h(y_j) log|x_t - y_j|
 *          + sum_{Delta in S(x_t) u N(x_t)} sum_k R_{t,Delta,k} c_k(Delta)
 *
 * i.e. the far rule applied to every triangle (Sec. 3.2, coupled as point
 * charges as in Sec. 3.6) plus the subtract-and-add correction (Sec. 3.6)
 * over the self and near triangles of the target, where the near field is
 * the union of three Bernstein ellipses per triangle (Sec. 4.1, eqs. rho0,
 * Erho0, threeE) and the correction row R = (A - B)/2pi holds the accurate
 * integral A (near: adaptive subdivision, Sec. 3.3 with the Sec. 4.1
 * stopping rule; self: radius-arc-length coordinates, Sec. 3.4, eq.
 * volpot_self_single) minus the far rule's own contribution B, both against
 * the Koornwinder basis (Sec. 2.1).
 *
 * Conventions shared by every call
 *  - Every function returns a vp_status.  On an error the library sets a
 *    thread-local message (vp_last_error) and leaves every output untouched,
 *    except that after VP_EDEVICE the contents of u_out are unspecified.
 *  - Reference simplex T = {(x,y): x,y >= 0, x + y <= 1}.  A triangle is
 *    stored as three vertex indices (A, B, C); if det[B-A, C-A] < 0 the
 *    library swaps its local vertices 1 and 2 (B <-> C).  Node xi of triangle
 *    (A, B, C) sits at A + xi_1 (B - A) + xi_2 (C - A), using the oriented
 *    order.  The collapsed quadrature rules collapse onto vertex B.
 *  - All coordinates, densities and potentials cross the ABI as double.
 *  - Host arrays stay owned by the caller; the library copies what it needs
 *    during the call and keeps no host pointer.  With VP_DEVICE_PTRS the
 *    density / output pointers are device pointers owned by the caller; they
 *    must stay valid until the call's work has finished on the context's
 *    stream (immediately, unless VP_ASYNC).
 *  - The library owns all mesh and plan device memory.  A mesh must outlive
 *    its plans (vp_mesh_destroy returns VP_EBUSY while plans exist).
 *  - One context per host thread, or external serialisation.  Plans are
 *    read-only after creation.
 *  - No PyTorch (or other framework) type crosses this ABI: device memory
 *    and streams arrive as raw pointers and hipStream_t (as void*).
 */
#ifndef VP_H
#define VP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VP_OK = 0,
  VP_EINVAL = 1,     /* invalid argument (sizes, orders, degenerate geometry, NaN) */
  VP_ENOMEM = 2,     /* device allocation failed or the context's HBM budget is exceeded */
  VP_EDEVICE = 3,    /* a HIP runtime call or kernel failed */
  VP_ENOTSUP = 4,    /* valid request the library does not support */
  VP_EBUSY = 5,      /* object still in use (mesh with live plans) */
  VP_EINTERNAL = 6   /* internal limit hit (reported with the message) */
} vp_status;

typedef enum {
  VP_FP64 = 0,   /* all per-solve arithmetic in double */
  VP_MIXED = 1   /* far-field sum in FP32 (differences rounded from FP64, hardware
                    log2, FP32 sums per 256-source tile joined in FP64); the
                    correction rows stay FP64.  Relative error ~1e-7. */
} vp_precision;

/* vp_execute flags */
#define VP_DEVICE_PTRS 1u  /* density and u_out are device pointers */
#define VP_FAR_ONLY    2u  /* skip the self/near corrections: u = far sum only */
#define VP_ASYNC       4u  /* return without synchronising the stream (device pointers only) */

typedef struct vp_ctx vp_ctx;
typedef struct vp_mesh vp_mesh;
typedef struct vp_plan vp_plan;

/* Optional plan parameters; a NULL pointer selects the defaults. */
typedef struct {
  double c_n;       /* C_N of eq. rho0 (default 1.0: the larger, sufficient ellipse E' of Sec. 4.1) */
  int q_near;       /* points per direction of the sub-triangle rule, N_n = 2 q_near - 1 (default 7) */
  int n_l;          /* Gauss-Legendre points per arc-length panel, N_l (default 16) */
  double tau;       /* barycentric tolerance of the self test (default 1e-13) */
  int depth_cap;    /* maximum subdivision depth of a near pair (default 50) */
  int dyadic_cap;   /* maximum dyadic levels per side of a self piece (default 60) */
  uint32_t flags;   /* VP_DEVICE_PTRS: tgt_xy of vp_plan_create is a device pointer (default 0) */
  int near_model;   /* VP_NEAR_ELLIPSES (default): the union of Bernstein ellipses of Sec. 4.1;
                       VP_NEAR_BALL: the naive near field the paper compares against (the opening
                       of Sec. 4; the superscript-0 setting of Table near_corr), for ablation: a
                       target is near a triangle, and a near sub-triangle is split, when it lies
                       within ball_factor * R of the centroid c, R = the largest vertex distance
                       from c */
  double ball_factor; /* kappa of VP_NEAR_BALL (default 2.0; 0 < kappa <= 64) */
  int fmm_terms;      /* 0 (default): the far sum is the direct sum over all sources.  8..63: the
                         far sum by a fast multipole method with this many expansion terms (the
                         FMM coupling of Sec. 3.6): uniform quadtree over sources and targets,
                         adjacent leaf boxes summed directly with the same kernel, the rest by
                         complex multipole/local expansions, error <= 1.2 (sum |Q|) 0.547^p
                         (p = 56: ~2e-15 sum |Q|); both precisions then run it in FP64 */
  int fmm_leaf;       /* FMM: average far sources per leaf box of the full grid (default 128,
                         8..4096); sets the number of levels */
} vp_plan_opts;

enum { VP_NEAR_ELLIPSES = 0, VP_NEAR_BALL = 1 };

/* Sizes and statistics of a plan. */
typedef struct {
  int64_t n_tri;           /* triangles of the quadrature mesh */
  int64_t n_src;           /* far-field sources = n_tri * q^2 */
  int64_t n_tgt;           /* targets */
  int64_t n_pairs;         /* self + near (target, triangle) pairs */
  int64_t n_self;          /* self pairs */
  int64_t near_subtri;     /* near-rule leaves summed over all near pairs (paper's s_n times pairs) */
  int64_t self_panels;     /* arc-length panels summed over all self pairs (paper's s_l) */
  int64_t capped_leaves;   /* near leaves integrated at the depth cap */
  int64_t depth_first_pairs; /* near pairs whose subdivision was too wide for the breadth-first
                                level buffers and ran depth-first (slivers) */
  int64_t bytes_resident;  /* device bytes held by the plan */
  int32_t p, q, n_p, n_f;  /* orders; n_p = (p+1)(p+2)/2 nodes, n_f = q^2 far nodes per triangle */
  double eps;
  double ms_classify;      /* device time of the near-list construction */
  double ms_rows;          /* device time of the correction-row precompute */
  int64_t far_split;       /* source chunks of the far sum (partial sums per target and RHS) */
  int64_t cluster_entries; /* (16-target cluster, triangle) blocks of the matrix-core correction
                              apply (used for blocks of densities; 0: not built, the apply then
                              stays on the vector ALUs); n_pairs / (16 cluster_entries) is the
                              share of those blocks' rows that are pairs, not padding */
  int32_t fmm_terms;       /* expansion terms of the FMM far sum (0: direct sum) */
  int32_t fmm_levels;      /* quadtree levels below the root (leaf level) */
  int64_t fmm_near_pairs;  /* target-source pairs the FMM sums directly (adjacent leaf boxes) */
  int64_t fmm_m2l_pairs;   /* (target box, source box) M2L translations over all levels */
  int64_t tab_pairs;       /* near pairs whose subdivision stops at the triangle or after one split
                              (their rows by fixed Koornwinder tables on the matrix cores) */
  int64_t tab_leaves;      /* their near-rule leaves (one or four per pair), part of near_subtri */
} vp_plan_stats;

/* Context on HIP device `device`.  `hip_stream_or_null` is a hipStream_t the
 * context issues all work on (NULL: the device's null stream).
 * `hbm_budget_bytes` caps the device memory its meshes, plans, plan
 * workspaces, server slots, captured evaluations and interpolation objects
 * may hold, together with the blocks its cache keeps (0: no cap).  The
 * cache keeps the blocks of destroyed plans and outgrown workspaces for
 * later plans, up to a quarter of the device's memory; vp_ctx_trim empties
 * it.  *out receives the context.  vp_ctx_destroy returns VP_EBUSY while
 * meshes or servers of the context are alive. */
vp_status vp_ctx_create(int device, void* hip_stream_or_null, uint64_t hbm_budget_bytes, vp_ctx** out);
vp_status vp_ctx_destroy(vp_ctx* ctx);

/* Message of the last error on the calling thread ("" if none).  Valid until
 * the next call into the library on this thread. */
const char* vp_last_error(void);

/* Reference interpolation nodes of order p, 1 <= p <= 10 (stand-in for the
 * Vioreanu-Rokhlin nodes of Sec. 2.2): the interior Blyth-Pozrikidis nodes
 * built from the Gauss-Lobatto-Legendre points of order p + 3.  Writes
 * n_p = (p+1)(p+2)/2 into *n_p_out and, if xy_out is not NULL, the nodes as
 * [n_p][2] doubles.  The density passed to vp_execute is sampled at these
 * nodes, in this order. */
vp_status vp_ref_nodes(int p, double* xy_out, int* n_p_out);

/* Reference quadrature rules the plans are built from (host-side data, no
 * device needed), for inspection:
 *   which = 0  n-point Gauss-Legendre on [0,1]            -> x, w
 *           1  n-point Gauss rule for -log(r) on [0,1]    -> x, w
 *           2  n x n collapsed Gauss rule on the simplex  -> x, y, w (n^2 nodes;
 *              Sec. 3.2 far rule / Sec. 3.3 near rule)
 *           3  radial rule for interpolation order n      -> x = r, y = alpha,
 *              w = beta: node j contributes (alpha_j log r0 + beta_j) phi(r_j)
 *              to int_0^1 r log(r0 r) phi(r) dr (Sec. 3.4)
 *           4  per-edge weights w-hat of the n x n collapsed rule (edges AB,
 *              BC, CA) used in eq. rho0 -> w[0..2]
 *           5  the radial rule of order n folded onto n + 1 nodes, as the
 *              plans use it for straight self pairs (same layout as 3; the
 *              same sums for phi of degree <= n): r = 0 (the ray's apex)
 *              and the n-point Gauss-Legendre nodes on [0,1]
 *           6  the row kernels' conversion from their product basis to the
 *              Koornwinder basis of order n <= 6 (Sec. 2.1) -> w only,
 *              [n_p][n + 1]: K_i(x,y) = sum_{j <= n_i - m_i} w[i][j]
 *              Qm_{m_i}(x,y) Pm_j(2x-1) for i = n_i(n_i+1)/2 + m_i, with Pm_j
 *              the monic Legendre polynomials (Pm_{j+1} = z Pm_j - j^2/(4j^2-1)
 *              Pm_{j-1}) and Qm_m = (1-x)^m Pm_m((2y-1+x)/(1-x))
 * *count receives the number of entries; any output may be NULL. */
vp_status vp_ref_rule(int which, int n, double* x, double* y, double* w, int* count);

/* Upload a triangle mesh: vert_xy [n_vert][2] doubles, tri [n_tri][3]
 * int32 vertex indices.  Rejects (VP_EINVAL) indices out of range,
 * non-finite coordinates and degenerate triangles (|det| <= 1e-14 times
 * the squared size of the triangle's bounding box). */
vp_status vp_mesh_create(vp_ctx* ctx, int64_t n_vert, const double* vert_xy, int64_t n_tri,
                         const int32_t* tri, vp_mesh** out);
vp_status vp_mesh_destroy(vp_mesh* mesh);

/* Curved boundary sides (Sec. 3.1, eq. blend).  Entry i gives triangle
 * tri[i] one curved side: the edge from its local vertex side[i] to local
 * vertex side[i]+1 mod 3 (vertex order as passed to vp_mesh_create), as
 * pts [n][deg+1][2]: the side at the Chebyshev-Lobatto parameters
 * u_j = (1 - cos(pi j / deg)) / 2, pts[i][0] and pts[i][deg] equal to the
 * edge's two vertices (to 1e-13 of the triangle's size).  The side
 * becomes the polynomial gamma through these points; with B = gamma(0),
 * A = gamma(1) (swapped, with the curve reversed, to keep (A, B, C)
 * counter-clockwise) and C the opposite vertex, the triangle is the image
 * of the reference simplex under
 *   rho(xi, eta) = A + xi (B - A) + eta (C - A) + ((u - eta) / u) beta(u),
 *   u = 1 - xi, beta(u) = gamma(u) - (B + u (A - B)),
 * and the density of vp_execute is sampled at rho(interpolation nodes)
 * (vp_mesh_map_points).  Far rule: nodes rho(xi_j), weights w_j |J(xi_j)|
 * (Thm. smooth_int_jac); self pairs: found by Newton's method for
 * rho^{-1}(x), integrated in radius-arc-length coordinates of the reference
 * simplex about rho^{-1}(x); near pairs: the curved side treated as its
 * chord for the ellipse tests (Sec. 4.1), with the largest |J| at the far
 * nodes.  1 <= deg <= 32; each triangle at most once; one call per mesh,
 * before any plan (VP_EBUSY otherwise).  The library copies the arrays. */
vp_status vp_mesh_set_curved_sides(vp_mesh* mesh, int64_t n, const int32_t* tri, const int32_t* side, int deg,
                                   const double* pts);

/* Physical positions of n_ref reference points (ref_xy [n_ref][2], xi < 1)
 * on every triangle: out_xy [n_tri][n_ref][2] (host), the affine map of a
 * straight triangle (vertex order after vp_mesh_create's orientation) or
 * the blending map of a curved one.  n_ref <= 4096. */
vp_status vp_mesh_map_points(const vp_mesh* mesh, int n_ref, const double* ref_xy, double* out_xy);

/* Build the plan for (mesh, p, q, eps, targets): rule tables, far sources,
 * the CSR list of self/near pairs per target (Def. of near field, Sec. 3.2;
 * ellipse union, Sec. 4.1) and the FP64 correction rows of every pair.
 *   p     interpolation order, 1..10
 *   q     far rule: q x q collapsed Gauss (exact through degree N = 2q-1), 2..32
 *   eps   far/near tolerance of eq. precise_far (> 0)
 *   tgt_xy [n_tgt][2] host doubles, n_tgt >= 0
 * The work runs on the device; the call returns when the plan is complete. */
vp_status vp_plan_create(vp_ctx* ctx, const vp_mesh* mesh, int p, int q, double eps, int64_t n_tgt,
                         const double* tgt_xy, const vp_plan_opts* opts_or_null, vp_plan** out);
vp_status vp_plan_info(const vp_plan* plan, vp_plan_stats* out);

/* Host copies of the plan's pair list (for inspection and tests):
 * row_ptr [n_tgt+1] int64 (CSR by target), tri [n_pairs] int32 (ascending
 * within a target), kind [n_pairs] uint8 (0 = self, 1 = near).  Any pointer
 * may be NULL. */
vp_status vp_plan_pairs(const vp_plan* plan, int64_t* row_ptr_out, int32_t* tri_out, uint8_t* kind_out);

/* Host copy of the correction rows [n_pairs][n_p] doubles, pair order as in
 * vp_plan_pairs: row = (A - B) / 2pi (Sec. 3.6 subtract-and-add). */
vp_status vp_plan_rows(const vp_plan* plan, double* rows_out);

/* Host copy of the rows of pairs [first_pair, first_pair + count) only,
 * [count][n_p] doubles, same order and values as vp_plan_rows (for
 * inspecting a few targets' rows of a plan whose full row array is too large
 * to copy).  VP_EINVAL when the range leaves [0, n_pairs). */
vp_status vp_plan_rows_range(const vp_plan* plan, int64_t first_pair, int64_t count, double* rows_out);

/* Evaluate the potential for n_rhs >= 1 densities at once.
 *   density [n_tri][n_p][n_rhs] doubles (values at the interpolation nodes,
 *           right-hand side fastest), u_out [n_tgt][n_rhs] doubles.
 *   prec    VP_FP64 or VP_MIXED.
 *   flags   VP_DEVICE_PTRS | VP_FAR_ONLY | VP_ASYNC.
 * Steps: per-triangle coefficients c = V^{-1} F (Sec. 2.2) and far charges,
 * the direct far sum over all sources, then the correction rows applied to
 * c. */
vp_status vp_execute(vp_plan* plan, int64_t n_rhs, const double* density, double* u_out,
                     vp_precision prec, uint32_t flags);

/* The same evaluation without allocating device memory, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments as in vp_execute; flags must
 * include VP_DEVICE_PTRS (density and u_out are caller-owned device
 * arrays) and may add VP_FAR_ONLY and VP_ASYNC.  The workspace
 * (coefficients, far charges, their FP32 copy in VP_MIXED, far partial
 * sums) comes from one fixed device array of VP_NOALLOC_SCRATCH_BYTES per
 * device, held from the first vp_ctx_create on that device until the
 * process ends and shared by every call on that device: calls that overlap
 * on one device (other streams, other threads, VP_ASYNC calls whose work
 * is still queued on another context's stream) race on it.  A call whose
 * workspace would exceed VP_NOALLOC_SCRATCH_BYTES returns VP_EINVAL; so
 * does an FMM plan with 2 or more densities before a vp_execute with 2 or
 * more densities has built the plan's FMM tables for blocks of densities.
 * The call makes no hipMalloc, hipFree or other allocating call. */
#define VP_NOALLOC_SCRATCH_BYTES (256ull << 20)
vp_status vp_execute_noalloc(vp_plan* plan, int64_t n_rhs, const double* density, double* u_out,
                             vp_precision prec, uint32_t flags);

/* Intermediates of vp_execute, for inspection: coefficients
 * [n_tri][n_p][n_rhs] (Sec. 2.2: c = V^{-1} F per triangle) and far charges
 * [n_src][n_rhs] = w_j |J| f_h(y_j) / (4 pi) (the 1/2 of log r = log(r^2)/2
 * folded in), sources ordered triangle-major, node index a*q + b of the
 * collapsed rule.  Either output may be NULL.  Same pointer flags as
 * vp_execute. */
vp_status vp_coefficients(vp_plan* plan, int64_t n_rhs, const double* density, double* coef_out,
                          double* charge_out, uint32_t flags);

/* Far-source positions [n_src][2] (host copy). */
vp_status vp_plan_sources(const vp_plan* plan, double* xy_out);

/* Destroys the plan.  Waits for all work queued on the device (as hipFree
 * does) and hands the plan's device blocks to its context, which keeps them
 * up to a quarter of the device's memory (and, with an HBM budget, within
 * the budget together with everything the context holds) for later plans
 * of similar sizes: a plan that is built and destroyed every step then
 * neither allocates nor frees device memory after the first.  Blocks beyond
 * that limit are freed.  The context frees its cached blocks when an
 * allocation finds the device out of memory or the budget full, on
 * vp_ctx_trim and on vp_ctx_destroy. */
vp_status vp_plan_destroy(vp_plan* plan);

/* Device bytes the context holds in cached blocks of destroyed plans
 * (*bytes_out), and vp_ctx_trim: free all of them now. */
vp_status vp_ctx_cached_bytes(const vp_ctx* ctx, uint64_t* bytes_out);
/* Device bytes the context holds: in use (meshes, plans, workspaces, server
 * slots, captured evaluations, interpolation objects, FMM operators) and in
 * its cache.  With an HBM budget their sum stays within it. */
vp_status vp_ctx_memory(const vp_ctx* ctx, uint64_t* in_use_out, uint64_t* cached_out);
vp_status vp_ctx_trim(vp_ctx* ctx);

/* Wait for all work issued on the context's stream. */
vp_status vp_sync(vp_ctx* ctx);

/* Device-time accounting (for benchmarks).  With profiling on, every plan
 * creation and every vp_execute on the context brackets its stages with HIP
 * events on the context's stream and adds their durations (ms) and launch
 * counts to the context's accumulators, indexed by vp_stage.  Reading
 * synchronises the stream; vp_ctx_profile(ctx, on) also resets the
 * accumulators. */
typedef enum {
  VP_STAGE_CLASSIFY = 0, /* near-field pair list (Sec. 4.1) */
  VP_STAGE_ROWS = 1,     /* correction rows (Sec. 3.3, 3.4, 3.6) */
  VP_STAGE_COEF = 2,     /* coefficients and far charges (Sec. 2.2, 3.6) */
  VP_STAGE_FAR = 3,      /* far-field direct sum: one launch per RHS block */
  VP_STAGE_FINISH = 4,   /* partial sums + corrections */
  VP_STAGE_ROWS_TAB = 5,  /* part of VP_STAGE_ROWS: near pairs whose subdivision stops at the triangle
                             or after one split, on the matrix cores */
  VP_STAGE_ROWS_NEAR = 6, /* part of VP_STAGE_ROWS: the other near pairs */
  VP_STAGE_ROWS_SELF = 7, /* part of VP_STAGE_ROWS: self pairs */
  VP_N_STAGES = 8
} vp_stage;
vp_status vp_ctx_profile(vp_ctx* ctx, int on);
vp_status vp_ctx_timings(vp_ctx* ctx, double* ms_out /* [VP_N_STAGES] */, int64_t* launches_out /* [VP_N_STAGES] */);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of evaluation requests (the paper evaluates
 * one right-hand side at a time; this is the device-side scheduling of many).
 *
 * A server owns n_slots HIP streams (default priority) and one workspace per
 * slot.  vp_submit queues a request (a plan, n_rhs densities, an output);
 * requests start as slots and HBM (the context's budget) free up.  When a
 * slot frees, the oldest pending request is started together with the other
 * pending requests for the same plan and precision, packed along the
 * right-hand-side axis up to max_batch_rhs columns, so they share every
 * far-field logarithm; requests on different slots overlap on the device.
 * Progress (completion checks and admission) happens inside vp_submit,
 * vp_poll and vp_wait.  density [n_tri][n_p][n_rhs] and u_out [n_tgt][n_rhs]
 * are DEVICE pointers owned by the caller and must stay valid until the
 * request is done; the density must be complete on the context's stream
 * when vp_submit is called (vp_submit records an event there that the slot
 * waits for; work on other streams must be ordered before it by the
 * caller).  A slot's workspace comes from the context's block cache: when a
 * batch does not fit the budget, the idle slots' workspaces go back to the
 * cache first; the batch then waits for a running one to retire, and fails
 * with VP_ENOMEM only when nothing is running and it still does not fit.
 * A request's result equals vp_execute of the same arguments up to rounding
 * (the far sum of a column does not depend on the other columns of its
 * batch).  Errors: VP_EINVAL (bad arguments), VP_ENOMEM (a request larger
 * than the whole budget), VP_EDEVICE.  A server keeps its context alive
 * (vp_ctx_destroy returns VP_EBUSY until vp_server_destroy).
 * ------------------------------------------------------------------------ */
typedef struct vp_server vp_server;
typedef int64_t vp_ticket;
vp_status vp_server_create(vp_ctx* ctx, int n_slots, int max_batch_rhs, vp_server** out);
vp_status vp_server_destroy(vp_server* srv); /* waits for all requests */
vp_status vp_submit(vp_server* srv, vp_plan* plan, int64_t n_rhs, const double* density, double* u_out,
                    vp_precision prec, vp_ticket* ticket_out);
vp_status vp_poll(vp_server* srv, vp_ticket ticket, int* done_out);
vp_status vp_wait(vp_server* srv, vp_ticket ticket);
/* Counters: requests completed, batches launched, RHS columns launched. */
vp_status vp_server_stats(const vp_server* srv, int64_t* requests_done, int64_t* batches, int64_t* columns);
/* Admission counters: times a batch waited for a running one to free memory
 * under the context's budget, and requests failed with VP_ENOMEM. */
vp_status vp_server_admission(const vp_server* srv, int64_t* budget_waits, int64_t* rejected);

/* A captured evaluation (HIP graph) for repeated solves with new density
 * values in the same device buffer: the launches of vp_execute (FP64 or
 * VP_MIXED; flags 0 or VP_FAR_ONLY) for `plan`, n_rhs densities at
 * density_dev [n_tri][n_p][n_rhs] and output u_dev [n_tgt][n_rhs] (device
 * pointers that must stay valid), with a workspace of the graph's own.
 * vp_graph_launch queues one replay on the context's stream (vp_sync to
 * wait); the result equals vp_execute's.  The plan cannot be destroyed
 * while a graph of it exists (VP_EBUSY).  For callers that run many small
 * solves, where launch overhead matters. */
typedef struct vp_graph vp_graph;
vp_status vp_graph_create(vp_plan* plan, int64_t n_rhs, const double* density_dev, double* u_dev, vp_precision prec,
                          uint32_t flags, vp_graph** out);
vp_status vp_graph_launch(vp_graph* g);
vp_status vp_graph_destroy(vp_graph* g);

/* Launch shape of the direct far sum (the sum over all far-rule nodes of
 * Sec. 3.6), kept per plan, right-hand-side count and precision.  Every
 * shape gives the same potential up to rounding; only speed differs.
 *   shape       kernel of the vector-ALU sums:
 *               VP_FAR_WIDE     1024-thread blocks, 2 targets per thread,
 *                               4096-entry logarithm table (large target sets)
 *               VP_FAR_NARROW1  256-thread blocks, 1 target per thread,
 *                               256-entry table (small target sets)
 *               VP_FAR_NARROW2  256-thread blocks, 2 targets per thread
 *               (sums of several right-hand sides and the FP32 sum always run
 *               256-thread blocks; WIDE then means 2 targets per thread)
 *   mfma_tiles  16-target tiles per wavefront of the matrix-core sums
 *               (blocks of 16 right-hand sides): 1, 2 or 4
 *   n_split     source chunks, 1 <= n_split <= max(1, n_src_pad / 64)
 *               (n_src_pad: far sources rounded up to a multiple of 256;
 *               chunks are whole multiples of 64 sources, so a large n_split
 *               can leave chunks empty); each target gets n_split partial
 *               sums that the correction step adds up.
 * Without a stored shape a plan uses one chosen from its sizes.
 * vp_plan_autotune times each candidate shape (far sum plus the step that
 * adds the partials) on the context's stream with HIP events, `reps`
 * launches each after one warm-up, stores the fastest for (n_rhs, prec) and
 * returns it with its mean time in ms.  It runs the far sum on the
 * workspace's zero charges and leaves no result; its cost is about
 * (candidates x (reps + 1)) far sums.  Not to be called while work of the
 * plan is queued on another stream, or while a server holds requests of it.
 * vp_plan_set_far_config stores a given shape (VP_EINVAL if out of range);
 * graphs and servers use the shape stored when they issue the work. */
typedef struct {
  int32_t shape;
  int32_t mfma_tiles;
  int64_t n_split;
} vp_far_config;
enum { VP_FAR_WIDE = 0, VP_FAR_NARROW1 = 1, VP_FAR_NARROW2 = 2 };
vp_status vp_plan_far_config(const vp_plan* plan, int64_t n_rhs, vp_precision prec, vp_far_config* out);
vp_status vp_plan_set_far_config(vp_plan* plan, int64_t n_rhs, vp_precision prec, const vp_far_config* cfg);
vp_status vp_plan_autotune(vp_plan* plan, int64_t n_rhs, vp_precision prec, int reps, vp_far_config* best_out,
                           double* best_ms_out);

/* The far-order policy (Sec. 4.2, the trade-off between the far rule's
 * order and the precomputed near corrections): builds the plan for every
 * far order q in [q_min, q_max] with the given options, runs evaluations of
 * n_rhs zero densities in precision prec, and returns in *q_best the order
 * with the least plan time + n_solves x evaluation time.  A larger q makes
 * the far sum dearer (q^2 sources per triangle) and the near field smaller
 * (fewer correction rows to build and apply); with the FMM far sum the
 * balance moves to high q, with the direct sum to low q once the plan serves
 * many evaluations.  plan_ms / exec_ms (optional, q_max - q_min + 1 entries
 * each) receive the measured times (ms; the plan time includes tables the
 * first evaluation builds; NaN for an order skipped because it does not fit
 * the device, the context's budget or 2^31 sources).  Costs one plan and
 * three evaluations per order.  Densities and outputs are taken from the
 * context's memory.  VP_ENOMEM if no order fits. */
vp_status vp_choose_q(vp_ctx* ctx, const vp_mesh* mesh, int p, double eps, int64_t n_tgt, const double* tgt_xy,
                      const vp_plan_opts* opts_or_null, int q_min, int q_max, int64_t n_rhs, vp_precision prec,
                      double n_solves, int* q_best, double* plan_ms, double* exec_ms);

/* Interpolation of the potential over a mesh (Sec. 3.5).  Given u at the
 * order-p interpolation nodes (vp_ref_nodes; vp_mesh_map_points for their
 * positions) of every triangle of `mesh` -- e.g. the staggered target mesh
 * whose nodes were the targets of vp_execute -- u at any point x of the
 * mesh is sum_k c_k K_k(rho^{-1}(x)), c = V^{-1} u of the triangle that
 * contains x (Sec. 2.2 interpolation matrix; rho^{-1} affine, or Newton's
 * method on a curved triangle).  The object references the mesh, which
 * must outlive it (vp_mesh_destroy returns VP_EBUSY meanwhile). */
typedef struct vp_interp vp_interp;
vp_status vp_interp_create(vp_ctx* ctx, const vp_mesh* mesh, int p, vp_interp** out);
vp_status vp_interp_destroy(vp_interp* it);
/* Point location: tri_out[i] = the lowest-index triangle whose closure
 * (barycentric tolerance 1e-13) contains pts_xy[i], -1 if none;
 * ref_out [n][2] = rho^{-1}(pts_xy[i]) in it.  Host arrays. */
vp_status vp_interp_locate(vp_interp* it, int64_t n, const double* pts_xy, int32_t* tri_out, double* ref_out);
/* u at n (triangle, reference point) pairs: u_nodes [n_tri][n_p][n_rhs],
 * tri [n], ref_xy [n][2] -> out [n][n_rhs] (NaN where tri[i] = -1).  The
 * boundary trace of a curved side (Remark rem:bndry_interp): its point
 * gamma(u) is at reference point (1 - u, 0) of its triangle, no Newton
 * step needed.  Host arrays, or device pointers with VP_DEVICE_PTRS (then
 * the work is queued on the context's stream: vp_sync before reading). */
vp_status vp_interp_eval(vp_interp* it, int64_t n_rhs, const double* u_nodes, int64_t n, const int32_t* tri,
                         const double* ref_xy, double* out, uint32_t flags);

#ifdef __cplusplus
}
#endif

#endif /* VP_H */
