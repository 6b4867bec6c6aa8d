/*
 * pdg.h -- C ABI of the MI355X (gfx950) deform-and-match step of
 * Preconditioned Deformation Grids (Kaltheuner et al., arXiv:2509.18097).
 *
 * Conventions for every call below
 * --------------------------------
 * - Pointers are DEVICE pointers unless marked [host].  The caller owns every
 *   buffer; the library never frees caller memory.
 * - Point sets are structure-of-arrays float32: a set of n points is three
 *   consecutive rows of n floats (x row, y row, z row).  Rows of a set must be
 *   4-byte aligned; 16-byte alignment of the set base is recommended.
 * - A grid stack ("transition grid", paper Sec. 3.1) packs its levels one
 *   after another; level l holds C channels of R_l^3 float32 values (C = 3,
 *   or 6 where a call says so), each channel a dense R x R x R block with x
 *   fastest:
 *       value(c, z, y, x) at  level_offset(l) + ((c*R + z)*R + y)*R + x.
 *   Values are cell-centred on the cube [-1,1]^3 (centre of cell i is
 *   -1 + (2i+1)/R) and sampling clamps to the hull of the cell centres.
 * - Every call validates its arguments on the host before enqueuing anything,
 *   enqueues its work on `stream` and returns without waiting (asynchronous),
 *   except pdg_problem_create, pdg_mesh_plan_create and pdg_mesh_precondition,
 *   which build host-side tables and wait (see there).
 *   Argument errors return PDG_EINVAL and enqueue nothing.  A HIP launch error
 *   returns PDG_EHIP.  A device fault shows up as PDG_EHIP on a later call or
 *   synchronisation.  pdg_last_error() returns a thread-local message for the
 *   most recent failing call.  No call allocates device memory: scratch space
 *   comes from the caller through the `*_workspace` size queries (a workspace
 *   base must be 256-byte aligned, PDG_EINVAL otherwise).  pdg_problem_create
 *   allocates only its host-side handle; its device tables live in the
 *   caller's workspace.
 * - Calls on one stream are ordered; calls sharing a workspace must not
 *   overlap on different streams.
 */
#ifndef PDG_H
#define PDG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PDG_OK = 0,
  PDG_EINVAL = 1,        /* invalid argument; nothing was enqueued            */
  PDG_ENOMEM = 2,        /* workspace too small / host allocation failed     */
  PDG_EHIP = 3,          /* HIP runtime error (launch failure, device fault) */
  PDG_EUNSUPPORTED = 4   /* valid request that this build does not implement */
} pdg_status;

#define PDG_MAX_LEVELS 16   /* the paper uses L = 10 (Sec. 3.1) */

/* [host] Thread-local message describing the last failing call ("" if none). */
const char *pdg_last_error(void);
/* [host] Library version, major*10000 + minor*100 + patch. */
int32_t pdg_version(void);

/* Multi-resolution grid stack (paper Sec. 3.1, Eq. 1).
 *   levels      : L, 1..PDG_MAX_LEVELS.
 *   res[l]      : cells per axis of level l (>= 1; R = 1 is a constant level).
 *   channels    : 3 -- a translation t per cell (the Cayley rotation of
 *                 Eq. 4-7 with z = 0, where R(0) = I); every call takes it.
 *                 6 -- the full cell vector T = [z0 z1 z2 tx ty tz] of Eq. 4
 *                 (channel order as written there); pdg_grid_size,
 *                 pdg_deform, pdg_deform_backward(+_workspace),
 *                 pdg_precondition(+_workspace) (the rotation and the
 *                 translation halves of every level preconditioned alike)
 *                 pdg_adam and the problem (its full step on these cells,
 *                 also on pruned grids: all six channels of a level on the
 *                 same kept cells) take it.
 *   level_scale : factor applied to the sum over levels; 1/L reproduces the
 *                 averaging of Eq. 1. */
typedef struct {
  int32_t levels;
  int32_t res[PDG_MAX_LEVELS];
  int32_t channels;
  float level_scale;
} pdg_grid_desc;

/* [host] Number of float32 values in one grid stack (C * sum_l R_l^3), or -1. */
int64_t pdg_grid_size(const pdg_grid_desc *d);

/* ---------------------------------------------------------------- deform --
 * Warp (paper Eq. 1 with the translation form of Eq. 7):
 *     out_i = x_i + level_scale * sum_l trilerp(G_l, x_i).
 * With six channels (Sec. 3.3, Eq. 4-7): [z^; t^] = level_scale * sum_l
 * trilerp(G_l, x_i) and out_i = R(z^) x_i + t^ with the Cayley rotation
 * R(z) = (I + Z)(I - Z)^{-1} (Eq. 5, Z of Eq. 6) acting about the origin.
 * grids: one packed stack; x, out: SoA [3][n]; n >= 0 (n = 0 is a no-op).
 * out may alias x. */
pdg_status pdg_deform(const pdg_grid_desc *d, const float *grids, const float *x,
                      int64_t n, float *out, hipStream_t stream);

/* [host] Workspace bytes needed by pdg_deform_backward for n samples. */
pdg_status pdg_deform_backward_workspace(const pdg_grid_desc *d, int64_t n, size_t *bytes);

/* Adjoint of pdg_deform for an upstream gradient gout (SoA [3][n]):
 *   ggrids (nullable) <- level_scale * A^T gout   (OVERWRITES the whole stack;
 *                        the sum at every node is taken in a fixed order, so
 *                        the result is bitwise reproducible -- no atomics);
 *   gx     (nullable) <- gout + J^T gout, with J the position Jacobian of the
 *                        displacement (zero along clamped axes).
 * With six channels the rotation channels receive level_scale * A^T u with
 * u = d<gout, out>/dz^, the translation channels level_scale * A^T gout, and
 * gx = R^T gout + J^T [u; gout] (J the Jacobian of the interpolated cell
 * vector); grids is then needed for ggrids too.
 * ws: device workspace of at least pdg_deform_backward_workspace() bytes
 * (needed only when ggrids != NULL). */
pdg_status pdg_deform_backward(const pdg_grid_desc *d, const float *grids, const float *x,
                               int64_t n, const float *gout, float *ggrids, float *gx,
                               void *ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------ mesh --
 * Mesh-vertex preconditioner (paper Sec. 3.2 applied to the vertices of X_0;
 * Sec. 3.6: lambda = 16):
 *   out = (I + lambda L)^{-2} g  per channel,  L = D - A of the edge graph.
 * V >= 0 vertices; edges: int32 [2][E] (each undirected edge listed once; an
 * edge listed twice counts twice; edges with an endpoint outside [0, V) are
 * ignored); g, out: SoA [3][V] float32 (out may alias g); lambda >= 0.
 * max_degree: [host] an upper bound on every vertex degree (checked: a larger
 * degree is PDG_EINVAL); it fixes the spectrum bound [1, kappa], kappa =
 * 1 + 2 lambda max_degree, of I + lambda L.  The operator is evaluated as one
 * Chebyshev series of t^-2 on [1, kappa] in float64 vectors; terms: series
 * terms, or 0 for the fewest whose dropped coefficients' magnitudes sum below
 * tol (a bound on the operator-norm error; 1e-8 gives about 146 terms at
 * lambda = 16 and degree 6).  lambda = 0 or no edge: out = g exactly.
 * ws: device workspace of at least pdg_mesh_precondition_workspace() bytes;
 * it holds the plan's tables and vectors, so it must outlive the plan.
 *
 * A plan is built once per edge list (on the host, from a copy of the edges:
 * pdg_mesh_plan_create synchronises `stream`) and applied any number of
 * times; pdg_mesh_plan_apply enqueues kernels only (no allocation, no host
 * synchronisation; capturable in a HIP graph).  Applications of one plan
 * share its ws: calls that overlap (different streams) race.
 * pdg_mesh_plan_info: series terms and the number of vertex parts (0: the
 * graph's neighbourhoods did not fit, one term per launch).
 * pdg_mesh_precondition = create, apply, destroy (synchronous). */
typedef struct pdg_mesh_plan pdg_mesh_plan;
pdg_status pdg_mesh_precondition_workspace(int64_t V, int64_t E, size_t *bytes);
pdg_status pdg_mesh_plan_create(int64_t V, const int32_t *edges, int64_t E, float lambda,
                                int32_t max_degree, int32_t terms, double tol, void *ws,
                                size_t ws_bytes, hipStream_t stream, pdg_mesh_plan **plan);
pdg_status pdg_mesh_plan_apply(const pdg_mesh_plan *plan, const float *g, float *out,
                               hipStream_t stream);
pdg_status pdg_mesh_plan_info(const pdg_mesh_plan *plan, int32_t *terms /*[host]*/,
                              int32_t *parts /*[host]*/);
pdg_status pdg_mesh_plan_destroy(pdg_mesh_plan *plan);
/* [host only, no GPU] The vertex parts a plan of this edge list would use
 * (edges: HOST int32 [2][E]): sizes[0] = parts (0: one term per launch),
 * sizes[1] = local vertices over all parts, sizes[2] = recurrence terms per
 * launch k, sizes[3] = local vertices a part may hold.  With the arrays
 * non-NULL (sized from a first call): part_off[parts + 1] first local vertex
 * of each part, part_core[parts] its own vertices (listed first),
 * local_vertex[] the global index and local_dist[] the edge distance from the
 * part of every local vertex (every vertex within k edges, by distance). */
pdg_status pdg_mesh_partition(int64_t V, const int32_t *edges, int64_t E, int32_t *part_off,
                              int32_t *part_core, int32_t *local_vertex, int32_t *local_dist,
                              int64_t *sizes);
pdg_status pdg_mesh_precondition(int64_t V, const int32_t *edges, int64_t E, float lambda,
                                 int32_t max_degree, int32_t terms, double tol, const float *g,
                                 float *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* -------------------------------------------------------------- keyframe --
 * Keyframe selection (paper Sec. 3.5, Eq. 19-20):
 *   t_key = argmax_t exp(-gamma (t - T/2)^2) |G(P_t)|,  T = frames - 1,
 * with |G(P_t)| the number of occupied voxels of a 128^3 grid over [-1,1]^3
 * (voxel of a coordinate: floor((s + 1) * 64) in float32, clamped to 0..127;
 * NaN coordinates count in voxel 0).  The first frame wins ties.
 * points: [frames][3][n] SoA; 1 <= frames <= 65535; n >= 0.
 * counts (nullable): int64[frames] <- |G(P_t)| (exact);  key: int32[1] <- t_key.
 * gamma >= 0 and finite (the paper: 0.001).
 * ws: device workspace of at least pdg_keyframe_workspace() bytes. */
pdg_status pdg_keyframe_workspace(int32_t frames, size_t *bytes);
pdg_status pdg_keyframe(const float *points, int32_t frames, int64_t n, double gamma,
                        int64_t *counts, int32_t *key, void *ws, size_t ws_bytes,
                        hipStream_t stream);

/* --------------------------------------------------------------- chamfer --
 * Robust bidirectional Chamfer distance (paper Sec. 3.4, Eq. 11-13) between a
 * moving set A (n points) and a fixed set B (m points):
 *   nn_a[i] = argmin_j d2(a_i, b_j),  nn_b[j] = argmin_i d2(a_i, b_j),
 *   loss[0] = 1/n sum_i exp(-alpha s_i) s_i,  s_i = |a_i - b_nn_a[i]|^2,
 *   loss[1] = 1/m sum_j exp(-alpha s_j) s_j,  s_j = |a_nn_b[j] - b_j|^2.
 * Neighbour contract: d2 is evaluated in float32 in difference form without
 * fused multiply-add, dx = a_x - b_x, d2 = (dx*dx + dy*dy) + dz*dz, and ties
 * go to the lowest index; every mode returns exactly these indices for finite
 * coordinates (NaN coordinates give unspecified indices in the screen and
 * culled modes).
 * Losses are float64 sums of float64 distances (alpha is taken in float64
 * there; the float32 gradient uses alpha rounded to float32).
 *   mode PDG_CHAMFER_FP32       : exact float32 tiles.
 *   mode PDG_CHAMFER_BF16_SCREEN: bf16 matrix-core screen of |x|^2+|y|^2-2x.y
 *                                 with float32 accumulation, followed by an
 *                                 exact float32 re-rank of every candidate the
 *                                 screen cannot rule out.
 *   mode PDG_CHAMFER_FP32_CULL  : exact float32 evaluation of every candidate
 *                                 in the 256-point Morton tiles that the box
 *                                 cull of the bf16 screen keeps (no matrix
 *                                 cores); it isolates what the cull buys.
 * dir_weight (device double[2], nullable = {1,1}) scales the two directions
 * for the gradient.  ga (nullable): OVERWRITTEN with
 *   d/da [dir_weight[0]*loss[0] + dir_weight[1]*loss[1]]
 * with the assignment held fixed and the Gaussian weight differentiated;
 * B receives no gradient.  loss: device double[2].  nn_a: int32[n],
 * nn_b: int32[m].  n, m >= 1 and < 2^31. */
typedef enum {
  PDG_CHAMFER_FP32 = 0,
  PDG_CHAMFER_BF16_SCREEN = 1,
  PDG_CHAMFER_FP32_CULL = 2
} pdg_chamfer_mode;

pdg_status pdg_chamfer_workspace(int64_t n, int64_t m, int32_t mode, size_t *bytes);
pdg_status pdg_chamfer(const float *a, int64_t n, const float *b, int64_t m, double alpha,
                       int32_t mode, const double *dir_weight, double *loss,
                       int32_t *nn_a, int32_t *nn_b, float *ga,
                       void *ws, size_t ws_bytes, hipStream_t stream);

/* pdg_chamfer for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same kernels and
 * results, with the workspace taken from a fixed 64 MiB device array that the
 * library holds per GPU from its first use until the process ends.  Calls no
 * hipMalloc, hipFree or allocating routine.  n and m must satisfy
 * pdg_chamfer_workspace(n, m, mode) <= 64 MiB (about 4M + 4M points in the
 * float32 mode, 0.55M + 0.55M with the bf16 screen), else PDG_ENOMEM and
 * nothing is enqueued.  Every call on one GPU uses that GPU's one array, which
 * keeps the last call's contents: calls that overlap on one GPU (different
 * streams, or host threads) race and must be serialised by the caller.  The
 * first call on a device looks the array's address up (hipGetSymbolAddress)
 * with that device current. */
pdg_status pdg_chamfer_noalloc(const float *a, int64_t n, const float *b, int64_t m,
                               double alpha, int32_t mode, const double *dir_weight, double *loss,
                               int32_t *nn_a, int32_t *nn_b, float *ga, hipStream_t stream);

/* Adjoint of pdg_chamfer from saved indices (no new search):
 *   ga <- d/da [dir_weight[0]*loss[0] + dir_weight[1]*loss[1]]  (OVERWRITTEN)
 * with nn_a, nn_b as returned by pdg_chamfer for the same a, b.  dir_weight is
 * a device double[2] (e.g. the upstream gradient of the two losses).  The
 * reverse-direction sum at every point of a is taken in a fixed order
 * (sorted runs, no atomics).  ws: pdg_chamfer_workspace(n, m, PDG_CHAMFER_FP32). */
pdg_status pdg_chamfer_backward(const float *a, int64_t n, const float *b, int64_t m,
                                double alpha, const int32_t *nn_a, const int32_t *nn_b,
                                const double *dir_weight, float *ga, void *ws, size_t ws_bytes,
                                hipStream_t stream);

/* ---------------------------------------------------------- precondition --
 * Grid Sobolev preconditioner (paper Sec. 3.2, Eq. 3), in place:
 *   g_l <- (I + lambda[l] L_l)^{-2} g_l for every level l and channel of
 *   `batch` consecutive packed stacks, L_l the 6-neighbour combinatorial
 *   Laplacian of the R_l^3 cell box (free boundary).
 * method PDG_PRECOND_CG : two matrix-free conjugate-gradient solves per
 *   system with float32 vectors and float64 inner products; iters > 0 fixes
 *   the iteration count, iters = 0 takes the a-priori count from
 *   kappa <= 1 + 12 lambda for the A-norm tolerance `tol`.
 * method PDG_PRECOND_DCT: exact separable DCT-II diagonalisation (dense box
 *   grids); iters and tol are ignored.
 * lambda: [host] float[levels], each >= 0. */
typedef enum { PDG_PRECOND_CG = 0, PDG_PRECOND_DCT = 1 } pdg_precond_method;

pdg_status pdg_precondition_workspace(const pdg_grid_desc *d, int32_t batch, int32_t method,
                                      size_t *bytes);
pdg_status pdg_precondition(const pdg_grid_desc *d, const float *lambda, float *g,
                            int32_t batch, int32_t method, int32_t iters, double tol,
                            void *ws, size_t ws_bytes, hipStream_t stream);

/* --------------------------------------------------------------- pruning --
 * Pruned grids (paper Sec. 3.6, implementation details): a cell of a level is
 * kept when an input point lies in it or within `halo` cells of such a cell
 * along every axis (the paper: halo 3); pruned cells hold zero and are not
 * optimised.  The cell of a point along an axis is floor((s + 1) R / 2)
 * clamped to 0..R-1, decided in float32 (a NaN coordinate: cell 0).
 *
 * Mask layout (one stack): every level in order, ceil(R^3 / 32) uint32 words
 * each; cell c = (z R + y) R + x of a level is bit (c & 31) of its word
 * c >> 5.  pdg_prune_mask_words gives the words per stack; stacks follow each
 * other at that stride.  The masks cover cells, so the three functions below
 * take a three- or six-channel descriptor alike (same words, same bits). */
pdg_status pdg_prune_mask_words(const pdg_grid_desc *d, int64_t *words /*[host]*/);
pdg_status pdg_prune_workspace(const pdg_grid_desc *d, int32_t stacks, size_t *bytes);
/* Masks of `stacks` grid stacks: stack b is pruned by frames b .. b+span-1 of
 * points [stacks + span - 1][3][n] (span 2: the grid of a transition by the
 * two frames it connects).  mask: [stacks][words] (written whole); active
 * (nullable): int64 [stacks][levels] kept cells per level; halo 0..16;
 * 0 <= n < 2^31; stacks + span - 1 <= 65535.  ws: pdg_prune_workspace bytes. */
pdg_status pdg_prune_mask(const pdg_grid_desc *d, int32_t stacks, int32_t span,
                          const float *points, int64_t n, int32_t halo, uint32_t *mask,
                          int64_t *active, void *ws, size_t ws_bytes, hipStream_t stream);
/* Preconditioner of pruned grids (Eq. 3 on the kept cells), in place:
 *   g_l <- (I + lambda[l] L_S)^{-2} g_l on the kept cells S of every level,
 *   channel and stack, 0 on the pruned ones,
 * L_S the combinatorial Laplacian of the 6-neighbour graph the kept cells
 * induce (a pruned neighbour counts as absent).  Conjugate gradients as
 * PDG_PRECOND_CG (iters, tol, the a-priori count: every eigenvalue of L_S is
 * below 12 as well); mask as pdg_prune_mask writes it, for `batch` stacks;
 * ws: pdg_precondition_workspace(d, batch, PDG_PRECOND_CG) bytes. */
pdg_status pdg_precondition_pruned(const pdg_grid_desc *d, const float *lambda, float *g,
                                   int32_t batch, int32_t iters, double tol,
                                   const uint32_t *mask, void *ws, size_t ws_bytes,
                                   hipStream_t stream);

/* ------------------------------------------------------------------ adam --
 * Adam with bias correction (paper Sec. 3.6) over `batch` packed stacks with
 * a per-level learning rate: for every value of level l,
 *   m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
 *   theta <- theta - lr[l] * (m / (1-b1^k)) / (sqrt(v / (1-b2^k)) + eps),
 * k = step (1-based).  lr: [host] float[levels]. */
pdg_status pdg_adam(const pdg_grid_desc *d, int32_t batch, const float *lr, float beta1,
                    float beta2, float eps, int32_t step, float *theta, float *m, float *v,
                    const float *g, hipStream_t stream);

/* ------------------------------------------------------------- problem ---
 * One reconstruction request (paper Sec. 3, problem statement): a point-cloud
 * sequence P_0..P_{F-1} (frame 0 is the keyframe), an initial mesh X_0 with
 * edge list E, and one grid stack per transition t = 1..T = F-1 mapping frame
 * t-1 to frame t.  One pdg_step performs one optimisation iteration:
 *   1. P^_t = warp(G_t, P_{t-1}) for all t; X_t = warp(G_t, X_{t-1}), t = 1..T
 *      (Eq. 1, Eq. 8);
 *   2. CD_R(P^_t, P_t) and CD_R(X_t, P_t) (Eq. 11-13), cd_max (Eq. 17),
 *      w_conf (Eq. 15-16, not differentiated), L_iso (Eq. 18) and
 *      L = 1/T sum_t [w_conf(t) CD_R(X_t,P_t) + CD_R(P^_t,P_t)] + w_iso L_iso;
 *   3. the gradient of L with respect to every grid value (reverse sweep of
 *      the template chain; deterministic scatter into the grids);
 *   4. (I + lambda_l L_l)^{-2} per level (Eq. 3), lambda_l = lambda0*growth^l;
 *   5. Adam with lr_l = eta0 * eta_growth^l (Sec. 3.6).
 * With verts = 0 the template terms are dropped (L = 1/T sum_t CD_R(P^_t,P_t)).
 *
 * All pointers in the descriptor are device pointers owned by the caller and
 * must stay valid until pdg_problem_destroy.  params, adam_m, adam_v are
 * [T][grid_size] float32 and are updated in place by pdg_step. */
typedef struct {
  double alpha;         /* Eq. 13, 5.56 (float64: it enters the float64 loss) */
  float w_iso;          /* Eq. 9, 250                                         */
  float eta0;           /* Sec. 3.6, 5e-3                                     */
  float eta_growth;     /* 1.1 (+10% per finer level)                         */
  float lambda0;        /* 0.25                                               */
  float lambda_growth;  /* 1.5 (+50% per finer level)                         */
  float beta1, beta2, eps;   /* 0.9, 0.999, 1e-8                              */
  int32_t e_max;        /* total epochs for delta = 1 - sqrt(e/e_max) (Eq. 16) */
  float mesh_lambda;    /* Sec. 3.6, 16: (I + mesh_lambda L)^-2 on X_0's gradient */
  float mesh_lr;        /* Sec. 3.6, 1e-4: Adam learning rate of X_0            */
} pdg_hyper;

typedef struct {
  int32_t frames;             /* F >= 2                                       */
  int64_t n;                  /* points per frame, >= 1                       */
  const float *points;        /* [F][3][n]                                    */
  int32_t verts;              /* V >= 0 (0: no template terms)                */
  const float *template_verts;/* [3][V] (X_0)                                 */
  int32_t n_edges;            /* E >= 0 (edges only with V > 0)               */
  const int32_t *edges;       /* [2][E], 0 <= i, j < V                        */
  pdg_grid_desc grid;
  pdg_hyper hp;
  int32_t chamfer_mode;       /* pdg_chamfer_mode                             */
  int32_t precond_method;     /* pdg_precond_method                           */
  int32_t cg_iters;           /* 0: a-priori count per level for cg_tol       */
  double cg_tol;              /* e.g. 1e-7                                    */
  const uint32_t *prune_mask; /* [T][pdg_prune_mask_words] kept-cell bits of
                                 every transition's grids (pruned grids, see
                                 pdg_prune_mask; needs PDG_PRECOND_CG), or
                                 NULL for dense grids.  pdg_problem_create
                                 zeroes params, adam_m and adam_v on pruned
                                 cells; the preconditioner then acts on the
                                 graph of the kept cells and leaves the
                                 pruned ones at zero.                         */
  float *params;              /* [T][grid_size] theta                         */
  float *adam_m;              /* [T][grid_size]                               */
  float *adam_v;              /* [T][grid_size]                               */
  float *template_adam_m;     /* [3][V] Adam moments of X_0, or NULL; with    */
  float *template_adam_v;     /* both set X_0 is optimised too (Eq. 9-10):    */
                              /* template_verts is then updated in place      */
  int32_t keyframe;           /* k in [0, F): X_0 is the mesh of frame k.  With
                                 k > 0 the grids propagate X_0 both ways (the
                                 mechanism of Eq. 8 in reverse, Sec. 3.3): a
                                 backward chain k -> k-1 -> .. -> 0 and a
                                 forward chain k -> .. -> F-1; the T = F-1
                                 stacks of params / adam_m / adam_v /
                                 prune_mask are in chain order: the backward
                                 chain's (frame k-b+1 -> k-b, b = 1..k), then
                                 the forward chain's (frame k+f-1 -> k+f).
                                 Eq. 14 and 18 normalise by the total T, cd_max
                                 (Eq. 17) spans both chains, the confidence
                                 products (Eq. 15) run outward from k along
                                 each; X_0 is optimised (if asked) with the
                                 forward chain, the backward one if k = F-1.  */
  void *workspace;            /* >= pdg_problem_workspace() bytes             */
  size_t workspace_bytes;
} pdg_problem_desc;

typedef struct pdg_problem pdg_problem;

/* [host] Workspace bytes for a problem (all intermediate buffers of a step). */
pdg_status pdg_problem_workspace(const pdg_problem_desc *pd, size_t *bytes);
/* Validates pd, lays out the workspace, writes the problem's job tables into
 * it and enqueues the one-time set-up (Morton orders, static scatter tables of
 * the input points, template edge incidence, pruned-grid zeroing) on
 * `stream`.  *out receives an opaque handle (host memory).
 * SYNCHRONOUS: the tables are written with blocking host-to-device copies;
 * with a template the edge list is copied to the host to validate it and to
 * take the maximum vertex degree (X_0 optimised: also to build the mesh
 * preconditioner's plan, pdg_mesh_plan_create); with prune_mask the call synchronises
 * `stream` and copies the mask to the host to list the kept conjugate-
 * gradient tiles.  Create problems outside graph capture. */
pdg_status pdg_problem_create(const pdg_problem_desc *pd, hipStream_t stream, pdg_problem **out);
/* One iteration at 0-based epoch `epoch` (0 <= epoch <= e_max).  loss_terms
 * (device double[9], nullable) receives {L, L_transform, L_iso, cd_max,
 * sum_t CD_R(P^_t,P_t)/T, sum_t w_conf CD_R(X_t,P_t)/T, w_conf(T), epoch,
 * L_mesh} (L_mesh and its share of L are 0 unless X_0 is optimised).
 * Optimising X_0 (template_adam_m/v set) adds, after the grids' Adam, the
 * TEMPLATE stage: L_mesh = CD_R(X_0, P_0) (Eq. 10) in the problem's Chamfer
 * mode, its gradient with respect to X_0, (I + mesh_lambda L)^-2 with the
 * mesh Laplacian of the edge list (the series of pdg_mesh_precondition, tol
 * 1e-8, its plan built at creation) and Adam with mesh_lr.  X_0 enters
 * the template chain of the next step; the chain's own terms are not
 * differentiated with respect to X_0 (the mesh follows the keyframe's
 * points only).
 * With use_graph != 0 the step is replayed from a HIP graph captured on the
 * first call for this stream.  With the DCT preconditioner the last inverse
 * pass of each level of R = 16, 32, 64 or 128 (with the parameter, moment and
 * gradient buffers 16-byte aligned) applies Adam to the values it computes
 * (same arithmetic as the Adam stage, so the same parameters bit for bit)
 * and does not store them: after pdg_step those levels of PDG_BUF_PGRAD are
 * not the preconditioned gradient (pdg_step_stage(PDG_STAGE_PRECOND) fills
 * them from PDG_BUF_GRAD without touching the parameters). */
pdg_status pdg_step(pdg_problem *p, int32_t epoch, double *loss_terms, int32_t use_graph,
                    hipStream_t stream);
/* One stage of pdg_step alone, in step order WARP, NN, LOSS, GRAD, SCATTER,
 * PRECOND, ADAM (for profiling and stage-by-stage checks).  Each stage reads
 * what the previous stages of the same or an earlier step left in the
 * workspace; PRECOND rewrites the preconditioned gradient from the raw one and
 * ADAM updates params/m/v, so replaying them alone changes the state exactly
 * as the step would.  PRECOND_ADAM runs PRECOND and ADAM as pdg_step does
 * (Adam inside the preconditioner's last pass where it can). */
typedef enum {
  PDG_STAGE_WARP = 0,     /* Eq. 1 and 8: P^_t and the template chain (and, in
                             the bf16 mode, the screen packs of the warped sets) */
  PDG_STAGE_NN = 1,       /* Eq. 12: nearest neighbours of every Chamfer term
                             (one kernel launch)                                */
  PDG_STAGE_LOSS = 2,     /* Eq. 9, 11, 13-18: losses and confidence weights    */
  PDG_STAGE_GRAD = 3,     /* adjoints wrt the warped positions, reverse sweep   */
  PDG_STAGE_SCATTER = 4,  /* transpose of Eq. 1 into the grid gradient          */
  PDG_STAGE_PRECOND = 5,  /* Eq. 3                                              */
  PDG_STAGE_ADAM = 6,     /* Sec. 3.6                                           */
  PDG_STAGE_PRECOND_ADAM = 7,  /* PRECOND then ADAM as in pdg_step             */
  PDG_STAGE_TEMPLATE = 8  /* Eq. 10 and Sec. 3.6: X_0's loss, gradient, mesh
                             preconditioner and Adam (only when X_0 is
                             optimised; PDG_EINVAL otherwise)                  */
} pdg_stage;
pdg_status pdg_step_stage(pdg_problem *p, int32_t stage, hipStream_t stream);

pdg_status pdg_problem_destroy(pdg_problem *p);

/* ------------------------------------------------------------- batches --
 * Continuous batching of served requests (several independent problems
 * iterated together; not in the paper).  A batch is a fixed set of problems
 * whose iterations run as one unit: the screen pack, the nearest-neighbour
 * search (Eq. 12) and the Chamfer terms (Eq. 11, 13) of every member are one
 * launch each over a device table of all members' jobs (a job per transition,
 * term and direction of a member), and every other stage of a member runs as
 * in pdg_step, the members' kernels overlapping on parallel branches.  A job
 * writes only its own problem's buffers, so each member's results are bitwise
 * those of pdg_step on it alone.  A server makes a new batch whenever the set
 * of resident requests changes (creation copies the members' tables and
 * captures nothing until the first pdg_batch_step with use_graph).
 * Members must share the Chamfer mode and alpha, and none may propagate from a
 * keyframe inside its sequence (PDG_EUNSUPPORTED); a problem may belong to
 * several batches but the batches' steps must not overlap.
 * ws: >= pdg_batch_workspace() bytes of device memory, 256-byte aligned, owned
 * by the caller for the batch's lifetime.  Creation enqueues copies on
 * `stream`; step the batch on that stream (or synchronise first).  The batch
 * handle and its branch streams are host resources freed by
 * pdg_batch_destroy (the members stay). */
typedef struct pdg_batch pdg_batch;
pdg_status pdg_batch_workspace(pdg_problem *const *ps /*[host]*/, int32_t count, size_t *bytes);
pdg_status pdg_batch_create(pdg_problem *const *ps /*[host]*/, int32_t count, void *ws,
                            size_t ws_bytes, hipStream_t stream, pdg_batch **out);
/* One iteration of every member: epochs [host] int32[count], in member order
 * (each in [0, e_max] of its member).  use_graph captures the batch's
 * iteration once into a HIP graph and replays it.  Loss terms are read per
 * member (PDG_BUF_TERMS). */
pdg_status pdg_batch_step(pdg_batch *b, const int32_t *epochs, int32_t use_graph,
                          hipStream_t stream);
pdg_status pdg_batch_destroy(pdg_batch *b);

/* Intermediate buffers of the last step, for checking stage by stage.
 *   PDG_BUF_PHAT   float [T][3][n]   warped input points
 *   PDG_BUF_XHAT   float [F][3][V]   template chain (frame 0 = X_0)
 *   PDG_BUF_NN     int32 [T][2n] (+ [T][V+n] with a template): per transition
 *                  nn of P^ in P, nn of P in P^ (then nn of X in P, nn of P in X)
 *   PDG_BUF_LOSSES double[T][4]      CD directions: P^->P, P->P^, X->P, P->X
 *   PDG_BUF_WCONF  double[T]
 *   PDG_BUF_GRAD   float [T][grid_size]  raw gradient dL/dG
 *   PDG_BUF_PGRAD  float [T][grid_size]  preconditioned gradient (after
 *                                        pdg_step with the DCT preconditioner
 *                                        only for levels other than 64^3 and
 *                                        128^3; see pdg_step)
 *   PDG_BUF_GPHAT  float [T][3][n]   dL/dP^_t
 *   PDG_BUF_GXHAT  float [T][3][V]   direct dL/dX_t (Chamfer + isometry), frames 1..T
 *   PDG_BUF_TERMS  double[9]         the loss terms of pdg_step
 *   PDG_BUF_LAM    float [T][3][V]   total dL/dX_t after the reverse sweep of Eq. 8
 *   PDG_BUF_SCREEN_TILES uint64[1]   matrix-core products the bf16 screen
 *                  issued (each one 32 x 32 x 16 bf16 MFMA: 1,024 candidate-query
 *                  pairs; a product recomputed for the exact re-rank counts
 *                  again), summed over every step since creation; in the
 *                  culled float32 mode, the 1,024-pair units of candidate-query
 *                  distances it evaluated (0 bytes for the float32 mode)
 * When X_0 is optimised (0 bytes otherwise), from the last TEMPLATE stage:
 *   PDG_BUF_NN0    int32 [V + n]     nn of X_0 in P_0, then nn of P_0 in X_0
 *   PDG_BUF_LOSS0  double[2]         CD directions X_0->P_0, P_0->X_0
 *   PDG_BUF_GX0    float [3][V]      dL_mesh/dX_0
 *   PDG_BUF_PGX0   float [3][V]      (I + mesh_lambda L)^-2 dL_mesh/dX_0 */
typedef enum {
  PDG_BUF_PHAT = 0, PDG_BUF_XHAT = 1, PDG_BUF_NN = 2, PDG_BUF_LOSSES = 3,
  PDG_BUF_WCONF = 4, PDG_BUF_GRAD = 5, PDG_BUF_PGRAD = 6, PDG_BUF_GPHAT = 7,
  PDG_BUF_GXHAT = 8, PDG_BUF_TERMS = 9, PDG_BUF_LAM = 10, PDG_BUF_SCREEN_TILES = 11,
  PDG_BUF_NN0 = 12, PDG_BUF_LOSS0 = 13, PDG_BUF_GX0 = 14, PDG_BUF_PGX0 = 15
} pdg_buffer;
pdg_status pdg_problem_buffer(const pdg_problem *p, int32_t which, void **ptr, size_t *bytes);
/* The chains of a problem: which = 0 the backward chain (NULL when the
 * keyframe is 0), which = 1 the forward chain (NULL when the keyframe is the
 * last frame; the problem itself when the keyframe is 0).  A chain handle
 * serves pdg_problem_buffer for its own intermediate buffers, with its frames
 * in chain order (the backward chain's frame b is frame k - b); the problem
 * handle of a keyframe k > 0 serves only PDG_BUF_TERMS (the sequence's terms).
 * Chain handles belong to the problem (no destroy, no step). */
pdg_status pdg_problem_branch(const pdg_problem *p, int32_t which, pdg_problem **chain);

#ifdef __cplusplus
}
#endif
#endif /* PDG_H */
