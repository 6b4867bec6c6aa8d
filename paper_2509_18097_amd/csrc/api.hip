// C ABI of libpdg (declared in include/pdg.h): argument validation,
// workspace layout and the orchestration of one optimisation step.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.h"

namespace pdg {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

pdg_status hip_fail(hipError_t e, const char *what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return PDG_EHIP;
}

pdg_status check_grid(const pdg_grid_desc *d, bool six_ok) {
  if (!d) {
    set_error("grid descriptor is NULL");
    return PDG_EINVAL;
  }
  if (d->levels < 1 || d->levels > PDG_MAX_LEVELS) {
    set_error("levels = %d outside 1..%d", d->levels, PDG_MAX_LEVELS);
    return PDG_EINVAL;
  }
  if (d->channels == 6 && !six_ok) {
    set_error("six-channel (Cayley) grids are implemented by pdg_deform and "
              "pdg_deform_backward only");
    return PDG_EUNSUPPORTED;
  }
  if (d->channels != 3 && d->channels != 6) {
    set_error("channels = %d: must be 3 (translation) or 6 (Cayley rotation + translation)",
              d->channels);
    return PDG_EINVAL;
  }
  for (int l = 0; l < d->levels; ++l)
    if (d->res[l] < 1 || d->res[l] > 1024) {
      set_error("res[%d] = %d outside 1..1024", l, d->res[l]);
      return PDG_EINVAL;
    }
  if (!(isfinite(d->level_scale))) {
    set_error("level_scale is not finite");
    return PDG_EINVAL;
  }
  return PDG_OK;
}

GridDev make_grid(const pdg_grid_desc &d) {
  GridDev g;
  memset(&g, 0, sizeof g);
  g.levels = d.levels;
  g.ch = d.channels;
  long long off = 0, noff = 0;
  for (int l = 0; l < d.levels; ++l) {
    const long long r3 = (long long)d.res[l] * d.res[l] * d.res[l];
    g.res[l] = d.res[l];
    g.off[l] = off;
    g.noff[l] = noff;
    off += g.ch * r3;
    noff += r3;
  }
  g.size = off;
  g.nodes = noff;
  g.scale = d.level_scale;
  return g;
}

namespace {

int bits_for(unsigned long long maxkey) {
  int b = 1;
  while (b < 32 && (1ull << b) <= maxkey) ++b;
  return b;
}

bool aligned4(const void *p) { return ((uintptr_t)p & 3) == 0; }

// Workspaces are carved into 256-byte aligned buffers (float4 and double
// accesses), so the base must be 256-byte aligned itself.
pdg_status need_ws(const void *ws, size_t have, size_t want) {
  if (!ws || have < want) {
    set_error("workspace of %zu bytes < %zu needed", have, want);
    return PDG_ENOMEM;
  }
  if (((uintptr_t)ws & 255) != 0) {
    set_error("workspace must be 256-byte aligned");
    return PDG_EINVAL;
  }
  return PDG_OK;
}

pdg_status need(const void *p, const char *name) {
  if (!p) {
    set_error("%s is NULL", name);
    return PDG_EINVAL;
  }
  if (!aligned4(p)) {
    set_error("%s is not 4-byte aligned", name);
    return PDG_EINVAL;
  }
  return PDG_OK;
}

// ------------------------------------------------------ deform backward --
struct DeformBwdWs {
  uint32_t *keys, *vals;
  int *pstart;
  float4 *ent;
  float2 *ent2;
  float *gscratch;
  float *u;                  // six-channel cells: d<g, out>/dz^, [3][n]
  void *sort;
};
DeformBwdWs deform_bwd_layout(Carve &c, const GridDev &g, long long n) {
  DeformBwdWs w;
  const long long ne = (long long)g.levels * n;
  w.keys = c.take<uint32_t>(ne);
  w.vals = c.take<uint32_t>(ne);
  w.pstart = c.take<int>(row_count(g) + 1);
  w.ent = c.take<float4>(ne);
  w.ent2 = c.take<float2>(ne);
  w.gscratch = c.take<float>((long long)(gather_scratch_bytes(g, 1, n) / sizeof(float)));
  w.u = g.ch == 6 ? c.take<float>(3 * n) : nullptr;
  w.sort = c.take<char>((long long)radix_sort_bytes(ne));
  return w;
}

// Builds the sorted entries and plane table of one scatter list (skipped for
// lists whose sample positions never change).
pdg_status scatter_entries(const GridDev &g, int segs, const ScatterList &L, uint32_t *keys,
                           uint32_t *vals, int *pstart, void *sort, hipStream_t st) {
  const long long nent = (long long)segs * g.levels * L.S;
  PDG_TRY(launch_scatter_keys(g, L.x, L.xstride, L.ldx, L.S, segs, keys, vals, st));
  // keys are below segs * nodes: sort only the bits they can set
  PDG_TRY(radix_sort(keys, vals, nent, bits_for((unsigned long long)segs * g.nodes - 1), sort, st));
  return launch_row_table(g, keys, nent, segs, pstart, st);
}

ScatterList scatter_list(const uint32_t *keys, const uint32_t *vals, const int *pstart,
                         long long S, const float *x, long long xstride, long long ldx,
                         const float *lam, long long lstride, long long ldl, float4 *ent,
                         float2 *ent2) {
  ScatterList L;
  L.ent = ent;
  L.ent2 = ent2;
  L.keys = keys;
  L.vals = vals;
  L.pstart = pstart;
  L.S = S;
  L.x = x;
  L.xstride = xstride;
  L.ldx = ldx;
  L.lam = lam;
  L.lstride = lstride;
  L.ldl = ldl;
  return L;
}

// --------------------------------------------------------------- chamfer --
ScreenSet screen_set(const float *x, long long n, const int *perm, uint4 *pack, float4 *coords,
                     float4 *boxes, int *inv = nullptr) {
  ScreenSet S;
  memset(&S, 0, sizeof S);
  S.x = x;
  S.n = (int)n;
  S.perm = perm;
  S.pack = pack;
  S.coords = coords;
  S.boxes = boxes;
  S.inv = inv;
  return S;
}
// queries from set Q, candidates from set C
ScreenJob screen_job(const ScreenSet &Q, const ScreenSet &C, int *nn, unsigned long long *tiles) {
  ScreenJob J;
  memset(&J, 0, sizeof J);
  J.c = C.x;
  J.q = Q.coords;
  J.qboxes = Q.boxes;
  J.nq = Q.n;
  J.nc = C.n;
  J.nn = nn;
  J.pack = C.pack;
  J.cc = C.coords;
  J.cboxes = C.boxes;
  J.tiles = tiles;
  J.cinv = C.inv;
  return J;
}

struct ChamferWs {
  NNJob *jobs;
  ChSeg *segs;
  unsigned *b_base;
  double *partials, *w_default;
  uint32_t *keys, *vals;
  float4 *rpart;
  void *sort;
  ScreenSet *ssets;
  ScreenJob *sjobs;
  uint4 *pack_a, *pack_b;
  float4 *coords_a, *coords_b, *boxes_a, *boxes_b;
  uint32_t *perm_a, *perm_b;
};
ChamferWs chamfer_layout(Carve &c, long long n, long long m, int mode) {
  ChamferWs w;
  memset(&w, 0, sizeof w);
  if (uses_packs(mode)) {
    w.ssets = c.take<ScreenSet>(2);
    w.sjobs = c.take<ScreenJob>(2);
    if (mode == PDG_CHAMFER_BF16_SCREEN) {   // bf16 rows (the exact culled search reads coordinates)
      w.pack_a = c.take<uint4>(2 * n);
      w.pack_b = c.take<uint4>(2 * m);
    }
    w.coords_a = c.take<float4>(n);
    w.coords_b = c.take<float4>(m);
    w.boxes_a = c.take<float4>(screen_box_count(n));
    w.boxes_b = c.take<float4>(screen_box_count(m));
    w.perm_a = c.take<uint32_t>(n);
    w.perm_b = c.take<uint32_t>(m);
  }
  const long long nk = uses_packs(mode) && n > m ? n : m;   // sort entries
  w.jobs = c.take<NNJob>(2);
  w.segs = c.take<ChSeg>(1);
  w.b_base = c.take<unsigned>(1);
  w.partials = c.take<double>(2 * kLossBlocks);
  w.w_default = c.take<double>(2);
  w.keys = c.take<uint32_t>(nk);
  w.vals = c.take<uint32_t>(nk);
  w.rpart = c.take<float4>(2 * rev_part_count(nk));
  w.sort = c.take<char>((long long)radix_sort_bytes(nk));
  return w;
}

// Both directions of the robust Chamfer distance of a (n) and b (m) with the
// loss and, when ga is set, the gradient with respect to a (the body of
// pdg_chamfer, on a carved workspace).
pdg_status enqueue_chamfer(const ChamferWs &w, const float *a, long long n, const float *b,
                           long long m, double alpha, int mode, const double *dir_weight,
                           double *loss, int32_t *nn_a, int32_t *nn_b, float *ga,
                           hipStream_t stream) {
  NNJob jobs[2];
  memset(jobs, 0, sizeof jobs);
  jobs[0].q = a;
  jobs[0].c = b;
  jobs[0].nq = (int)n;
  jobs[0].nc = (int)m;
  jobs[0].nn = nn_a;
  jobs[1].q = b;
  jobs[1].c = a;
  jobs[1].nq = (int)m;
  jobs[1].nc = (int)n;
  jobs[1].nn = nn_b;
  ChSeg seg;
  memset(&seg, 0, sizeof seg);
  seg.a = a;
  seg.b = b;
  seg.n = (int)n;
  seg.m = (int)m;
  seg.nn_a = nn_a;
  seg.nn_b = nn_b;
  seg.ga = ga;
  seg.a_base = 0;
  seg.loss = loss;
  seg.part = w.partials;
  seg.w = dir_weight ? dir_weight : w.w_default;
  const unsigned bb = 0;
  const double ones[2] = {1.0, 1.0};
  PDG_TRY(upload_small(w.jobs, jobs, sizeof jobs, stream));
  PDG_TRY(upload_small(w.segs, &seg, sizeof seg, stream));
  PDG_TRY(upload_small(w.b_base, &bb, sizeof bb, stream));
  PDG_TRY(upload_small(w.w_default, ones, sizeof ones, stream));
  if (uses_packs(mode)) {
    ScreenSet ss[2];
    ScreenJob sj[2];
    memset(ss, 0, sizeof ss);
    memset(sj, 0, sizeof sj);
    // Morton order of both sets (the sorted index arrays are the permutations)
    PDG_TRY(launch_morton(a, n, (int)n, w.keys, w.perm_a, stream));
    PDG_TRY(radix_sort(w.keys, w.perm_a, n, 30, w.sort, stream));
    PDG_TRY(launch_morton(b, m, (int)m, w.keys, w.perm_b, stream));
    PDG_TRY(radix_sort(w.keys, w.perm_b, m, 30, w.sort, stream));
    ss[0] = screen_set(a, n, (const int *)w.perm_a, w.pack_a, w.coords_a, w.boxes_a);
    ss[1] = screen_set(b, m, (const int *)w.perm_b, w.pack_b, w.coords_b, w.boxes_b);
    sj[0] = screen_job(ss[0], ss[1], nn_a, nullptr);
    sj[1] = screen_job(ss[1], ss[0], nn_b, nullptr);
    PDG_TRY(upload_small(w.ssets, ss, sizeof ss, stream));
    PDG_TRY(upload_small(w.sjobs, sj, sizeof sj, stream));
    PDG_TRY(launch_screen_pack(w.ssets, 2, (int)(n > m ? n : m), stream));
    if (mode == PDG_CHAMFER_BF16_SCREEN)
      PDG_TRY(launch_nn_screen(w.sjobs, 2, (int)(n > m ? n : m), 0, stream));
    else
      PDG_TRY(launch_nn_cull(w.sjobs, 2, (int)(n > m ? n : m), 0, stream));
  } else {
    PDG_TRY(launch_nn_exact(w.jobs, 2, (int)(n > m ? n : m), stream));
  }
  PDG_TRY(launch_chamfer_loss(w.segs, 1, alpha, stream));
  if (ga) {
    PDG_TRY(launch_chamfer_grad_fwd(w.segs, 1, (int)n, (float)alpha, stream));
    PDG_TRY(launch_chamfer_rev_keys(w.segs, 1, (int)m, w.b_base, w.keys, w.vals, stream));
    PDG_TRY(radix_sort(w.keys, w.vals, m, bits_for((unsigned long long)n), w.sort, stream));
    PDG_TRY(launch_chamfer_rev_scatter(w.segs, 1, w.b_base, w.keys, w.vals, m, (float)alpha,
                                       w.rpart, stream));
  }
  return PDG_OK;
}

// ---------------------------------------------------------- precondition --
int cg_count(float lam, double tol) {
  const double kappa = 1.0 + 12.0 * (double)lam;
  const double sq = sqrt(kappa);
  const double rho = (sq - 1.0) / (sq + 1.0);
  if (rho <= 0.0) return 1;
  const double k = ceil(log(2.0 / tol) / -log(rho));
  return k < 1.0 ? 1 : (int)k;
}

// Per-level iteration counts: iters > 0 fixes them; otherwise the a-priori
// count for the A-norm tolerance from kappa <= 1 + 12 lambda.  lambda = 0
// gives A = I, where one iteration reproduces the input exactly.
CGPlanDev cg_plan(const GridDev &g, int batch, const float *lam, int iters, double tol,
                  bool aligned16) {
  int it[PDG_MAX_LEVELS];
  for (int l = 0; l < g.levels; ++l)
    it[l] = lam[l] == 0.0f ? 1 : (iters > 0 ? iters : cg_count(lam[l], tol));
  return cg_make_plan(g, batch, lam, it, aligned16);
}

pdg_status check_precond_args(const pdg_grid_desc *d, const float *lambda, int32_t batch,
                              int32_t method, int32_t iters, double tol) {
  PDG_TRY(check_grid(d));
  if (!lambda) {
    set_error("lambda is NULL");
    return PDG_EINVAL;
  }
  for (int l = 0; l < d->levels; ++l)
    if (!(lambda[l] >= 0.0f) || !isfinite(lambda[l])) {
      set_error("lambda[%d] must be finite and >= 0", l);
      return PDG_EINVAL;
    }
  if (batch < 0) {
    set_error("batch < 0");
    return PDG_EINVAL;
  }
  if (method != PDG_PRECOND_CG && method != PDG_PRECOND_DCT) {
    set_error("unknown preconditioner method %d", method);
    return PDG_EINVAL;
  }
  if (method == PDG_PRECOND_DCT) {
    for (int l = 0; l < d->levels; ++l)
      if (d->res[l] > 256) {
        set_error("DCT preconditioner supports R <= 256 (level %d has %d)", l, d->res[l]);
        return PDG_EUNSUPPORTED;
      }
    return PDG_OK;
  }
  if (iters < 0 || (iters == 0 && !(tol > 0.0 && tol < 1.0))) {
    set_error("iters must be >= 0, and tol in (0,1) when iters == 0");
    return PDG_EINVAL;
  }
  return PDG_OK;
}

size_t cg_ws_bytes(const CGPlanDev &p, long long floats) {
  return cg_bytes(floats, p.nsys, p.ntiles);
}

}  // namespace
}  // namespace pdg

using namespace pdg;

// ----------------------------------------------------------------- problem --
struct pdg_problem {
  pdg_problem_desc d;
  GridDev g;
  int T = 0, F = 0;
  long long N = 0, V = 0, E = 0, P = 0;
  bool has_tm = false;
  // intermediate buffers (carved from the workspace)
  float *phat = nullptr, *xhat = nullptr, *grad = nullptr, *pgrad = nullptr;
  float *gphat = nullptr, *gxhat = nullptr, *lam = nullptr, *sig = nullptr, *u = nullptr;
  int *nn = nullptr, *inc_off = nullptr, *epoch = nullptr;
  double *losses = nullptr, *w = nullptr, *wconf = nullptr, *terms = nullptr;
  double *partials = nullptr, *iso_partials = nullptr;
  uint32_t *pkeys = nullptr, *pvals = nullptr, *tkeys = nullptr, *tvals = nullptr;
  int *pstart_p = nullptr, *pstart_t = nullptr;   // row tables (points, template)
  float4 *ent_p = nullptr, *ent_t = nullptr;       // staged scatter entries
  float2 *ent2_p = nullptr, *ent2_t = nullptr;
  float *gscratch = nullptr;                       // partial bands of the split gather
  uint32_t *rkeys = nullptr, *rvals = nullptr, *ikeys = nullptr, *ivals = nullptr;
  float4 *rpart = nullptr;                         // run partials of the reverse scatter
  void *sort = nullptr;
  NNJob *jobs = nullptr;
  ScreenSet *ssets = nullptr;          // nseg moving sets, then T fixed frames
  ScreenJob *sjobs = nullptr;
  uint4 *packs = nullptr;
  float4 *coords = nullptr, *boxes = nullptr;
  int *pinv = nullptr;                 // packed sets: original index -> packed position
  int *fperm = nullptr, *tperm = nullptr;   // Morton order of every frame / of X_0
  unsigned long long *tiles = nullptr;     // candidate tiles screened (all steps)
  long long pack_rows = 0, box_tiles = 0;
  ChSeg *segs = nullptr;
  unsigned *b_base = nullptr;
  void *cgws = nullptr;
  void *dctws = nullptr;
  float lambda_l[PDG_MAX_LEVELS];    // preconditioner weight per level
  int njobs = 0, nseg = 0, max_nq = 0, max_n = 0, max_m = 0;
  long long nrev = 0;
  CGPlanDev cg;
  AdamLevels adam;
  unsigned fused = 0u;                             // levels whose Adam ran in the preconditioner
  // six-channel cells [z; t] (Eq. 4-7): rotation adjoints of the point and
  // template samples, and the conjugate-gradient plan of the t half
  float *u_p = nullptr, *u_t = nullptr;
  int *klist = nullptr;                            // kept CG tiles of pruned grids
  CGPlanDev cg_t;
  // optimisation of X_0 (Eq. 10, Sec. 3.6)
  bool opt_x0 = false;
  float *gx0 = nullptr, *pgx0 = nullptr;           // dL_mesh/dX_0, preconditioned
  int *nn0 = nullptr;                              // [V + N]
  double *loss0 = nullptr;                         // [2]
  ChamferWs cw0;                                   // Chamfer workspace of (X_0, P_0)
  void *meshws = nullptr;
  int max_degree = 0;
  MeshPlan *mesh = nullptr;                        // its preconditioner's plan (in meshws)
  // Eq. 14 and 17 across the two chains of a sequence whose keyframe lies
  // inside it (reverse-time propagation): the 1/T count and the other chain
  long long Tn = 0;
  const double *partner_losses = nullptr;
  int partner_T = 0;
  // such a sequence is a joint handle over the backward (0) and forward (1)
  // chains; the backward chain reads a reversed copy of frames k..0
  bool joint = false;
  pdg_problem *child[2] = {nullptr, nullptr};
  float *rev_points = nullptr;
  double *jterms = nullptr;
  size_t ws_used = 0;
  // graph replay
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~pdg_problem() { mesh_plan_free(mesh); }
};

namespace pdg {
namespace {

pdg_status check_problem(const pdg_problem_desc *pd) {
  if (!pd) {
    set_error("problem descriptor is NULL");
    return PDG_EINVAL;
  }
  PDG_TRY(check_grid(&pd->grid, true));
  if (pd->frames < 2) {
    set_error("frames = %d: need at least 2", pd->frames);
    return PDG_EINVAL;
  }
  if (pd->keyframe < 0 || pd->keyframe >= pd->frames) {
    set_error("keyframe = %d outside [0, frames)", pd->keyframe);
    return PDG_EINVAL;
  }
  if (pd->n < 1 || pd->n >= (1ll << 31)) {
    set_error("n = %lld outside [1, 2^31)", (long long)pd->n);
    return PDG_EINVAL;
  }
  if (pd->verts < 0 || pd->n_edges < 0 || (pd->verts == 0 && pd->n_edges > 0)) {
    set_error("verts/n_edges invalid");
    return PDG_EINVAL;
  }
  PDG_TRY(need(pd->points, "points"));
  if (pd->verts > 0) PDG_TRY(need(pd->template_verts, "template_verts"));
  if (pd->n_edges > 0) PDG_TRY(need(pd->edges, "edges"));
  PDG_TRY(need(pd->params, "params"));
  PDG_TRY(need(pd->adam_m, "adam_m"));
  PDG_TRY(need(pd->adam_v, "adam_v"));
  if (pd->chamfer_mode != PDG_CHAMFER_FP32 && !uses_packs(pd->chamfer_mode)) {
    set_error("unknown chamfer mode %d", pd->chamfer_mode);
    return PDG_EINVAL;
  }
  const pdg_hyper &h = pd->hp;
  if (!(h.alpha >= 0.0) || !isfinite(h.alpha) || !(h.w_iso >= 0.f) || !(h.eta0 > 0.f) || !(h.eta_growth > 0.f) ||
      !(h.lambda0 >= 0.f) || !(h.lambda_growth > 0.f) || !(h.beta1 >= 0.f && h.beta1 < 1.f) ||
      !(h.beta2 >= 0.f && h.beta2 < 1.f) || !(h.eps > 0.f) || h.e_max < 1) {
    set_error("hyperparameters out of range");
    return PDG_EINVAL;
  }
  float lam[PDG_MAX_LEVELS];
  for (int l = 0; l < pd->grid.levels; ++l) lam[l] = pd->hp.lambda0 * powf(pd->hp.lambda_growth, (float)l);
  pdg_grid_desc d3 = pd->grid;   // six channels are preconditioned as two three-channel halves
  d3.channels = 3;
  PDG_TRY(check_precond_args(&d3, lam, 1, pd->precond_method, pd->cg_iters, pd->cg_tol));
  if ((pd->template_adam_m || pd->template_adam_v) &&
      (!pd->template_adam_m || !pd->template_adam_v || pd->verts < 1 ||
       !(pd->hp.mesh_lambda >= 0.f) || !isfinite(pd->hp.mesh_lambda) || !(pd->hp.mesh_lr > 0.f))) {
    set_error("optimising X_0 needs both template Adam moments, verts >= 1, mesh_lambda >= 0 "
              "and mesh_lr > 0");
    return PDG_EINVAL;
  }
  if (pd->prune_mask && pd->precond_method != PDG_PRECOND_CG) {
    set_error("pruned grids need the conjugate-gradient preconditioner");
    return PDG_EUNSUPPORTED;
  }
  const GridDev g = make_grid(pd->grid);
  const long long T = pd->frames - 1;
  if ((unsigned long long)T * g.nodes >= (1ull << 32)) {
    set_error("T * nodes = %lld does not fit the 32-bit scatter keys", T * g.nodes);
    return PDG_EINVAL;
  }
  if ((unsigned long long)T * g.levels * (pd->n > pd->verts ? pd->n : pd->verts) >= (1ull << 31)) {
    set_error("T * levels * samples exceeds 2^31 scatter entries");
    return PDG_EINVAL;
  }
  if ((unsigned long long)T * (pd->n + pd->verts) >= (1ull << 31)) {
    set_error("T * (n + V) exceeds 2^31");
    return PDG_EINVAL;
  }
  return PDG_OK;
}

// Lays out (or sizes, with base == nullptr) every buffer of a problem.
void layout(pdg_problem &p, Carve &c) {
  const long long T = p.T, F = p.F, N = p.N, V = p.V, E = p.E, P = p.P, L = p.g.levels;
  p.phat = c.take<float>(T * 3 * N);
  p.xhat = c.take<float>(F * 3 * V);
  p.nn = c.take<int>(T * (2 * N + V + N));
  p.losses = c.take<double>(4 * T);
  p.w = c.take<double>(4 * T);
  p.wconf = c.take<double>(T);
  p.terms = c.take<double>(kTerms);
  p.partials = c.take<double>(4 * T * kLossBlocks);
  p.iso_partials = c.take<double>(kIsoBlocks);
  p.grad = c.take<float>(T * P);
  p.pgrad = c.take<float>(T * P);
  p.gphat = c.take<float>(T * 3 * N);
  p.gxhat = c.take<float>(T * 3 * V);
  p.lam = c.take<float>(T * 3 * V);
  p.sig = c.take<float>(T * E);
  p.u = c.take<float>(T * 3 * E);
  p.inc_off = c.take<int>(V + 1);
  p.epoch = c.take<int>(1);
  p.pkeys = c.take<uint32_t>(T * L * N);
  p.pvals = c.take<uint32_t>(T * L * N);
  p.tkeys = c.take<uint32_t>(T * L * V);
  p.tvals = c.take<uint32_t>(T * L * V);
  p.pstart_p = c.take<int>(T * row_count(p.g) + 1);
  p.pstart_t = c.take<int>(T * row_count(p.g) + 1);
  p.ent_p = c.take<float4>(T * L * N);
  p.ent2_p = c.take<float2>(T * L * N);
  p.ent_t = c.take<float4>(T * L * V);
  p.ent2_t = c.take<float2>(T * L * V);
  p.gscratch = c.take<float>((long long)(gather_scratch_bytes(p.g, (int)T, N + V) / sizeof(float)));
  p.nrev = T * N * (p.has_tm ? 2 : 1);
  p.rkeys = c.take<uint32_t>(p.nrev);
  p.rvals = c.take<uint32_t>(p.nrev);
  p.rpart = c.take<float4>(2 * rev_part_count(p.nrev));
  p.ikeys = c.take<uint32_t>(2 * E);
  p.ivals = c.take<uint32_t>(2 * E);
  long long smax = T * L * N;
  if (T * L * V > smax) smax = T * L * V;
  if (p.nrev > smax) smax = p.nrev;
  if (2 * E > smax) smax = 2 * E;
  p.sort = c.take<char>((long long)radix_sort_bytes(smax));
  if (p.g.ch == 6) {
    p.u_p = c.take<float>(T * 3 * N);
    p.u_t = c.take<float>(T * 3 * V);
  }
  if (p.opt_x0) {
    p.gx0 = c.take<float>(3 * V);
    p.pgx0 = c.take<float>(3 * V);
    p.nn0 = c.take<int>(V + N);
    p.loss0 = c.take<double>(2);
    p.cw0 = chamfer_layout(c, V, N, p.d.chamfer_mode);
    p.meshws = c.take<char>((long long)mesh_precond_bytes(V, E));
  }
  p.nseg = (int)(p.has_tm ? 2 * T : T);
  p.njobs = 2 * p.nseg;
  p.jobs = c.take<NNJob>(p.njobs);
  if (uses_packs(p.d.chamfer_mode)) {
    // every segment packs its moving set A and its fixed set B
    // moving sets (P^_t, then X_t) are packed every step, the frames P_1..P_T once
    p.pack_rows = T * N + (p.has_tm ? T * V : 0) + T * N;
    p.box_tiles = T * screen_box_count(N) + (p.has_tm ? T * screen_box_count(V) : 0) + T * screen_box_count(N);
    p.ssets = c.take<ScreenSet>(p.nseg + T);
    p.sjobs = c.take<ScreenJob>(p.njobs);
    if (p.d.chamfer_mode == PDG_CHAMFER_BF16_SCREEN) p.packs = c.take<uint4>(2 * p.pack_rows);
    p.coords = c.take<float4>(p.pack_rows);
    p.pinv = c.take<int>(p.pack_rows);
    p.boxes = c.take<float4>(p.box_tiles);
    p.tiles = c.take<unsigned long long>(1);
  }
  p.fperm = c.take<int>(F * N);
  p.tperm = c.take<int>(V);
  p.segs = c.take<ChSeg>(p.nseg);
  p.b_base = c.take<unsigned>(p.nseg);
  if (p.d.precond_method == PDG_PRECOND_DCT)
    p.dctws = c.take<char>((long long)dct_bytes(p.g));
  else
    p.cgws = c.take<char>((long long)cg_bytes(T * P, p.cg.nsys, p.cg.ntiles));
  if (p.d.prune_mask) p.klist = c.take<int>(p.cg.ntiles > 0 ? p.cg.ntiles : 1);
}

void init_problem(pdg_problem &p, const pdg_problem_desc &pd) {
  p.d = pd;
  p.g = make_grid(pd.grid);
  p.F = pd.frames;
  p.T = pd.frames - 1;
  p.N = pd.n;
  p.V = pd.verts;
  p.E = pd.verts > 0 ? pd.n_edges : 0;
  p.P = p.g.size;
  p.has_tm = p.V > 0;
  p.opt_x0 = p.has_tm && pd.template_adam_m && pd.template_adam_v;
  p.Tn = p.T;
  float *lam = p.lambda_l;
  p.adam.levels = p.g.levels;
  for (int l = 0; l < p.g.levels; ++l) {
    lam[l] = pd.hp.lambda0 * powf(pd.hp.lambda_growth, (float)l);
    p.adam.lr[l] = pd.hp.eta0 * powf(pd.hp.eta_growth, (float)l);
    p.adam.off[l] = p.g.off[l];
  }
  p.adam.off[p.g.levels] = p.g.size;
  // every buffer the solver touches is carved at 256-byte alignment
  if (p.g.ch == 6) {   // each half of the six channels is preconditioned as a grid
    p.cg = cg_plan(half_view(p.g, 0), p.T, lam, pd.cg_iters, pd.cg_tol, true);
    p.cg_t = cg_plan(half_view(p.g, 1), p.T, lam, pd.cg_iters, pd.cg_tol, true);
  } else {
    p.cg = cg_plan(p.g, p.T, lam, pd.cg_iters, pd.cg_tol, true);
  }
  if (pd.prune_mask) {   // six channels: both halves on the same kept cells
    cg_set_mask(p.cg, p.g, pd.prune_mask);
    if (p.g.ch == 6) cg_set_mask(p.cg_t, p.g, pd.prune_mask);
    adam_set_mask(p.adam, p.g, pd.prune_mask);
  }
}

IsoArgs iso_args(pdg_problem &p) {
  IsoArgs ia;
  ia.xhat = p.xhat;
  ia.edges = p.d.edges;
  ia.V = (int)p.V;
  ia.E = (int)p.E;
  ia.T = p.T;
  ia.sig = p.sig;
  ia.u = p.u;
  ia.partials = p.iso_partials;
  ia.inc_off = p.inc_off;
  ia.inc = p.ivals;
  ia.gx = p.gxhat;
  ia.coef = p.E > 0 ? (double)p.d.hp.w_iso / ((double)p.Tn * (double)p.E) : 0.0;
  return ia;
}

// The loss stage in two halves (a sequence's two chains both compute their
// terms before either assembles: cd_max spans both).
constexpr int kStageLossTerms = 100;
// series tolerance of the mesh preconditioner in a problem's TEMPLATE stage
constexpr double kMeshTol = 1e-8;
constexpr int kStageAssemble = 101;

// Parts of a stage that a batch of problems runs as one launch over its
// merged job tables (see pdg_batch) and a member therefore skips.
constexpr unsigned kSkipPack = 1u, kSkipNN = 2u, kSkipChamferLoss = 4u;
constexpr unsigned kSkipMerged = kSkipPack | kSkipNN | kSkipChamferLoss;

// One stage of the step (the stages in order make one iteration).
// fuse: part of a full step (the preconditioner may apply Adam itself, see
// run_dct); false for stages enqueued one at a time.
pdg_status enqueue_stage(pdg_problem &p, int stage, hipStream_t st, double *user_terms,
                         bool fuse, unsigned skip = 0u) {
  const GridDev &g = p.g;
  const long long T = p.T, N = p.N, V = p.V, P = p.P;
  const pdg_hyper &h = p.d.hp;
  switch (stage) {
    case PDG_STAGE_WARP:  // P^_t = warp(G_t, P_{t-1}); X_t = warp(G_t, X_{t-1}) (Eq. 1, 8)
      if (g.ch == 6) {   // x' = R(z^) x + t^ (Eq. 5-7), one launch per transition
        PDG_TRY(launch_warp6_batch(g, p.d.params, P, p.d.points, 3 * N, p.phat, 3 * N, N, (int)T,
                                   st));
        if (p.has_tm) {
          PDG_TRY(launch_copy(p.xhat, p.d.template_verts, 3 * V, st));
          PDG_TRY(launch_chain_warp6(g, p.d.params, P, p.xhat, V, (int)T, st));
        }
      } else {
        // points and vertices in Morton order of P_t and X_0 (cache reuse of grid cells)
        PDG_TRY(launch_warp(g, p.d.params, P, p.d.points, 3 * N, N, p.phat, 3 * N, N, N, (int)T,
                            st, p.fperm, N));
        if (p.has_tm)
          PDG_TRY(launch_chain_warp(g, p.d.params, P, p.d.template_verts, p.xhat, V, (int)T,
                                    p.tperm, st));
      }
      if (uses_packs(p.d.chamfer_mode) && !(skip & kSkipPack))
        PDG_TRY(launch_screen_pack(p.ssets, p.nseg, p.max_n, st));   // the moving sets P^_t, X_t
      return PDG_OK;
    case PDG_STAGE_NN:  // nearest neighbours (Eq. 12)
      if (skip & kSkipNN) return PDG_OK;
      if (p.d.chamfer_mode == PDG_CHAMFER_BF16_SCREEN)   // warm start: last step's assignment
        return launch_nn_screen(p.sjobs, p.njobs, p.max_nq, 1, st);
      if (p.d.chamfer_mode == PDG_CHAMFER_FP32_CULL)
        return launch_nn_cull(p.sjobs, p.njobs, p.max_nq, 1, st);
      return launch_nn_exact(p.jobs, p.njobs, p.max_nq, st);
    case PDG_STAGE_LOSS:  // CD_R (Eq. 11, 13), L_iso (Eq. 18), w_conf and L (Eq. 9, 14-17)
      PDG_TRY(enqueue_stage(p, kStageLossTerms, st, user_terms, fuse, skip));
      return enqueue_stage(p, kStageAssemble, st, user_terms, fuse, skip);
    case kStageLossTerms:  // the Chamfer terms and the isometry partials
      if (!(skip & kSkipChamferLoss)) PDG_TRY(launch_chamfer_loss(p.segs, p.nseg, h.alpha, st));
      if (p.has_tm && p.E > 0) PDG_TRY(launch_iso_edges(iso_args(p), st));
      return PDG_OK;
    case kStageAssemble: {  // cd_max, w_conf, L
      AssembleArgs aa;
      aa.losses = p.losses;
      aa.iso_partials = p.iso_partials;
      aa.T = (int)T;
      aa.E = (int)p.E;
      aa.has_tm = p.has_tm ? 1 : 0;
      aa.epoch = p.epoch;
      aa.e_max = h.e_max;
      aa.w_iso = h.w_iso;
      aa.w = p.w;
      aa.wconf = p.wconf;
      aa.terms = p.terms;
      aa.user_terms = user_terms;
      aa.Tn = (int)p.Tn;
      aa.partner_losses = p.partner_losses;
      aa.partner_T = p.partner_T;
      return launch_assemble(aa, st);
    }
    case PDG_STAGE_GRAD:  // dL/dP^, dL/dX (Chamfer adjoint, isometry), reverse sweep of Eq. 8
      PDG_TRY(launch_chamfer_grad_fwd(p.segs, p.nseg, p.max_n, (float)h.alpha, st));
      PDG_TRY(launch_chamfer_rev_keys(p.segs, p.nseg, p.max_m, p.b_base, p.rkeys, p.rvals, st));
      PDG_TRY(radix_sort(p.rkeys, p.rvals, p.nrev,
                         bits_for((unsigned long long)(T * N + T * V)), p.sort, st));
      PDG_TRY(launch_chamfer_rev_scatter(p.segs, p.nseg, p.b_base, p.rkeys, p.rvals, p.nrev,
                                         (float)h.alpha, p.rpart, st));
      if (p.has_tm && p.E > 0) PDG_TRY(launch_iso_vertices(iso_args(p), st));
      if (g.ch == 6) {
        // reverse sweep of Eq. 8 one transition at a time: lam_{t-1} = direct
        // + J_t^T lam_t, with the rotation adjoint u_t of every vertex on the way
        if (p.has_tm)
          PDG_TRY(launch_chain_reverse6(g, p.d.params, P, p.xhat, p.gxhat, p.lam, p.u_t, V,
                                        (int)T, st));
        PDG_TRY(launch_adjoint6_batch(g, p.d.params, P, p.d.points, 3 * N, p.gphat, 3 * N, p.u_p,
                                      3 * N, nullptr, nullptr, 0, N, (int)T, st));
        return PDG_OK;
      }
      if (p.has_tm)
        PDG_TRY(launch_chain_reverse(g, p.d.params, P, p.xhat, p.gxhat, p.lam, V, (int)T,
                                     p.tperm, st));
      return PDG_OK;
    case PDG_STAGE_SCATTER: {  // dL/dG: deterministic transpose of Eq. 1
      ScatterLists sl;
      sl.count = 1;
      sl.list[0] = scatter_list(p.pkeys, p.pvals, p.pstart_p, N, p.d.points, 3 * N, N, p.gphat,
                                3 * N, N, p.ent_p, p.ent2_p);
      PDG_TRY(launch_scatter_stage(g, (int)T, sl.list[0], st, true));   // fractions staged at creation
      if (p.has_tm) {
        sl.list[1] = scatter_list(p.tkeys, p.tvals, p.pstart_t, V, p.xhat, 3 * V, V, p.lam,
                                  3 * V, V, p.ent_t, p.ent2_t);
        sl.count = 2;
        PDG_TRY(scatter_entries(g, (int)T, sl.list[1], p.tkeys, p.tvals, p.pstart_t, p.sort, st));
        PDG_TRY(launch_scatter_stage(g, (int)T, sl.list[1], st));
      }
      if (g.ch != 6) return launch_gather(g, (int)T, sl, N + V, p.grad, p.gscratch, st);
      // six channels: translation channels from the position adjoints, then
      // the rotation channels from u on the same sorted entries
      PDG_TRY(launch_gather(g, (int)T, sl, N + V, p.grad, p.gscratch, st, 3));
      sl.list[0].lam = p.u_p;
      PDG_TRY(launch_scatter_stage(g, (int)T, sl.list[0], st, true));
      if (p.has_tm) {
        sl.list[1].lam = p.u_t;
        PDG_TRY(launch_scatter_stage(g, (int)T, sl.list[1], st, true));
      }
      return launch_gather(g, (int)T, sl, N + V, p.grad, p.gscratch, st, 0);
    }
    case PDG_STAGE_PRECOND:  // (I + lambda_l L_l)^-2 (Eq. 3)
      p.fused = 0u;
      if (g.ch == 6) {   // each half of the six channels as a three-channel grid
        PDG_TRY(launch_copy(p.pgrad, p.grad, T * P, st));
        for (int half = 0; half < 2; ++half) {
          if (p.d.precond_method == PDG_PRECOND_DCT)
            PDG_TRY(run_dct(half_view(g, half), (int)T, p.lambda_l, p.pgrad, p.pgrad, p.dctws, st));
          else
            PDG_TRY(run_cg(half ? p.cg_t : p.cg, p.pgrad, T * P, p.cgws, st));
        }
        return PDG_OK;
      }
      if (p.d.precond_method == PDG_PRECOND_DCT) {
        if (!fuse) return run_dct(g, (int)T, p.lambda_l, p.grad, p.pgrad, p.dctws, st);
        // full step: levels whose last inverse pass can apply Adam do so
        AdamFuse af;
        af.th = p.d.params;
        af.m = p.d.adam_m;
        af.v = p.d.adam_v;
        af.lv = p.adam;
        af.b1 = h.beta1;
        af.b2 = h.beta2;
        af.eps = h.eps;
        af.step_dev = p.epoch;
        af.step_host = 0;
        return run_dct(g, (int)T, p.lambda_l, p.grad, p.pgrad, p.dctws, st, &af, &p.fused);
      }
      PDG_TRY(launch_copy(p.pgrad, p.grad, T * P, st));
      return run_cg(p.cg, p.pgrad, T * P, p.cgws, st);
    case PDG_STAGE_ADAM:  // Sec. 3.6 (levels not already updated by the preconditioner)
      return launch_adam_levels(p.adam, fuse ? p.fused : 0u, P, (int)T, h.beta1, h.beta2, h.eps,
                                p.epoch, 0, p.d.params, p.d.adam_m, p.d.adam_v, p.pgrad, st);
    case PDG_STAGE_TEMPLATE: {  // X_0: L_mesh = CD_R(X_0, P_0) (Eq. 10), Sec. 3.6
      if (!p.opt_x0) {
        set_error("the TEMPLATE stage needs X_0 to be optimised (template Adam moments)");
        return PDG_EINVAL;
      }
      float *x0 = const_cast<float *>(p.d.template_verts);
      PDG_TRY(enqueue_chamfer(p.cw0, x0, V, p.d.points, N, h.alpha, p.d.chamfer_mode, nullptr,
                              p.loss0, p.nn0, p.nn0 + V, p.gx0, st));
      PDG_TRY(launch_mesh_terms(p.terms, user_terms, p.loss0, st));
      // (I + mesh_lambda L)^-2 with the mesh Laplacian, then Adam with mesh_lr
      PDG_TRY(mesh_plan_apply(*p.mesh, p.gx0, p.pgx0, st));   // plan built at creation
      AdamLevels al;
      memset(&al, 0, sizeof al);
      al.levels = 1;
      al.off[0] = 0;
      al.off[1] = 3 * V;
      al.lr[0] = h.mesh_lr;
      return launch_adam(al, 3 * V, 1, h.beta1, h.beta2, h.eps, p.epoch, 0, x0,
                         p.d.template_adam_m, p.d.template_adam_v, p.pgx0, st);
    }
    default:
      set_error("unknown stage %d", stage);
      return PDG_EINVAL;
  }
}

pdg_status enqueue_precond_adam(pdg_problem &p, hipStream_t st) {
  PDG_TRY(enqueue_stage(p, PDG_STAGE_PRECOND, st, nullptr, true));
  return enqueue_stage(p, PDG_STAGE_ADAM, st, nullptr, true);
}

// A stage of a sequence propagated both ways: the stage on each chain (the
// loss stage's halves interleaved), then the sequence's terms.
pdg_status enqueue_joint_stage(pdg_problem &J, int stage, hipStream_t st, double *user_terms,
                               bool fuse) {
  pdg_problem *const *ch = J.child;
  if (stage == PDG_STAGE_LOSS) {
    for (int c = 0; c < 2; ++c)
      if (ch[c]) PDG_TRY(enqueue_stage(*ch[c], kStageLossTerms, st, nullptr, fuse));
    for (int c = 0; c < 2; ++c)
      if (ch[c]) PDG_TRY(enqueue_stage(*ch[c], kStageAssemble, st, nullptr, fuse));
  } else if (stage == PDG_STAGE_TEMPLATE) {
    pdg_problem *m = ch[1] && ch[1]->opt_x0 ? ch[1] : ch[0];
    if (!m || !m->opt_x0) {
      set_error("the TEMPLATE stage needs X_0 to be optimised (template Adam moments)");
      return PDG_EINVAL;
    }
    PDG_TRY(enqueue_stage(*m, stage, st, nullptr, fuse));
  } else {
    for (int c = 0; c < 2; ++c)
      if (ch[c]) {
        if (stage == PDG_STAGE_PRECOND_ADAM)
          PDG_TRY(enqueue_precond_adam(*ch[c], st));
        else
          PDG_TRY(enqueue_stage(*ch[c], stage, st, nullptr, fuse));
      }
  }
  if (stage == PDG_STAGE_LOSS || stage == PDG_STAGE_TEMPLATE)
    return launch_joint_terms(ch[0] ? ch[0]->terms : nullptr, ch[1] ? ch[1]->terms : nullptr,
                              J.jterms, user_terms, st);
  return PDG_OK;
}

pdg_status enqueue_step(pdg_problem &p, hipStream_t st, double *user_terms) {
  if (p.joint) {
    for (int s = PDG_STAGE_WARP; s <= PDG_STAGE_ADAM; ++s)
      PDG_TRY(enqueue_joint_stage(p, s, st, user_terms, true));
    if (p.opt_x0) PDG_TRY(enqueue_joint_stage(p, PDG_STAGE_TEMPLATE, st, user_terms, true));
    return PDG_OK;
  }
  for (int s = PDG_STAGE_WARP; s <= PDG_STAGE_ADAM; ++s)
    PDG_TRY(enqueue_stage(p, s, st, user_terms, true));
  if (p.opt_x0) PDG_TRY(enqueue_stage(p, PDG_STAGE_TEMPLATE, st, user_terms, true));
  return PDG_OK;
}

// -------------------------------------------------------------- batches --
// One iteration of several problems (served requests) at once.  The screen
// pack, the nearest-neighbour search and the Chamfer loss of every member run
// as one launch each over merged device tables (the members' job tables
// copied one after another into the batch's workspace); every other stage is
// the member's own, enqueued on one of kBatchLanes branches of the captured
// graph so that the members' kernels overlap.  A job writes only its own
// problem's buffers, so a member's results do not depend on the batch.
constexpr int kBatchLanes = 4;

}  // namespace
}  // namespace pdg

struct pdg_batch {
  std::vector<pdg_problem *> members;
  int mode = 0;
  double alpha = 0.0;
  ScreenSet *ssets = nullptr;      // merged moving sets (screen mode)
  ScreenJob *sjobs = nullptr;      // merged screen jobs
  NNJob *jobs = nullptr;           // merged exact jobs
  ChSeg *segs = nullptr;           // merged Chamfer segments
  int nsets = 0, njobs = 0, nseg = 0, max_n = 0, max_nq = 0;
  hipStream_t cap = nullptr, lane[kBatchLanes] = {};
  hipEvent_t fork[2] = {}, join[2][kBatchLanes] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace pdg {
namespace {

struct BatchTables {
  ScreenSet *ssets;
  ScreenJob *sjobs;
  NNJob *jobs;
  ChSeg *segs;
};
BatchTables batch_layout(Carve &c, int mode, int nsets, int njobs, int nseg) {
  BatchTables t;
  memset(&t, 0, sizeof t);
  if (uses_packs(mode)) {
    t.ssets = c.take<ScreenSet>(nsets);
    t.sjobs = c.take<ScreenJob>(njobs);
  } else {
    t.jobs = c.take<NNJob>(njobs);
  }
  t.segs = c.take<ChSeg>(nseg);
  return t;
}

pdg_status check_batch(pdg_problem *const *ps, int32_t count) {
  if (count < 1 || !ps) {
    set_error("a batch needs at least one problem");
    return PDG_EINVAL;
  }
  for (int i = 0; i < count; ++i) {
    if (!ps[i]) {
      set_error("batch member %d is NULL", i);
      return PDG_EINVAL;
    }
    if (ps[i]->joint) {
      set_error("batch member %d propagates from a keyframe inside its sequence; step it alone", i);
      return PDG_EUNSUPPORTED;
    }
    if (ps[i]->d.chamfer_mode != ps[0]->d.chamfer_mode || ps[i]->d.hp.alpha != ps[0]->d.hp.alpha) {
      set_error("batch members need one Chamfer mode and one alpha (member %d differs)", i);
      return PDG_EINVAL;
    }
    for (int j = 0; j < i; ++j)
      if (ps[j] == ps[i]) {
        set_error("problem %d appears twice in the batch", i);
        return PDG_EINVAL;
      }
  }
  return PDG_OK;
}

// Fork: every lane waits for what `main` has enqueued so far.
pdg_status batch_fork(pdg_batch &b, hipStream_t main, int k) {
  PDG_TRY_HIP(hipEventRecord(b.fork[k], main));
  for (int l = 0; l < kBatchLanes; ++l) PDG_TRY_HIP(hipStreamWaitEvent(b.lane[l], b.fork[k], 0));
  return PDG_OK;
}
// Join: `main` waits for every lane.
pdg_status batch_join(pdg_batch &b, hipStream_t main, int k) {
  for (int l = 0; l < kBatchLanes; ++l) {
    PDG_TRY_HIP(hipEventRecord(b.join[k][l], b.lane[l]));
    PDG_TRY_HIP(hipStreamWaitEvent(main, b.join[k][l], 0));
  }
  return PDG_OK;
}

// One iteration of every member (the members' epochs set beforehand).
pdg_status enqueue_batch(pdg_batch &b, hipStream_t main) {
  const int cnt = (int)b.members.size();
  PDG_TRY(batch_fork(b, main, 0));
  for (int i = 0; i < cnt; ++i)   // warps (Eq. 1, 8)
    PDG_TRY(enqueue_stage(*b.members[i], PDG_STAGE_WARP, b.lane[i % kBatchLanes], nullptr, true,
                          kSkipMerged));
  PDG_TRY(batch_join(b, main, 0));
  // every member's packs, nearest neighbours (Eq. 12) and Chamfer terms (Eq. 11, 13)
  if (uses_packs(b.mode)) {
    PDG_TRY(launch_screen_pack(b.ssets, b.nsets, b.max_n, main));
    if (b.mode == PDG_CHAMFER_BF16_SCREEN)
      PDG_TRY(launch_nn_screen(b.sjobs, b.njobs, b.max_nq, 1, main));
    else
      PDG_TRY(launch_nn_cull(b.sjobs, b.njobs, b.max_nq, 1, main));
  } else {
    PDG_TRY(launch_nn_exact(b.jobs, b.njobs, b.max_nq, main));
  }
  PDG_TRY(launch_chamfer_loss(b.segs, b.nseg, b.alpha, main));
  PDG_TRY(batch_fork(b, main, 1));
  for (int i = 0; i < cnt; ++i) {   // the rest of each member's iteration
    pdg_problem &p = *b.members[i];
    const hipStream_t st = b.lane[i % kBatchLanes];
    PDG_TRY(enqueue_stage(p, PDG_STAGE_LOSS, st, nullptr, true, kSkipMerged));
    for (int s = PDG_STAGE_GRAD; s <= PDG_STAGE_ADAM; ++s)
      PDG_TRY(enqueue_stage(p, s, st, nullptr, true, kSkipMerged));
    if (p.opt_x0) PDG_TRY(enqueue_stage(p, PDG_STAGE_TEMPLATE, st, nullptr, true, kSkipMerged));
  }
  return batch_join(b, main, 1);
}

void release_batch(pdg_batch *b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (int k = 0; k < 2; ++k) {
    if (b->fork[k]) (void)hipEventDestroy(b->fork[k]);
    for (int l = 0; l < kBatchLanes; ++l)
      if (b->join[k][l]) (void)hipEventDestroy(b->join[k][l]);
  }
  for (int l = 0; l < kBatchLanes; ++l)
    if (b->lane[l]) (void)hipStreamDestroy(b->lane[l]);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

// ----------------------------------------------- fixed device scratch --
// Workspace of pdg_chamfer_noalloc: one file-scope device array per GPU, held
// from module load until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol): the device address comes from hipGetSymbolAddress, taken once per
// device with that device current.
constexpr size_t kScratchBytes = 64ull << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices];

pdg_status scratch_of_current_device(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kScratchDevices) {
    set_error("device %d: the fixed scratch table holds devices 0..%d", dev, kScratchDevices - 1);
    return PDG_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr || ((uintptr_t)ptr & 255) != 0) {
      set_error("fixed scratch of device %d is not 256-byte aligned", dev);
      return PDG_EHIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return PDG_OK;
}

}  // namespace
}  // namespace pdg

extern "C" {

const char *pdg_last_error(void) { return g_err.c_str(); }

int32_t pdg_version(void) { return 100; }

int64_t pdg_grid_size(const pdg_grid_desc *d) {
  if (check_grid(d, true) != PDG_OK) return -1;
  return make_grid(*d).size;
}

pdg_status pdg_deform(const pdg_grid_desc *d, const float *grids, const float *x, int64_t n,
                      float *out, hipStream_t stream) {
  PDG_TRY(check_grid(d, true));
  if (n < 0 || n >= (1ll << 40)) {
    set_error("n = %lld invalid", (long long)n);
    return PDG_EINVAL;
  }
  if (n == 0) return PDG_OK;
  PDG_TRY(need(grids, "grids"));
  PDG_TRY(need(x, "x"));
  PDG_TRY(need(out, "out"));
  const GridDev g = make_grid(*d);
  if (g.ch == 6) return launch_warp6(g, grids, x, out, n, stream);
  return launch_warp(g, grids, 0, x, 0, n, out, 0, n, n, 1, stream);
}

pdg_status pdg_deform_backward_workspace(const pdg_grid_desc *d, int64_t n, size_t *bytes) {
  PDG_TRY(check_grid(d, true));
  if (!bytes || n < 0) {
    set_error("bytes is NULL or n < 0");
    return PDG_EINVAL;
  }
  Carve c(nullptr);
  deform_bwd_layout(c, make_grid(*d), n);
  *bytes = c.off;
  return PDG_OK;
}

pdg_status pdg_deform_backward(const pdg_grid_desc *d, const float *grids, const float *x,
                               int64_t n, const float *gout, float *ggrids, float *gx, void *ws,
                               size_t ws_bytes, hipStream_t stream) {
  PDG_TRY(check_grid(d, true));
  if (n < 0) {
    set_error("n < 0");
    return PDG_EINVAL;
  }
  const GridDev g = make_grid(*d);
  if ((long long)d->levels * n >= (1ll << 31) ||
      (unsigned long long)g.nodes >= (1ull << 32)) {
    set_error("problem too large for 32-bit scatter entries");
    return PDG_EINVAL;
  }
  if (ggrids) PDG_TRY(need(ggrids, "ggrids"));
  if (gx || (ggrids && g.ch == 6)) PDG_TRY(need(grids, "grids"));   // the rotation needs G
  if (n > 0) {
    PDG_TRY(need(x, "x"));
    PDG_TRY(need(gout, "gout"));
  }
  if (ggrids) {
    Carve probe(nullptr);
    deform_bwd_layout(probe, g, n);
    PDG_TRY(need_ws(ws, ws_bytes, probe.off));
    Carve c(ws);
    DeformBwdWs w = deform_bwd_layout(c, g, n);
    ScatterLists sl;
    memset(&sl, 0, sizeof sl);
    if (n > 0) {
      sl.count = 1;
      sl.list[0] = scatter_list(w.keys, w.vals, w.pstart, n, x, 0, n, gout, 0, n, w.ent, w.ent2);
      PDG_TRY(scatter_entries(g, 1, sl.list[0], w.keys, w.vals, w.pstart, w.sort, stream));
    }
    if (g.ch == 6) {
      // rotation channels from d<g, out>/dz^ (with gx, in the same pass),
      // then the translation channels from g itself, on the same entries
      PDG_TRY(launch_adjoint6(g, grids, x, gout, w.u, gx, n, stream));
      if (n > 0) {
        sl.list[0].lam = w.u;
        PDG_TRY(launch_scatter_stage(g, 1, sl.list[0], stream));
      }
      PDG_TRY(launch_gather(g, 1, sl, n, ggrids, w.gscratch, stream, 0));
      if (n > 0) {
        sl.list[0].lam = gout;
        PDG_TRY(launch_scatter_stage(g, 1, sl.list[0], stream, true));
      }
      return launch_gather(g, 1, sl, n, ggrids, w.gscratch, stream, 3);
    }
    if (n > 0) PDG_TRY(launch_scatter_stage(g, 1, sl.list[0], stream));
    PDG_TRY(launch_gather(g, 1, sl, n, ggrids, w.gscratch, stream));
  }
  if (gx && n > 0) {
    if (g.ch == 6) return launch_adjoint6(g, grids, x, gout, nullptr, gx, n, stream);
    PDG_TRY(launch_chain_adjoint(g, grids, x, n, gout, n, nullptr, 0, gx, n, n, stream));
  }
  return PDG_OK;
}

pdg_status pdg_mesh_precondition_workspace(int64_t V, int64_t E, size_t *bytes) {
  if (!bytes || V < 0 || E < 0 || V >= (1ll << 31) - 1 || E >= (1ll << 30)) {
    set_error("bytes NULL or V, E outside [0, 2^31 - 1), [0, 2^30)");
    return PDG_EINVAL;
  }
  *bytes = mesh_precond_bytes(V, E);
  return PDG_OK;
}

struct pdg_mesh_plan {
  MeshPlan *p = nullptr;
};

pdg_status pdg_mesh_plan_create(int64_t V, const int32_t *edges, int64_t E, float lambda,
                                int32_t max_degree, int32_t terms, double tol, void *ws,
                                size_t ws_bytes, hipStream_t stream, pdg_mesh_plan **plan) {
  size_t need_bytes = 0;
  PDG_TRY(pdg_mesh_precondition_workspace(V, E, &need_bytes));
  if (!plan || !(lambda >= 0.0f) || !isfinite(lambda) || max_degree < 0 || terms < 0 ||
      (terms == 0 && !(tol > 0.0 && tol < 1.0))) {
    set_error("plan NULL, or lambda not finite and >= 0, max_degree or terms < 0, tol not in (0, 1)");
    return PDG_EINVAL;
  }
  if (E > 0) PDG_TRY(need(edges, "edges"));
  PDG_TRY(need_ws(ws, ws_bytes, need_bytes));
  pdg_mesh_plan *h = new (std::nothrow) pdg_mesh_plan;
  if (!h) {
    set_error("host allocation failed");
    return PDG_ENOMEM;
  }
  pdg_status s = mesh_plan_build(V, (const int *)edges, E, lambda, max_degree, terms, tol, ws,
                                 stream, &h->p);
  if (s != PDG_OK) {
    delete h;
    return s;
  }
  *plan = h;
  return PDG_OK;
}

pdg_status pdg_mesh_plan_apply(const pdg_mesh_plan *plan, const float *g, float *out,
                               hipStream_t stream) {
  if (!plan) {
    set_error("plan is NULL");
    return PDG_EINVAL;
  }
  if (mesh_plan_vertices(*plan->p) > 0) {
    PDG_TRY(need(g, "g"));
    PDG_TRY(need(out, "out"));
  }
  return mesh_plan_apply(*plan->p, g, out, stream);
}

pdg_status pdg_mesh_plan_info(const pdg_mesh_plan *plan, int32_t *terms, int32_t *parts) {
  if (!plan) {
    set_error("plan is NULL");
    return PDG_EINVAL;
  }
  if (terms) *terms = mesh_plan_terms(*plan->p);
  if (parts) *parts = mesh_plan_parts(*plan->p);
  return PDG_OK;
}

pdg_status pdg_mesh_partition(int64_t V, const int32_t *edges, int64_t E, int32_t *part_off,
                              int32_t *part_core, int32_t *local_vertex, int32_t *local_dist,
                              int64_t *sizes) {
  if (!sizes || V < 0 || E < 0 || V >= (1ll << 31) - 1 || E >= (1ll << 30) || (E > 0 && !edges)) {
    set_error("sizes NULL, edges NULL with E > 0, or V, E outside [0, 2^31 - 1), [0, 2^30)");
    return PDG_EINVAL;
  }
  return mesh_partition_query(V, (const int *)edges, E, (int *)part_off, (int *)part_core,
                              (int *)local_vertex, (int *)local_dist, (long long *)sizes);
}

pdg_status pdg_mesh_plan_destroy(pdg_mesh_plan *plan) {
  if (plan) {
    mesh_plan_free(plan->p);
    delete plan;
  }
  return PDG_OK;
}

pdg_status pdg_mesh_precondition(int64_t V, const int32_t *edges, int64_t E, float lambda,
                                 int32_t max_degree, int32_t terms, double tol, const float *g,
                                 float *out, void *ws, size_t ws_bytes, hipStream_t stream) {
  pdg_mesh_plan *plan = nullptr;
  PDG_TRY(pdg_mesh_plan_create(V, edges, E, lambda, max_degree, terms, tol, ws, ws_bytes, stream,
                               &plan));
  const pdg_status s = pdg_mesh_plan_apply(plan, g, out, stream);
  pdg_mesh_plan_destroy(plan);
  return s;
}

pdg_status pdg_keyframe_workspace(int32_t frames, size_t *bytes) {
  if (!bytes || frames < 1 || frames > 65535) {
    set_error("bytes NULL or frames outside 1..65535");
    return PDG_EINVAL;
  }
  *bytes = keyframe_bytes(frames);
  return PDG_OK;
}

pdg_status pdg_keyframe(const float *points, int32_t frames, int64_t n, double gamma,
                        int64_t *counts, int32_t *key, void *ws, size_t ws_bytes,
                        hipStream_t stream) {
  size_t need_bytes = 0;
  PDG_TRY(pdg_keyframe_workspace(frames, &need_bytes));
  if (n < 0 || n >= (1ll << 40) || !(gamma >= 0.0) || !isfinite(gamma)) {
    set_error("n < 0 or gamma not finite and >= 0");
    return PDG_EINVAL;
  }
  if (n > 0) PDG_TRY(need(points, "points"));
  PDG_TRY(need(key, "key"));
  if (counts) PDG_TRY(need(counts, "counts"));
  PDG_TRY(need_ws(ws, ws_bytes, need_bytes));
  return launch_keyframe(points, frames, n, gamma, (long long *)counts, key, ws, stream);
}

pdg_status pdg_chamfer_workspace(int64_t n, int64_t m, int32_t mode, size_t *bytes) {
  if (!bytes || n < 1 || m < 1 || n >= (1ll << 31) || m >= (1ll << 31)) {
    set_error("bytes NULL or n, m outside [1, 2^31)");
    return PDG_EINVAL;
  }
  if (mode != PDG_CHAMFER_FP32 && !uses_packs(mode)) {
    set_error("unknown chamfer mode %d", mode);
    return PDG_EINVAL;
  }
  Carve c(nullptr);
  chamfer_layout(c, n, m, mode);
  *bytes = c.off;
  return PDG_OK;
}

pdg_status pdg_chamfer(const float *a, int64_t n, const float *b, int64_t m, double alpha,
                       int32_t mode, const double *dir_weight, double *loss, int32_t *nn_a,
                       int32_t *nn_b, float *ga, void *ws, size_t ws_bytes, hipStream_t stream) {
  size_t need_bytes = 0;
  PDG_TRY(pdg_chamfer_workspace(n, m, mode, &need_bytes));
  if (!(alpha >= 0.0) || !isfinite(alpha)) {
    set_error("alpha must be finite and >= 0");
    return PDG_EINVAL;
  }
  PDG_TRY(need(a, "a"));
  PDG_TRY(need(b, "b"));
  PDG_TRY(need(loss, "loss"));
  PDG_TRY(need(nn_a, "nn_a"));
  PDG_TRY(need(nn_b, "nn_b"));
  if (ga) PDG_TRY(need(ga, "ga"));
  PDG_TRY(need_ws(ws, ws_bytes, need_bytes));
  Carve c(ws);
  ChamferWs w = chamfer_layout(c, n, m, mode);
  return enqueue_chamfer(w, a, n, b, m, alpha, mode, dir_weight, loss, nn_a, nn_b, ga, stream);
}

pdg_status pdg_chamfer_noalloc(const float *a, int64_t n, const float *b, int64_t m,
                               double alpha, int32_t mode, const double *dir_weight, double *loss,
                               int32_t *nn_a, int32_t *nn_b, float *ga, hipStream_t stream) {
  size_t need_bytes = 0;
  PDG_TRY(pdg_chamfer_workspace(n, m, mode, &need_bytes));
  if (need_bytes > kScratchBytes) {
    set_error("pdg_chamfer_noalloc: n = %lld, m = %lld need %zu workspace bytes, above the fixed "
              "scratch of %zu bytes (use pdg_chamfer with a caller workspace)",
              (long long)n, (long long)m, need_bytes, kScratchBytes);
    return PDG_ENOMEM;
  }
  void *ws = nullptr;
  PDG_TRY(scratch_of_current_device(&ws));
  return pdg_chamfer(a, n, b, m, alpha, mode, dir_weight, loss, nn_a, nn_b, ga, ws, need_bytes,
                     stream);
}

pdg_status pdg_chamfer_backward(const float *a, int64_t n, const float *b, int64_t m,
                                double alpha, const int32_t *nn_a, const int32_t *nn_b,
                                const double *dir_weight, float *ga, void *ws, size_t ws_bytes,
                                hipStream_t stream) {
  size_t need_bytes = 0;
  PDG_TRY(pdg_chamfer_workspace(n, m, PDG_CHAMFER_FP32, &need_bytes));
  if (!(alpha >= 0.0) || !isfinite(alpha)) {
    set_error("alpha must be finite and >= 0");
    return PDG_EINVAL;
  }
  PDG_TRY(need(a, "a"));
  PDG_TRY(need(b, "b"));
  PDG_TRY(need(nn_a, "nn_a"));
  PDG_TRY(need(nn_b, "nn_b"));
  PDG_TRY(need(dir_weight, "dir_weight"));
  PDG_TRY(need(ga, "ga"));
  PDG_TRY(need_ws(ws, ws_bytes, need_bytes));
  Carve c(ws);
  ChamferWs w = chamfer_layout(c, n, m, PDG_CHAMFER_FP32);
  ChSeg seg;
  memset(&seg, 0, sizeof seg);
  seg.a = a;
  seg.b = b;
  seg.n = (int)n;
  seg.m = (int)m;
  seg.nn_a = const_cast<int32_t *>(nn_a);   // read only on this path
  seg.nn_b = const_cast<int32_t *>(nn_b);
  seg.ga = ga;
  seg.w = dir_weight;
  const unsigned bb = 0;
  PDG_TRY(upload_small(w.segs, &seg, sizeof seg, stream));
  PDG_TRY(upload_small(w.b_base, &bb, sizeof bb, stream));
  PDG_TRY(launch_chamfer_grad_fwd(w.segs, 1, (int)n, (float)alpha, stream));
  PDG_TRY(launch_chamfer_rev_keys(w.segs, 1, (int)m, w.b_base, w.keys, w.vals, stream));
  PDG_TRY(radix_sort(w.keys, w.vals, m, bits_for((unsigned long long)n), w.sort, stream));
  return launch_chamfer_rev_scatter(w.segs, 1, w.b_base, w.keys, w.vals, m, (float)alpha,
                                    w.rpart, stream);
}

pdg_status pdg_precondition_workspace(const pdg_grid_desc *d, int32_t batch, int32_t method,
                                      size_t *bytes) {
  PDG_TRY(check_grid(d, true));
  if (!bytes || batch < 0) {
    set_error("bytes NULL or batch < 0");
    return PDG_EINVAL;
  }
  if (method != PDG_PRECOND_CG && method != PDG_PRECOND_DCT) {
    set_error("unknown preconditioner method %d", method);
    return PDG_EINVAL;
  }
  const GridDev g = make_grid(*d);
  if (method == PDG_PRECOND_DCT) {
    *bytes = dct_bytes(g);
    return PDG_OK;
  }
  float lam[PDG_MAX_LEVELS];
  for (int l = 0; l < d->levels; ++l) lam[l] = 1.0f;
  CGPlanDev p = cg_plan(g.ch == 6 ? half_view(g, 0) : g, batch, lam, 1, 0.5, false);
  *bytes = cg_ws_bytes(p, g.size * batch);
  return PDG_OK;
}

pdg_status pdg_precondition(const pdg_grid_desc *d, const float *lambda, float *g, int32_t batch,
                            int32_t method, int32_t iters, double tol, void *ws, size_t ws_bytes,
                            hipStream_t stream) {
  PDG_TRY(check_grid(d, true));
  pdg_grid_desc d3 = *d;   // six channels: the rotation and translation halves as grids
  d3.channels = 3;
  PDG_TRY(check_precond_args(&d3, lambda, batch, method, iters, tol));
  if (batch == 0) return PDG_OK;
  PDG_TRY(need(g, "g"));
  size_t nb = 0;
  PDG_TRY(pdg_precondition_workspace(d, batch, method, &nb));
  PDG_TRY(need_ws(ws, ws_bytes, nb));
  const GridDev gd = make_grid(*d);
  const int halves = gd.ch == 6 ? 2 : 1;
  if (method == PDG_PRECOND_DCT) {
    PDG_TRY(dct_basis(gd, ws, stream));
    for (int h = 0; h < halves; ++h)
      PDG_TRY(run_dct(halves == 2 ? half_view(gd, h) : gd, batch, lambda, g, g, ws, stream));
    return PDG_OK;
  }
  const bool aligned16 = ((uintptr_t)g & 15) == 0;
  for (int h = 0; h < halves; ++h) {
    CGPlanDev p = cg_plan(halves == 2 ? half_view(gd, h) : gd, batch, lambda, iters, tol, aligned16);
    PDG_TRY(run_cg(p, g, gd.size * batch, ws, stream));
  }
  return PDG_OK;
}

pdg_status pdg_prune_mask_words(const pdg_grid_desc *d, int64_t *words) {
  PDG_TRY(check_grid(d, true));   // masks cover cells: the channel count does not matter
  PDG_TRY(need(words, "words"));
  *words = mask_stack_words(make_grid(*d));
  return PDG_OK;
}

pdg_status pdg_prune_workspace(const pdg_grid_desc *d, int32_t stacks, size_t *bytes) {
  PDG_TRY(check_grid(d, true));
  if (!bytes || stacks < 0) {
    set_error("bytes NULL or stacks < 0");
    return PDG_EINVAL;
  }
  *bytes = prune_bytes(make_grid(*d), stacks);
  return PDG_OK;
}

pdg_status pdg_prune_mask(const pdg_grid_desc *d, int32_t stacks, int32_t span, const float *points,
                          int64_t n, int32_t halo, uint32_t *mask, int64_t *active, void *ws,
                          size_t ws_bytes, hipStream_t stream) {
  PDG_TRY(check_grid(d, true));
  if (stacks < 0 || span < 1 || n < 0 || n >= (1ll << 31) || halo < 0 || halo > 16) {
    set_error("prune: stacks >= 0, span >= 1, 0 <= n < 2^31 and 0 <= halo <= 16 required");
    return PDG_EINVAL;
  }
  const long long frames = (long long)stacks + span - 1;
  if (frames > 65535) {
    set_error("prune: %lld frames exceed the grid's 65535", frames);
    return PDG_EINVAL;
  }
  if (stacks == 0) return PDG_OK;
  PDG_TRY(need(mask, "mask"));
  if (n > 0) PDG_TRY(need(points, "points"));
  const GridDev g = make_grid(*d);
  PDG_TRY(need_ws(ws, ws_bytes, prune_bytes(g, stacks)));
  return launch_prune_mask(g, stacks, span, points, n, halo, mask, (long long *)active, ws,
                           stream);
}

pdg_status pdg_precondition_pruned(const pdg_grid_desc *d, const float *lambda, float *g,
                                   int32_t batch, int32_t iters, double tol, const uint32_t *mask,
                                   void *ws, size_t ws_bytes, hipStream_t stream) {
  PDG_TRY(check_precond_args(d, lambda, batch, PDG_PRECOND_CG, iters, tol));
  if (batch == 0) return PDG_OK;
  PDG_TRY(need(g, "g"));
  PDG_TRY(need(mask, "mask"));
  size_t nb = 0;
  PDG_TRY(pdg_precondition_workspace(d, batch, PDG_PRECOND_CG, &nb));
  PDG_TRY(need_ws(ws, ws_bytes, nb));
  const GridDev gd = make_grid(*d);
  const bool aligned16 = ((uintptr_t)g & 15) == 0;
  CGPlanDev p = cg_plan(gd, batch, lambda, iters, tol, aligned16);
  cg_set_mask(p, gd, mask);
  return run_cg(p, g, gd.size * batch, ws, stream);
}

pdg_status pdg_adam(const pdg_grid_desc *d, int32_t batch, const float *lr, float beta1,
                    float beta2, float eps, int32_t step, float *theta, float *m, float *v,
                    const float *g, hipStream_t stream) {
  PDG_TRY(check_grid(d, true));   // any channel count: per-level rates over the packed values
  if (!lr || batch < 0 || step < 1 || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f)) {
    set_error("invalid Adam arguments");
    return PDG_EINVAL;
  }
  if (batch == 0) return PDG_OK;
  PDG_TRY(need(theta, "theta"));
  PDG_TRY(need(m, "m"));
  PDG_TRY(need(v, "v"));
  PDG_TRY(need(g, "g"));
  const GridDev gd = make_grid(*d);
  AdamLevels lv;
  lv.levels = gd.levels;
  for (int l = 0; l < gd.levels; ++l) {
    lv.off[l] = gd.off[l];
    lv.lr[l] = lr[l];
  }
  lv.off[gd.levels] = gd.size;
  return launch_adam(lv, gd.size, batch, beta1, beta2, eps, nullptr, step, theta, m, v, g, stream);
}

namespace pdg {
namespace {

// One chain of a sequence propagated both ways from keyframe k: the backward
// chain (c = 0) reads frames k, k-1, .., 0 from `rev` and owns the first k
// grid stacks; the forward chain (c = 1) reads frames k .. F-1 in place and
// owns the rest.  X_0 is optimised with the forward chain (with the backward
// one when k = F - 1).
pdg_problem_desc chain_desc(const pdg_problem_desc &pd, int c, const float *rev) {
  pdg_problem_desc d = pd;
  d.keyframe = 0;
  d.workspace = nullptr;
  d.workspace_bytes = 0;
  const long long k = pd.keyframe, N = pd.n;
  const GridDev g = make_grid(pd.grid);
  if (c == 0) {
    d.frames = (int32_t)(k + 1);
    d.points = rev;
    if (pd.frames - 1 - k > 0) d.template_adam_m = d.template_adam_v = nullptr;
  } else {
    d.frames = (int32_t)(pd.frames - k);
    d.points = pd.points + k * 3 * N;
    d.params = pd.params + k * g.size;
    d.adam_m = pd.adam_m + k * g.size;
    d.adam_v = pd.adam_v + k * g.size;
    if (pd.prune_mask) d.prune_mask = pd.prune_mask + k * mask_stack_words(g);
  }
  return d;
}

bool chain_exists(const pdg_problem_desc &pd, int c) {
  return c == 0 ? pd.keyframe >= 1 : pd.keyframe <= pd.frames - 2;
}

}  // namespace
}  // namespace pdg

static pdg_status chain_workspace(const pdg_problem_desc *pd, size_t *bytes);
static pdg_status create_chain(const pdg_problem_desc *pd, hipStream_t stream, pdg_problem **out);

static pdg_status joint_layout(const pdg_problem_desc *pd, Carve &c, float **rev, double **jterms,
                               size_t chain_bytes[2]) {
  const long long k = pd->keyframe, N = pd->n;
  *rev = c.take<float>((k + 1) * 3 * N);
  *jterms = c.take<double>(kTerms);
  for (int i = 0; i < 2; ++i) {
    chain_bytes[i] = 0;
    if (!chain_exists(*pd, i)) continue;
    const pdg_problem_desc d = chain_desc(*pd, i, *rev ? *rev : (const float *)pd->points);
    PDG_TRY(chain_workspace(&d, &chain_bytes[i]));
    c.take<char>((long long)chain_bytes[i]);
  }
  return PDG_OK;
}

pdg_status pdg_problem_workspace(const pdg_problem_desc *pd, size_t *bytes) {
  PDG_TRY(check_problem(pd));
  if (!bytes) {
    set_error("bytes is NULL");
    return PDG_EINVAL;
  }
  if (pd->keyframe > 0) {
    Carve c(nullptr);
    float *rev = nullptr;
    double *jt = nullptr;
    size_t cb[2];
    PDG_TRY(joint_layout(pd, c, &rev, &jt, cb));
    *bytes = c.off;
    return PDG_OK;
  }
  return chain_workspace(pd, bytes);
}

static pdg_status chain_workspace(const pdg_problem_desc *pd, size_t *bytes) {
  pdg_problem p;
  init_problem(p, *pd);
  Carve c(nullptr);
  layout(p, c);
  *bytes = c.off;
  return PDG_OK;
}

pdg_status pdg_problem_create(const pdg_problem_desc *pd, hipStream_t stream, pdg_problem **out) {
  PDG_TRY(check_problem(pd));
  if (!out) {
    set_error("out is NULL");
    return PDG_EINVAL;
  }
  if (pd->keyframe == 0) return create_chain(pd, stream, out);
  // reverse-time propagation: two chains leave the keyframe
  size_t need_bytes = 0;
  PDG_TRY(pdg_problem_workspace(pd, &need_bytes));
  PDG_TRY(need_ws(pd->workspace, pd->workspace_bytes, need_bytes));
  pdg_problem *J = new (std::nothrow) pdg_problem;
  if (!J) {
    set_error("host allocation failed");
    return PDG_ENOMEM;
  }
  J->joint = true;
  J->d = *pd;
  J->F = pd->frames;
  J->T = pd->frames - 1;
  J->N = pd->n;
  J->V = pd->verts;
  J->has_tm = pd->verts > 0;
  J->opt_x0 = J->has_tm && pd->template_adam_m && pd->template_adam_v;
  Carve c(pd->workspace);
  const long long k = pd->keyframe, N = pd->n;
  J->rev_points = c.take<float>((k + 1) * 3 * N);
  J->jterms = c.take<double>(kTerms);
  pdg_status s = PDG_OK;
  for (long long b = 0; b <= k && s == PDG_OK; ++b)   // frames k, k-1, .., 0
    s = launch_copy(J->rev_points + b * 3 * N, pd->points + (k - b) * 3 * N, 3 * N, stream);
  for (int i = 0; i < 2 && s == PDG_OK; ++i) {
    if (!chain_exists(*pd, i)) continue;
    pdg_problem_desc d = chain_desc(*pd, i, J->rev_points);
    size_t cb = 0;
    s = chain_workspace(&d, &cb);
    if (s != PDG_OK) break;
    d.workspace = c.take<char>((long long)cb);
    d.workspace_bytes = cb;
    s = create_chain(&d, stream, &J->child[i]);
    if (s == PDG_OK) J->child[i]->Tn = J->T;
  }
  if (s != PDG_OK) {
    (void)pdg_problem_destroy(J);
    return s;
  }
  if (J->child[0] && J->child[1]) {
    J->child[0]->partner_losses = J->child[1]->losses;
    J->child[0]->partner_T = J->child[1]->T;
    J->child[1]->partner_losses = J->child[0]->losses;
    J->child[1]->partner_T = J->child[0]->T;
  }
  J->ws_used = c.off;
  *out = J;
  return PDG_OK;
}

static pdg_status create_chain(const pdg_problem_desc *pd, hipStream_t stream, pdg_problem **out) {
  pdg_problem *p = new (std::nothrow) pdg_problem;
  if (!p) {
    set_error("host allocation failed");
    return PDG_ENOMEM;
  }
  init_problem(*p, *pd);
  Carve probe(nullptr);
  layout(*p, probe);
  {
    pdg_status s = need_ws(pd->workspace, pd->workspace_bytes, probe.off);
    if (s != PDG_OK) {
      delete p;
      return s;
    }
  }
  Carve c(pd->workspace);
  layout(*p, c);
  p->ws_used = c.off;
  const long long T = p->T, N = p->N, V = p->V;
  // Chamfer pairs: point term P^_t <-> P_t, template term X_t <-> P_t
  std::vector<ChSeg> segs(p->nseg);
  std::vector<NNJob> jobs(p->njobs);
  std::vector<unsigned> bb(p->nseg);
  unsigned bsum = 0;
  for (int s = 0; s < p->nseg; ++s) {
    const bool tm = s >= T;
    const long long t = tm ? s - T : s;
    ChSeg &q = segs[s];
    memset(&q, 0, sizeof q);
    q.b = pd->points + (t + 1) * 3 * N;
    q.m = (int)N;
    q.loss = p->losses + 2 * s;
    q.part = p->partials + 2 * (long long)s * kLossBlocks;
    q.w = p->w + 2 * s;
    if (!tm) {
      q.a = p->phat + t * 3 * N;
      q.n = (int)N;
      q.nn_a = p->nn + t * 2 * N;
      q.nn_b = q.nn_a + N;
      q.ga = p->gphat + t * 3 * N;
      q.a_base = (unsigned)(t * N);
    } else {
      q.a = p->xhat + (t + 1) * 3 * V;
      q.n = (int)V;
      q.nn_a = p->nn + T * 2 * N + t * (V + N);
      q.nn_b = q.nn_a + V;
      q.ga = p->gxhat + t * 3 * V;
      q.a_base = (unsigned)(T * N + t * V);
    }
    bb[s] = bsum;
    bsum += (unsigned)q.m;
    NNJob &j0 = jobs[2 * s];
    NNJob &j1 = jobs[2 * s + 1];
    memset(&j0, 0, sizeof j0);
    memset(&j1, 0, sizeof j1);
    j0.q = q.a;
    j0.c = q.b;
    j0.nq = q.n;
    j0.nc = q.m;
    j0.nn = q.nn_a;
    j1.q = q.b;
    j1.c = q.a;
    j1.nq = q.m;
    j1.nc = q.n;
    j1.nn = q.nn_b;
    if (q.n > p->max_nq) p->max_nq = q.n;
    if (q.m > p->max_nq) p->max_nq = q.m;
    if (q.n > p->max_n) p->max_n = q.n;
    if (q.m > p->max_m) p->max_m = q.m;
  }
  std::vector<ScreenSet> ssets;
  std::vector<ScreenJob> sjobs;
  if (p->coords) {
    long long row = 0, tile = 0;
    auto add_set = [&](const float *x, long long n, const int *perm) {
      ssets.push_back(screen_set(x, n, perm, p->packs ? p->packs + 2 * row : nullptr, p->coords + row,
                                 p->boxes + tile, p->pinv + row));
      row += n;
      tile += screen_box_count(n);
    };
    for (int s = 0; s < p->nseg; ++s) {        // moving sets: P^_t keeps P_t's order, X_t X_0's
      const ChSeg &q = segs[s];
      add_set(q.a, q.n, s < T ? p->fperm + (long long)s * N : p->tperm);
    }
    for (long long t = 0; t < T; ++t)          // fixed frames P_1..P_T
      add_set(pd->points + (t + 1) * 3 * N, N, p->fperm + (t + 1) * N);
    for (int s = 0; s < p->nseg; ++s) {
      const ChSeg &q = segs[s];
      const ScreenSet &A = ssets[s], &B = ssets[p->nseg + s % T];
      sjobs.push_back(screen_job(A, B, q.nn_a, p->tiles));
      sjobs.push_back(screen_job(B, A, q.nn_b, p->tiles));
    }
  }
  hipError_t e = hipSuccess;
  if (p->E > 0) {
    // edge indices index the template on the GPU: check their range once
    std::vector<int32_t> eh(2 * p->E);
    e = hipMemcpy(eh.data(), pd->edges, eh.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      pdg_status s = hip_fail(e, "pdg_problem_create edge check");
      delete p;
      return s;
    }
    for (size_t i = 0; i < eh.size(); ++i)
      if (eh[i] < 0 || eh[i] >= V) {
        set_error("edge index %d at position %zu outside [0, %lld)", eh[i], i, V);
        delete p;
        return PDG_EINVAL;
      }
    if (p->opt_x0) {  // the Gershgorin bound of the mesh preconditioner needs d_max
      std::vector<int> deg(V, 0);
      for (size_t i = 0; i < eh.size(); ++i) ++deg[eh[i]];
      for (long long v = 0; v < V; ++v) p->max_degree = deg[v] > p->max_degree ? deg[v] : p->max_degree;
    }
  }
  if (e == hipSuccess) e = hipMemcpy(p->segs, segs.data(), segs.size() * sizeof(ChSeg), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->jobs, jobs.data(), jobs.size() * sizeof(NNJob), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->b_base, bb.data(), bb.size() * sizeof(unsigned), hipMemcpyHostToDevice);
  if (e == hipSuccess && p->coords)
    e = hipMemcpy(p->ssets, ssets.data(), ssets.size() * sizeof(ScreenSet), hipMemcpyHostToDevice);
  if (e == hipSuccess && p->coords)
    e = hipMemcpy(p->sjobs, sjobs.data(), sjobs.size() * sizeof(ScreenJob), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    pdg_status s = hip_fail(e, "pdg_problem_create table upload");
    delete p;
    return s;
  }
  pdg_status s = PDG_OK;
  // Morton order of every frame and of the template (processing order of the
  // warps and the screen packs' row order)
  for (long long f = 0; f < p->F && s == PDG_OK; ++f) {
    uint32_t *perm = (uint32_t *)(p->fperm + f * N);
    s = launch_morton(pd->points + f * 3 * N, N, (int)N, p->rkeys, perm, stream);
    if (s == PDG_OK) s = radix_sort(p->rkeys, perm, N, 30, p->sort, stream);
  }
  if (s == PDG_OK && p->has_tm) {
    s = launch_morton(pd->template_verts, V, (int)V, p->tkeys, (uint32_t *)p->tperm, stream);
    if (s == PDG_OK) s = radix_sort(p->tkeys, (uint32_t *)p->tperm, V, 30, p->sort, stream);
  }
  if (p->coords) {
    // the fixed frames' packs (their rows, coordinates and boxes never change)
    if (s == PDG_OK) s = launch_screen_pack(p->ssets + p->nseg, (int)T, (int)N, stream);
    if (s == PDG_OK) s = launch_fill((float *)p->tiles, 2, 0.f, stream);
  }
  // static scatter entries of the input points (fixed positions): keys, row
  // table and the stencil fractions (the steps re-stage only the adjoints)
  if (s == PDG_OK) {
    const ScatterList pl = scatter_list(p->pkeys, p->pvals, p->pstart_p, N, pd->points, 3 * N, N,
                                        p->gphat, 3 * N, N, p->ent_p, p->ent2_p);
    s = scatter_entries(p->g, (int)T, pl, p->pkeys, p->pvals, p->pstart_p, p->sort, stream);
    if (s == PDG_OK) s = launch_scatter_stage(p->g, (int)T, pl, stream);
  }
  if (s == PDG_OK && p->has_tm)
    s = launch_incidence(pd->edges, (int)p->E, (int)V, p->ikeys, p->ivals, p->inc_off, p->sort,
                         stream);
  if (s == PDG_OK && p->dctws) s = dct_basis(p->g, p->dctws, stream);
  // X_0 optimised: the plan of its preconditioner (fixed edges)
  if (s == PDG_OK && p->opt_x0)
    s = mesh_plan_build(V, pd->edges, p->E, pd->hp.mesh_lambda, p->max_degree, 0, kMeshTol,
                        p->meshws, stream, &p->mesh);
  // pruned grids: pruned cells hold zero and keep zero moments
  if (pd->prune_mask)
    for (float *buf : {pd->params, pd->adam_m, pd->adam_v})
      if (s == PDG_OK) s = launch_mask_apply(p->g, (int)T, pd->prune_mask, buf, stream);
  // pruned grids: the conjugate-gradient launches cover the kept tiles only
  // (their list is built on the host from the masks, once)
  if (s == PDG_OK && pd->prune_mask && p->cg.ntiles > 0) {
    const long long words = (long long)T * mask_stack_words(p->g);
    std::vector<uint32_t> hm(words);
    std::vector<int> kl(p->cg.ntiles);
    hipError_t he = hipStreamSynchronize(stream);
    if (he == hipSuccess)
      he = hipMemcpy(hm.data(), pd->prune_mask, words * sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (he == hipSuccess) {
      const int nk = cg_kept_tiles(p->cg, p->g, hm.data(), kl.data());
      if (nk > 0) he = hipMemcpy(p->klist, kl.data(), nk * sizeof(int), hipMemcpyHostToDevice);
      p->cg.klist = p->klist;
      if (p->g.ch == 6) {   // the other half's plan numbers its tiles the same way
        p->cg_t.klist = p->klist;
        for (int l = 0; l < p->g.levels; ++l) {
          p->cg_t.kfirst[l] = p->cg.kfirst[l];
          p->cg_t.kcount[l] = p->cg.kcount[l];
        }
      }
    }
    if (he != hipSuccess) s = hip_fail(he, "pdg_problem_create kept tiles");
  }
  if (s == PDG_OK) s = launch_set_int(p->epoch, 0, stream);
  if (s != PDG_OK) {
    delete p;
    return s;
  }
  *out = p;
  return PDG_OK;
}

pdg_status pdg_step(pdg_problem *p, int32_t epoch, double *loss_terms, int32_t use_graph,
                    hipStream_t stream) {
  if (!p) {
    set_error("problem is NULL");
    return PDG_EINVAL;
  }
  if (epoch < 0 || epoch > p->d.hp.e_max) {
    set_error("epoch %d outside [0, e_max = %d]", epoch, p->d.hp.e_max);
    return PDG_EINVAL;
  }
  if (p->joint) {
    for (int c = 0; c < 2; ++c)
      if (p->child[c]) PDG_TRY(launch_set_int(p->child[c]->epoch, epoch, stream));
  } else {
    PDG_TRY(launch_set_int(p->epoch, epoch, stream));
  }
  if (!use_graph) return enqueue_step(*p, stream, loss_terms);
  if (loss_terms) {
    set_error("loss_terms must be NULL with use_graph (read PDG_BUF terms instead)");
    return PDG_EINVAL;
  }
  if (!p->exec) {
    if (!p->cap) PDG_TRY_HIP(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
    PDG_TRY_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    pdg_status s = enqueue_step(*p, p->cap, nullptr);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap, &graph);
    if (s != PDG_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    p->graph = graph;
    PDG_TRY_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
  }
  PDG_TRY_HIP(hipGraphLaunch(p->exec, stream));
  return PDG_OK;
}

pdg_status pdg_step_stage(pdg_problem *p, int32_t stage, hipStream_t stream) {
  if (!p) {
    set_error("problem is NULL");
    return PDG_EINVAL;
  }
  if (stage < PDG_STAGE_WARP || stage > PDG_STAGE_TEMPLATE) {
    set_error("unknown stage %d", stage);
    return PDG_EINVAL;
  }
  if (p->joint) return enqueue_joint_stage(*p, stage, stream, nullptr, false);
  if (stage == PDG_STAGE_PRECOND_ADAM) return enqueue_precond_adam(*p, stream);
  return enqueue_stage(*p, stage, stream, nullptr, false);
}

pdg_status pdg_batch_workspace(pdg_problem *const *ps, int32_t count, size_t *bytes) {
  PDG_TRY(check_batch(ps, count));
  PDG_TRY(need(bytes, "bytes"));
  int nsets = 0, njobs = 0, nseg = 0;
  for (int i = 0; i < count; ++i) {
    nsets += ps[i]->nseg;
    njobs += ps[i]->njobs;
    nseg += ps[i]->nseg;
  }
  Carve c(nullptr);
  batch_layout(c, ps[0]->d.chamfer_mode, nsets, njobs, nseg);
  *bytes = c.off;
  return PDG_OK;
}

pdg_status pdg_batch_create(pdg_problem *const *ps, int32_t count, void *ws, size_t ws_bytes,
                            hipStream_t stream, pdg_batch **out) {
  size_t need_bytes = 0;
  PDG_TRY(pdg_batch_workspace(ps, count, &need_bytes));
  PDG_TRY(need(out, "out"));
  PDG_TRY(need_ws(ws, ws_bytes, need_bytes));
  pdg_batch *b = new (std::nothrow) pdg_batch;
  if (!b) {
    set_error("host allocation failed");
    return PDG_ENOMEM;
  }
  b->members.assign(ps, ps + count);
  b->mode = ps[0]->d.chamfer_mode;
  b->alpha = ps[0]->d.hp.alpha;
  for (int i = 0; i < count; ++i) {
    b->nsets += ps[i]->nseg;
    b->njobs += ps[i]->njobs;
    b->nseg += ps[i]->nseg;
    b->max_n = ps[i]->max_n > b->max_n ? ps[i]->max_n : b->max_n;
    b->max_nq = ps[i]->max_nq > b->max_nq ? ps[i]->max_nq : b->max_nq;
  }
  Carve c(ws);
  const BatchTables t = batch_layout(c, b->mode, b->nsets, b->njobs, b->nseg);
  b->ssets = t.ssets;
  b->sjobs = t.sjobs;
  b->jobs = t.jobs;
  b->segs = t.segs;
  // the members' tables, one after another (device to device, on `stream`)
  hipError_t e = hipSuccess;
  int os = 0, oj = 0;
  for (int i = 0; i < count && e == hipSuccess; ++i) {
    const pdg_problem &p = *ps[i];
    if (uses_packs(b->mode)) {
      e = hipMemcpyAsync(b->ssets + os, p.ssets, p.nseg * sizeof(ScreenSet),
                         hipMemcpyDeviceToDevice, stream);   // the moving sets come first
      if (e == hipSuccess)
        e = hipMemcpyAsync(b->sjobs + oj, p.sjobs, p.njobs * sizeof(ScreenJob),
                           hipMemcpyDeviceToDevice, stream);
    } else {
      e = hipMemcpyAsync(b->jobs + oj, p.jobs, p.njobs * sizeof(NNJob), hipMemcpyDeviceToDevice,
                         stream);
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->segs + os, p.segs, p.nseg * sizeof(ChSeg), hipMemcpyDeviceToDevice,
                         stream);
    os += p.nseg;
    oj += p.njobs;
  }
  for (int l = 0; l < kBatchLanes && e == hipSuccess; ++l)
    e = hipStreamCreateWithFlags(&b->lane[l], hipStreamNonBlocking);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = hipEventCreateWithFlags(&b->fork[k], hipEventDisableTiming);
    for (int l = 0; l < kBatchLanes && e == hipSuccess; ++l)
      e = hipEventCreateWithFlags(&b->join[k][l], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    release_batch(b);
    return hip_fail(e, "pdg_batch_create");
  }
  *out = b;
  return PDG_OK;
}

pdg_status pdg_batch_step(pdg_batch *b, const int32_t *epochs, int32_t use_graph,
                          hipStream_t stream) {
  if (!b || !epochs) {
    set_error("batch or epochs is NULL");
    return PDG_EINVAL;
  }
  const int cnt = (int)b->members.size();
  for (int i = 0; i < cnt; ++i)
    if (epochs[i] < 0 || epochs[i] > b->members[i]->d.hp.e_max) {
      set_error("epoch %d of member %d outside [0, e_max = %d]", epochs[i], i,
                b->members[i]->d.hp.e_max);
      return PDG_EINVAL;
    }
  for (int i = 0; i < cnt; ++i) PDG_TRY(launch_set_int(b->members[i]->epoch, epochs[i], stream));
  if (!use_graph) return enqueue_batch(*b, stream);
  if (!b->exec) {
    if (!b->cap) PDG_TRY_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    PDG_TRY_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    pdg_status s = enqueue_batch(*b, b->cap);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap, &graph);
    if (s != PDG_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture (batch)");
    b->graph = graph;
    PDG_TRY_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  PDG_TRY_HIP(hipGraphLaunch(b->exec, stream));
  return PDG_OK;
}

pdg_status pdg_batch_destroy(pdg_batch *b) {
  release_batch(b);
  return PDG_OK;
}

pdg_status pdg_problem_destroy(pdg_problem *p) {
  if (!p) return PDG_OK;
  for (int c = 0; c < 2; ++c) (void)pdg_problem_destroy(p->child[c]);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  delete p;
  return PDG_OK;
}

pdg_status pdg_problem_branch(const pdg_problem *p, int32_t which, pdg_problem **chain) {
  if (!p || !chain || which < 0 || which > 1) {
    set_error("NULL argument or which outside {0, 1}");
    return PDG_EINVAL;
  }
  if (p->joint)
    *chain = p->child[which];
  else
    *chain = which == 1 ? const_cast<pdg_problem *>(p) : nullptr;
  return PDG_OK;
}

pdg_status pdg_problem_buffer(const pdg_problem *p, int32_t which, void **ptr, size_t *bytes) {
  if (!p || !ptr || !bytes) {
    set_error("NULL argument");
    return PDG_EINVAL;
  }
  if (p->joint) {
    if (which != PDG_BUF_TERMS) {
      set_error("a sequence propagated both ways keeps its buffers per chain: "
                "see pdg_problem_branch");
      return PDG_EINVAL;
    }
    *ptr = p->jterms;
    *bytes = kTerms * 8;
    return PDG_OK;
  }
  const long long T = p->T, N = p->N, V = p->V, P = p->P;
  switch (which) {
    case PDG_BUF_PHAT: *ptr = p->phat; *bytes = T * 3 * N * 4; break;
    case PDG_BUF_XHAT: *ptr = p->xhat; *bytes = (T + 1) * 3 * V * 4; break;
    case PDG_BUF_NN: *ptr = p->nn; *bytes = T * (2 * N + (p->has_tm ? V + N : 0)) * 4; break;
    case PDG_BUF_LOSSES: *ptr = p->losses; *bytes = T * 4 * 8; break;
    case PDG_BUF_WCONF: *ptr = p->wconf; *bytes = T * 8; break;
    case PDG_BUF_GRAD: *ptr = p->grad; *bytes = T * P * 4; break;
    case PDG_BUF_PGRAD: *ptr = p->pgrad; *bytes = T * P * 4; break;
    case PDG_BUF_GPHAT: *ptr = p->gphat; *bytes = T * 3 * N * 4; break;
    case PDG_BUF_GXHAT: *ptr = p->gxhat; *bytes = T * 3 * V * 4; break;
    case PDG_BUF_TERMS: *ptr = p->terms; *bytes = kTerms * 8; break;
    case PDG_BUF_LAM: *ptr = p->lam; *bytes = T * 3 * V * 4; break;
    case PDG_BUF_SCREEN_TILES: *ptr = p->tiles; *bytes = p->tiles ? 8 : 0; break;
    case PDG_BUF_NN0: *ptr = p->nn0; *bytes = p->opt_x0 ? (V + N) * 4 : 0; break;
    case PDG_BUF_LOSS0: *ptr = p->loss0; *bytes = p->opt_x0 ? 16 : 0; break;
    case PDG_BUF_GX0: *ptr = p->gx0; *bytes = p->opt_x0 ? 3 * V * 4 : 0; break;
    case PDG_BUF_PGX0: *ptr = p->pgx0; *bytes = p->opt_x0 ? 3 * V * 4 : 0; break;
    default:
      set_error("unknown buffer %d", which);
      return PDG_EINVAL;
  }
  return PDG_OK;
}

}  // extern "C"
