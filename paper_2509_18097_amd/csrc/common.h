// Internal declarations shared by the HIP translation units of libpdg.
// Not part of the public ABI (that is include/pdg.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>

#include <atomic>

#include "pdg.h"

namespace pdg {

// ---------------------------------------------------------------- errors --
void set_error(const char *fmt, ...);
pdg_status hip_fail(hipError_t e, const char *what);

#define PDG_TRY_HIP(expr)                                                  \
  do {                                                                     \
    hipError_t _e = (expr);                                                \
    if (_e != hipSuccess) return ::pdg::hip_fail(_e, #expr);               \
  } while (0)

#define PDG_TRY(expr)                                                      \
  do {                                                                     \
    pdg_status _s = (expr);                                                \
    if (_s != PDG_OK) return _s;                                           \
  } while (0)

// Check the launch that was just enqueued.
inline pdg_status launched(const char *what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? PDG_OK : hip_fail(e, what);
}

// ------------------------------------------------------------ grid layout --
// Device-side copy of a grid stack description: per level the resolution,
// the float offset of the level inside the packed stack and the node offset
// (one channel) inside the stack's node numbering.
struct GridDev {
  int levels;
  int ch;                            // channels per cell: 3 (t) or 6 ([z; t], Eq. 4)
  int res[PDG_MAX_LEVELS];
  long long off[PDG_MAX_LEVELS];     // float offset of level l (ch channels)
  long long noff[PDG_MAX_LEVELS];    // node offset of level l (per channel)
  long long size;                    // floats per stack = ch * nodes
  long long nodes;                   // nodes per stack (per channel)
  float scale;
};

GridDev make_grid(const pdg_grid_desc &d);
// six_ok: the caller implements six-channel (Cayley) cells.
pdg_status check_grid(const pdg_grid_desc *d, bool six_ok = false);

// Trilinear stencil of coordinate s on a level with R >= 2 cells per axis:
// cell-centred values, border clamp to the hull of the centres.
__device__ __forceinline__ void stencil1(int R, float s, int &i0, float &f, bool &inside) {
  float u = (s + 1.0f) * (0.5f * (float)R) - 0.5f;
  inside = (u >= 0.0f) && (u <= (float)(R - 1));
  u = fminf(fmaxf(u, 0.0f), (float)(R - 1));
  int i = (int)floorf(u);
  i = i < R - 2 ? i : R - 2;
  i0 = i;
  f = u - (float)i;
}

// Weight of corner k (bit 0: +x, bit 1: +y, bit 2: +z) of the trilinear
// stencil with fractions (fx, fy, fz).
__device__ __forceinline__ float corner_weight(int k, float fx, float fy, float fz) {
  const float wx = (k & 1) ? fx : 1.0f - fx;
  const float wy = (k & 2) ? fy : 1.0f - fy;
  const float wz = (k & 4) ? fz : 1.0f - fz;
  return (wx * wy) * wz;
}

inline unsigned div_up(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// One-time set-up per device (kernel attributes such as the dynamic LDS limit
// are set per device): done(d) after mark(d); devices beyond the table repeat
// the set-up on every call.  Instances are function-local statics.
struct PerDevice {
  static constexpr int kDevices = 64;
  std::atomic<bool> f[kDevices];
  bool done(int d) const { return d >= 0 && d < kDevices && f[d].load(std::memory_order_acquire); }
  void mark(int d) {
    if (d >= 0 && d < kDevices) f[d].store(true, std::memory_order_release);
  }
};

// Workgroups are dealt to the eight XCDs (each with its own L2) in turn by
// linear id.  job_block maps workgroup lin of a grid of job_grid(njobs, nb)
// workgroups to (job, block < nb): with at least eight jobs every workgroup of
// a job runs on one XCD (its data cached in one L2); with fewer, job-major
// order.  It returns false for padding workgroups.
constexpr unsigned kXcdCount = 8;
__device__ __forceinline__ bool job_block(unsigned lin, unsigned njobs, unsigned nb, unsigned &job,
                                          unsigned &blk) {
  if (njobs >= kXcdCount) {
    const unsigned x = lin % kXcdCount, k = lin / kXcdCount;
    job = (k / nb) * kXcdCount + x;
    blk = k % nb;
  } else {
    job = lin / nb;
    blk = lin % nb;
  }
  return job < njobs;
}
inline unsigned long long job_grid(unsigned njobs, unsigned nb) {
  return njobs >= kXcdCount ? (unsigned long long)(njobs + kXcdCount - 1) / kXcdCount * kXcdCount * nb
                            : (unsigned long long)njobs * nb;
}
// For a 1-D grid of xcd_pad(n) workgroups: logical block of workgroup lin such
// that each XCD takes one contiguous range (consecutive blocks share an L2).
inline unsigned xcd_pad(unsigned long long n) {
  return (unsigned)((n + kXcdCount - 1) / kXcdCount * kXcdCount);
}
__device__ __forceinline__ unsigned xcd_block(unsigned lin, unsigned padded) {
  return (lin % kXcdCount) * (padded / kXcdCount) + lin / kXcdCount;
}

// Bump allocator over a caller workspace; with base == nullptr it only sizes.
struct Carve {
  char *base;
  size_t off = 0;
  explicit Carve(void *b) : base((char *)b) {}
  template <class T>
  T *take(long long count) {
    T *p = base ? (T *)(base + off) : nullptr;
    off += a256((size_t)(count > 0 ? count : 0) * sizeof(T));
    return p;
  }
};

// Pointers that kernels read from device-side tables (job and segment
// descriptors) are generic to the compiler, which then emits flat memory
// instructions and, unable to tell their counters apart, waits for all
// outstanding loads before each use.  Every such pointer addresses global
// memory; glb() states that, so global instructions with exact waits are used.
// (The qualifier means something only to the device pass; the host pass,
// which parses device code without generating it, sees plain pointers.)
// PDG_CONST marks memory that no lane writes while the kernel runs (the
// constant address space): uniform loads from it go through the scalar cache.
#if defined(__HIP_DEVICE_COMPILE__)
#define PDG_GLOBAL __attribute__((address_space(1)))
#define PDG_CONST __attribute__((address_space(4)))
#else
#define PDG_GLOBAL
#define PDG_CONST
#endif
template <typename T>
__device__ __forceinline__ PDG_GLOBAL T *glb(T *p) {
  return (PDG_GLOBAL T *)p;
}

// ------------------------------------------------------------ radix sort --
// Stable LSD radix sort of (key, value) pairs on uint32 keys, 8 bits a pass.
// Scratch: two key/value buffers of n entries plus a histogram.
size_t radix_sort_bytes(long long n);
// Sorts keys/vals in place (the scratch is used as the alternate buffer).
// bits: number of significant key bits (1..32).
pdg_status radix_sort(uint32_t *keys, uint32_t *vals, long long n, int bits, void *scratch,
                      hipStream_t stream);

// ------------------------------------------------------------- launchers --
// warp.hip
// order (nullable): batch b processes its points in the order
// order[b * order_stride + 0 .. n-1] (a spatial order gathers grid cells
// with better cache reuse; the result does not depend on it).
// Six-channel cells (Eq. 4-7): out = R(z^) x + t^ with [z^; t^] = level_scale *
// sum_l trilerp(G_l, x); x, out SoA [3][n] (out may alias x).
pdg_status launch_warp6(const GridDev &g, const float *grids, const float *x, float *out,
                        long long n, hipStream_t st);
// Its adjoint for an upstream gradient g (SoA [3][n]): u (nullable) receives
// d<g, out>/dz^ ([3][n]); gx (nullable) receives d<g, out>/dx.
pdg_status launch_adjoint6(const GridDev &g, const float *grids, const float *x,
                           const float *gout, float *u, float *gx, long long n, hipStream_t st);
// The same over `batch` grids / sample sets at the given strides (floats);
// gx = J^T g + gx_add (gx_add nullable, strided like gx).
pdg_status launch_warp6_batch(const GridDev &g, const float *grids, long long gs, const float *x,
                              long long xs, float *out, long long os, long long n, int batch,
                              hipStream_t st);
pdg_status launch_adjoint6_batch(const GridDev &g, const float *grids, long long gs,
                                 const float *x, long long xs, const float *gout, long long gos,
                                 float *u, long long us, float *gx, const float *gx_add,
                                 long long gxs, long long n, int batch, hipStream_t st);
// The template chain on six-channel cells in one launch each way: xhat
// [T+1][3][V] with frame 0 = X_0 set; reverse: lam [T][3][V] total adjoints
// (lam[T-1] = gd[T-1]), u [T][3][V] rotation adjoints of every transition.
pdg_status launch_chain_warp6(const GridDev &g, const float *params, long long P, float *xhat,
                              long long V, int T, hipStream_t st);
pdg_status launch_chain_reverse6(const GridDev &g, const float *params, long long P,
                                 const float *xhat, const float *gd, float *lam, float *u,
                                 long long V, int T, hipStream_t st);
pdg_status launch_warp(const GridDev &g, const float *grids, long long gstride, const float *x,
                       long long xstride, long long ldx, float *out, long long ostride,
                       long long ldo, long long n, int batch, hipStream_t st,
                       const int *order = nullptr, long long order_stride = 0);
// lam_out = gdir (nullable) + lam + J^T lam at positions x under `grids`.
pdg_status launch_chain_adjoint(const GridDev &g, const float *grids, const float *x, long long ldx,
                                const float *lam, long long ldl, const float *gdir, long long ldd,
                                float *lam_out, long long ldo, long long n, hipStream_t st);
// Template chain of Eq. 8 for all transitions in one launch: xhat[0] = x0,
// xhat[t+1] = warp(params + t*P, xhat[t]) ([F][3][V] SoA).
// order (nullable): vertex processing order, as for launch_warp.
pdg_status launch_chain_warp(const GridDev &g, const float *params, long long P, const float *x0,
                             float *xhat, long long V, int T, const int *order, hipStream_t st);
// Its reverse sweep: lam[T-1] = gd[T-1], lam[k-1] = gd[k-1] + lam[k] + J_k^T lam[k],
// J_k the Jacobian of grids k at xhat[k] (xhat: frames 0..T).
pdg_status launch_chain_reverse(const GridDev &g, const float *params, long long P,
                                const float *xhat, const float *gd, float *lam, long long V, int T,
                                const int *order, hipStream_t st);
// Entry keys for the deterministic grid scatter: for sample s of segment
// seg and level l (entry e = (seg*L + l)*S + s) the key is the global node id
// of the base cell, seg*nodes + noff[l] + cell (below 2^32), the value e.
pdg_status launch_scatter_keys(const GridDev &g, const float *x, long long xstride, long long ldx,
                               long long S, int segs, uint32_t *keys, uint32_t *vals,
                               hipStream_t st);
// Cell rows per segment: RS2 = R_0^2 + ... + R_{L-1}^2.
long long row_count(const GridDev &g);
// Row table of sorted keys: rstart[q], q = 0..segs*RS2, is the first entry of
// row q = seg*RS2 + R_0^2 + ... + R_{l-1}^2 + z*R + y ((z, y) of the base
// cell) or later.
pdg_status launch_row_table(const GridDev &g, const uint32_t *keys, long long nent, int segs,
                            int *rstart, hipStream_t st);
pdg_status launch_fill(float *p, long long count, float value, hipStream_t st);
// dst += src (count floats)
pdg_status launch_add(float *dst, const float *src, long long count, hipStream_t st);
// Three-channel view of half of a six-channel grid (half 0: the rotation
// channels z, 1: the translation channels t of every level), same stack
// stride: the preconditioner treats each half as a grid of its own.
GridDev half_view(const GridDev &g, int half);
pdg_status launch_copy(float *dst, const float *src, long long count, hipStream_t st);
// Upload up to 2 KB of host bytes to device memory in stream order (the bytes
// travel as a kernel argument, so the call is safe under graph capture).
pdg_status upload_small(void *dst, const void *src, size_t bytes, hipStream_t st);
// One list of sorted scatter entries (S samples per segment) and the values
// scattered: sample s of segment seg sits at x[seg*xstride + c*ldx + s] and
// carries lam[seg*lstride + c*ldl + s], c = 0..2.
struct ScatterList {
  const uint32_t *keys, *vals;
  const int *pstart;           // row table of the keys
  long long S;
  const float *x;
  long long xstride, ldx;
  const float *lam;
  long long lstride, ldl;
  float4 *ent;                 // [nent] staged (fx, fy, fz, lam0) in sorted order
  float2 *ent2;                // [nent] staged (lam1, lam2)
};
struct ScatterLists {
  ScatterList list[2];
  int count;
};
// Stages every sorted entry of a list: the stencil fractions of its sample on
// its level and the three values scattered (ent, ent2).
// lam_only: re-stage only the adjoint values of entries staged before.
pdg_status launch_scatter_stage(const GridDev &g, int segs, const ScatterList &L, hipStream_t st,
                                bool lam_only = false);
// grad = level_scale * sum_s w_k(s) lam(s) over the samples s of every list
// that have node k as a corner of their base cell, for every node of `segs`
// stacks (grad is overwritten; deterministic summation order).
// samples: sample count per segment over all lists (sizes the work split);
// scratch: gather_scratch_bytes(g, segs, samples) bytes (nullable when 0).
size_t gather_scratch_bytes(const GridDev &g, int segs, long long samples);
// ch0: first of the three channels written (0 or 3 for six-channel cells).
pdg_status launch_gather(const GridDev &g, int segs, const ScatterLists &sl, long long samples,
                         float *grad, float *scratch, hipStream_t st, int ch0 = 0);

// chamfer.hip
struct ChSeg {               // one (moving A, fixed B) Chamfer pair
  const float *a;            // SoA [3][n]
  const float *b;            // SoA [3][m]
  int n, m;
  int *nn_a;                 // [n]
  int *nn_b;                 // [m]
  float *ga;                 // SoA [3][n] gradient wrt a (nullable)
  unsigned a_base;           // global index of a_0 for the reverse scatter
  int pad;
  double *loss;              // [2] out: the two directional means
  double *part;              // [2][kLossBlocks] partial sums of those means
  const double *w;           // [2] gradient weights of the two directions
};
struct NNJob {               // one directed nearest-neighbour search
  const float *q; const float *c;
  int nq, nc;
  int *nn;
  int pad[2];
};
pdg_status launch_nn_exact(const NNJob *jobs, int njobs, int max_nq, hipStream_t st);

// chamfer_screen.hip: bf16 matrix-core screen + exact float32 re-rank with
// box culling over Morton-ordered 256-point tiles
struct ScreenSet {           // one point set packed as screen candidates and queries
  const float *x;            // SoA [3][n], original order
  int n;
  int pad;
  const int *perm;           // [n] packed position -> original index (nullable: identity)
  uint4 *pack;               // [n][2] packed bf16 rows (32 B per point), packed order
  float4 *coords;            // [n] (x, y, z, original index as int bits), packed order
  float4 *boxes;             // [ceil(n/256)][3] per 256-point tile: min corner, max corner,
                             // (centre C, radius): the frame the tile's rows are packed in
  int *inv;                  // nullable: [n] original index -> packed position
};
struct ScreenJob {           // one directed search: packed queries over packed candidates
  const float *c;            // candidates SoA [3][nc], original order (warm start)
  const float4 *q;           // query coords, packed order
  const float4 *qboxes;      // query tile boxes
  int nq, nc;
  int *nn;                   // [nq] original order; out, and the warm start when enabled
  const uint4 *pack;         // candidate rows, packed order
  const float4 *cc;          // candidate coords, packed order
  const float4 *cboxes;      // candidate tile boxes
  unsigned long long *tiles; // nullable: += 32x32x16 bf16 products issued
  const int *cinv;           // nullable: candidates' original index -> packed position
};
inline long long screen_tiles(long long n) { return (n + 255) / 256; }
// float4 entries of a set's box array: per tile its min corner, max corner,
// (centre, radius) and the min and max corners of its eight 32-point sub-tiles
inline long long screen_box_count(long long n) { return 19 * screen_tiles(n); }
// keys = 30-bit Morton codes over [-1, 1]^3 of x ([3][ld] SoA, n points), vals = index
pdg_status launch_morton(const float *x, long long ld, int n, uint32_t *keys, uint32_t *vals,
                         hipStream_t st);
pdg_status launch_screen_pack(const ScreenSet *sets, int nsets, int max_n, hipStream_t st);
pdg_status launch_nn_screen(const ScreenJob *jobs, int njobs, int max_nq, int warm,
                            hipStream_t st);
// the same jobs searched exactly in float32 (no matrix cores) with the same tile cull
pdg_status launch_nn_cull(const ScreenJob *jobs, int njobs, int max_nq, int warm, hipStream_t st);
// Chamfer modes that use the Morton-ordered packs and tile boxes
inline bool uses_packs(int mode) { return mode == PDG_CHAMFER_BF16_SCREEN || mode == PDG_CHAMFER_FP32_CULL; }
constexpr int kLossBlocks = 32;  // fixed partial count per (segment, direction)
constexpr int kIsoBlocks = 1024; // fixed partial count of the isometry loss
// each segment's part[dir*kLossBlocks + blk]; then its loss[dir] = mean.
// Segments may belong to different problems: each writes through its own
// pointers only.
pdg_status launch_chamfer_loss(const ChSeg *segs, int nseg, double alpha, hipStream_t st);
// ga <- forward-direction gradient (overwrite), with each segment's weight w[0].
pdg_status launch_chamfer_grad_fwd(const ChSeg *segs, int nseg, int max_n, float alpha,
                                   hipStream_t st);
// Reverse-direction keys: for b_j of segment seg the key is a_base + nn_b[j],
// value = global b index (seg base + j).  b_base[seg] = first global b index.
pdg_status launch_chamfer_rev_keys(const ChSeg *segs, int nseg, int max_m,
                                   const unsigned *b_base, uint32_t *keys, uint32_t *vals,
                                   hipStream_t st);
// Sorted (keys, vals) from launch_chamfer_rev_keys; part: 2 * rev_part_count(nent)
// float4 of scratch (run partials of workgroups).
long long rev_part_count(long long nent);
pdg_status launch_chamfer_rev_scatter(const ChSeg *segs, int nseg, const unsigned *b_base,
                                      const uint32_t *keys, const uint32_t *vals, long long nent,
                                      float alpha, float4 *part, hipStream_t st);

// precond.hip
struct CGLevel {             // one level of every stack in a preconditioner call
  int R;
  int shift;                 // log2(R), or -1 when R is not a power of two
  int iters;                 // CG iterations per solve
  float lam;
  long long off;             // float offset of the level in a stack
  int tile0;                 // first tile (level-major numbering)
  int tps;                   // tiles per system
  int sys0;                  // first system (level-major: level, stack, channel)
  int vec;                   // float4 path usable (R % 4 == 0, aligned)
  long long moff;            // word offset of the level in a stack's pruning mask
};
struct CGPlanDev {
  int levels;
  int batch;
  long long stack;           // floats per stack
  int ntiles, nsys;
  const uint32_t *mask;      // pruning masks [batch][mstack] words, or null (box)
  long long mstack;          // mask words per stack
  // kept tiles of pruned grids (ascending tile ids, level-major), or null:
  // launches then cover only these, level l's at [kfirst[l], kfirst[l] + kcount[l])
  const int *klist;
  int kfirst[PDG_MAX_LEVELS], kcount[PDG_MAX_LEVELS];
  CGLevel lv[PDG_MAX_LEVELS];
};
CGPlanDev cg_make_plan(const GridDev &g, int batch, const float *lam, const int *iters,
                       bool aligned16);
size_t cg_bytes(long long floats, int nsys, int ntiles);
pdg_status run_cg(const CGPlanDev &plan, float *g, long long floats, void *ws, hipStream_t st);

// dct.hip: exact (I + lam L)^-2 by the separable DCT-II (R <= 256)
size_t dct_bytes(const GridDev &g);
pdg_status dct_basis(const GridDev &g, void *ws, hipStream_t st);
// Adam (paper Sec. 3.6) on one value: the moments m, v are updated in
// place and the new parameter is returned; bc1, bc2 are 1 - beta^k.
__device__ __forceinline__ float adam_one(float b1, float b2, float eps, float lr, float bc1,
                                          float bc2, float gi, float &m, float &v, float th) {
  const float mi = b1 * m + (1.0f - b1) * gi;
  const float vi = b2 * v + (1.0f - b2) * gi * gi;
  m = mi;
  v = vi;
  const float mh = mi / bc1;
  const float vh = vi / bc2;
  return th - lr * mh / (sqrtf(vh) + eps);
}
// Bias corrections of step k = *step_dev + 1 (or step_host when step_dev is
// null) into sbc[0..1] (shared); every thread of the block must call it.
__device__ __forceinline__ void adam_bias(float b1, float b2, const int *step_dev, int step_host,
                                          float *sbc) {
  if (threadIdx.x == 0) {
    const int k = step_dev ? (*step_dev + 1) : step_host;
    sbc[0] = (float)(1.0 - pow((double)b1, (double)k));
    sbc[1] = (float)(1.0 - pow((double)b2, (double)k));
  }
  __syncthreads();
}

struct AdamLevels {
  int levels;
  long long off[PDG_MAX_LEVELS + 1];
  float lr[PDG_MAX_LEVELS];
  // pruned grids (adam_set_mask): the kept-cell bits ([stacks][mstack] words,
  // level l at moff[l], one bit per cell of its R^3 = r3[l], shared by the
  // channels); a value whose cell is pruned has zero gradient, parameter and
  // moments, which Adam leaves as they are, so it may be skipped.  Null: none.
  const uint32_t *mask = nullptr;
  long long mstack = 0;
  long long moff[PDG_MAX_LEVELS] = {};
  long long r3[PDG_MAX_LEVELS] = {};
};
// Adam applied by the last pass of the preconditioner: params, moments and
// per-level rates laid out like the preconditioned gradient.
struct AdamFuse {
  float *th, *m, *v;
  AdamLevels lv;
  float b1, b2, eps;
  const int *step_dev;
  int step_host;
};

// src -> data (src may equal data).  With adam non-null, levels whose last
// pass can apply Adam to the preconditioned values do so instead of writing
// them to data (data then holds those levels' spectra); their bits are set in
// *fused (levels not set need launch_adam_levels afterwards).
pdg_status run_dct(const GridDev &g, int batch, const float *lam, const float *src, float *data,
                   const void *ws, hipStream_t st, const AdamFuse *adam = nullptr,
                   unsigned *fused = nullptr);

// mesh.hip: (I + lambda L)^-2 on a mesh's vertices by one Chebyshev series.
// A plan (host metadata; its device tables and vectors live in the caller's
// ws of mesh_precond_bytes(V, E)) is built once from the edge list -- which
// synchronises the stream -- and applied any number of times.
struct MeshPlan;
size_t mesh_precond_bytes(long long V, long long E);
pdg_status mesh_plan_build(long long V, const int *edges, long long E, float lambda,
                           int max_degree, int terms, double tol, void *ws, hipStream_t st,
                           MeshPlan **out);
pdg_status mesh_plan_apply(const MeshPlan &p, const float *g, float *out, hipStream_t st);
void mesh_plan_free(MeshPlan *p);
int mesh_plan_terms(const MeshPlan &p);
long long mesh_plan_vertices(const MeshPlan &p);
// the parts a plan of this edge list (host copy) would use; arrays nullable
pdg_status mesh_partition_query(long long V, const int *edges_host, long long E, int *part_off,
                                int *part_core, int *lglob, int *ldist, long long *sizes);
int mesh_plan_parts(const MeshPlan &p);

// prune.hip: pruned grids.  A stack's mask holds one bit per cell of every
// level (levels packed in order, mask_words(R) words each; bit c of a level is
// bit c & 31 of its word c >> 5, c = (z R + y) R + x).
__host__ __device__ inline long long mask_words(int R) { return ((long long)R * R * R + 31) / 32; }
long long mask_stack_words(const GridDev &g);
size_t prune_bytes(const GridDev &g, int stacks);
pdg_status launch_prune_mask(const GridDev &g, int stacks, int span, const float *points,
                             long long n, int halo, uint32_t *mask, long long *active, void *ws,
                             hipStream_t st);
// values of pruned cells (every channel) of `batch` stacks set to zero
pdg_status launch_mask_apply(const GridDev &g, int batch, const uint32_t *mask, float *data,
                             hipStream_t st);
// plan fields for masked conjugate gradients (run_cg then solves on the
// graphs the kept cells induce)
void cg_set_mask(CGPlanDev &p, const GridDev &g, const uint32_t *mask);
// the same for Adam: values of pruned cells are skipped
void adam_set_mask(AdamLevels &lv, const GridDev &g, const uint32_t *mask);
// The kept-tile list of a masked plan from the masks on the host (hmask:
// [batch][mstack] words): fills p.kfirst / p.kcount and writes the list to
// `list` (host, p.ntiles entries at most); returns its length.
int cg_kept_tiles(CGPlanDev &p, const GridDev &g, const uint32_t *hmask, int *list);

// keyframe.hip: Eq. 19-20 (occupied 128^3 voxels per frame, weighted argmax)
size_t keyframe_bytes(int frames);
pdg_status launch_keyframe(const float *points, int frames, long long n, double gamma,
                           long long *counts, int *key, void *ws, hipStream_t st);

// optim.hip
pdg_status launch_adam(const AdamLevels &lv, long long stack, int batch, float b1, float b2,
                       float eps, const int *step_dev, int step_host, float *theta, float *m,
                       float *v, const float *g, hipStream_t st);
// The same for the levels whose bit in skip is clear.
pdg_status launch_adam_levels(const AdamLevels &lv, unsigned skip, long long stack, int batch,
                              float b1, float b2, float eps, const int *step_dev, int step_host,
                              float *theta, float *m, float *v, const float *g, hipStream_t st);
pdg_status launch_set_int(int *p, int value, hipStream_t st);
struct IsoArgs {
  const float *xhat;   // [F][3][V]
  const int *edges;    // [2][E]
  int V, E, T;
  float *sig;          // [T][E]   sign of the length change at frame t
  float *u;            // [T][3][E] unit edge vector at frame t
  double *partials;    // [kIsoBlocks]
  const int *inc_off;  // [V+1] incidence offsets
  const uint32_t *inc; // [2E] sorted incidences: edge*2 + side
  float *gx;           // [T][3][V] direct gradient (accumulated into)
  double coef;         // w_iso / (T*E)
};
// Edge pass: signs, unit vectors and loss partials (before the assembly).
pdg_status launch_iso_edges(const IsoArgs &a, hipStream_t st);
// Vertex pass: adds the isometry gradient into gx (after the Chamfer gradient).
pdg_status launch_iso_vertices(const IsoArgs &a, hipStream_t st);
pdg_status launch_incidence(const int *edges, int E, int V, uint32_t *keys, uint32_t *vals,
                            int *inc_off, void *sort_scratch, hipStream_t st);
struct AssembleArgs {
  const double *losses;      // [seg][2]: seg t = point term, seg T+t = template term
  const double *iso_partials;
  int T;
  int E;
  int has_tm;
  const int *epoch;
  int e_max;
  float w_iso;
  double *w;                 // out [seg][2] gradient weights
  double *wconf;             // out [T]
  double *terms;             // out [kTerms]
  double *user_terms;        // out [kTerms] nullable
  int Tn;                    // the 1/T of Eq. 14 (the sequence's T; T unless the
                             // chain is one of two leaving a keyframe)
  const double *partner_losses;  // the other chain's losses (its point terms
  int partner_T;                 // enter cd_max, Eq. 17), or null / 0
};
pdg_status launch_assemble(const AssembleArgs &a, hipStream_t st);
constexpr int kTerms = 9;  // loss terms of a step: L, L_transform, L_iso, cd_max,
                           // point mean, template mean, w_conf(T), epoch, L_mesh
// X_0 optimised (Eq. 9-10): terms[8] = L_mesh = loss0[0] + loss0[1] and
// terms[0] = terms[1] + terms[2] + terms[8]; the same two slots of user
// (nullable).
pdg_status launch_mesh_terms(double *terms, double *user, const double *loss0, hipStream_t st);
// Terms of a sequence propagated both ways from its keyframe from those of its
// backward (tb) and forward (tf) chains (either nullable): sums, the shared
// cd_max, w_conf and epoch of the forward chain (else the backward one).
pdg_status launch_joint_terms(const double *tb, const double *tf, double *out, double *user,
                              hipStream_t st);

}  // namespace pdg
