// Grid Sobolev preconditioner (paper Sec. 3.2, Eq. 3): g <- (I + lam L)^-2 g
// per (stack, level, channel) system, L the 6-neighbour combinatorial
// Laplacian of the R^3 cell box with free boundary.
//
// Two conjugate-gradient solves per system, matrix-free, float32 vectors and
// float64 inner products, with a fixed per-system iteration count (so the
// whole solve is stream-ordered with no host synchronisation).  All systems
// of all levels and stacks run in the same launches: a launch covers the
// concatenated tiles of every system; each workgroup finds its system by a
// binary search over the systems' first-tile table.
//
// Per iteration (p' = r + beta p, ping-pong buffers for p):
//   kernel A: p' from r and p, pq = <p', A p'> (A p' recomputed from p'
//             at the seven stencil points), writes p';
//   reduce  : alpha = rr / pq;
//   kernel B: x += alpha p', r -= alpha A p' (stencil on p'), rr' = <r, r>;
//   reduce  : beta = rr' / rr.
// HBM traffic per cell and iteration: A reads r, p and writes p' (12 B);
// B reads p', x, r and writes x, r (20 B).
#include "common.h"

namespace pdg {
namespace {

constexpr int kThreads = 256;
constexpr int kCells = 4;                 // consecutive x cells per thread
constexpr int kTileCells = kThreads * kCells;

struct CGState {
  float *x, *r, *p0, *p1;
  double *pq_part, *rr_part;   // [ntiles]
  double *rr, *alpha, *beta;   // [nsys]
};

__device__ __forceinline__ int find_sys(const CGSys *__restrict__ sys, int nsys, int tile) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sys[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// XCD-aware tile order: consecutive workgroup ids go to different XCDs, so
// give each XCD a contiguous range of tiles (neighbouring z-planes stay in
// the same L2).
__device__ __forceinline__ int tile_of_block(int ntiles) {
  const int per = (ntiles + 7) >> 3;
  return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) t += sh[i];
  return t;
}

// (A v)(c) = v(c) + lam * sum_{nbr} (v(c) - v(nbr)) over in-box neighbours,
// with v given by a functor.
template <class F>
__device__ __forceinline__ float apply_A(const F &v, float vc, int x, int y, int z, int R, int c,
                                         float lam) {
  const int R2 = R * R;
  float s = 0.f;
  if (x > 0) s += vc - v(c - 1);
  if (x < R - 1) s += vc - v(c + 1);
  if (y > 0) s += vc - v(c - R);
  if (y < R - 1) s += vc - v(c + R);
  if (z > 0) s += vc - v(c - R2);
  if (z < R - 1) s += vc - v(c + R2);
  return vc + lam * s;
}

__global__ __launch_bounds__(kThreads) void cg_init_kernel(const CGSys *__restrict__ sys, int nsys,
                                                           int ntiles, const float *__restrict__ src,
                                                           float *__restrict__ r,
                                                           float *__restrict__ x,
                                                           double *__restrict__ rr_part) {
  __shared__ double sh[kThreads / 64];
  const int tile = tile_of_block(ntiles);
  if (tile >= ntiles) return;
  const CGSys S = sys[find_sys(sys, nsys, tile)];
  const long long n = (long long)S.R * S.R * S.R;
  const long long c0 = (long long)(tile - S.tile0) * kTileCells + threadIdx.x * kCells;
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < kCells; ++k) {
    const long long c = c0 + k;
    if (c < n) {
      const float v = src[S.base + c];
      r[S.base + c] = v;
      x[S.base + c] = 0.f;
      acc += (double)v * (double)v;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) rr_part[tile] = t;
}

__global__ __launch_bounds__(kThreads) void cg_a_kernel(const CGSys *__restrict__ sys, int nsys,
                                                        int ntiles, int k, CGState s,
                                                        const float *__restrict__ pin,
                                                        float *__restrict__ pout) {
  __shared__ double sh[kThreads / 64];
  const int tile = tile_of_block(ntiles);
  if (tile >= ntiles) return;
  const int si = find_sys(sys, nsys, tile);
  const CGSys S = sys[si];
  if (k >= S.iters) return;
  const int R = S.R;
  const int n = R * R * R;
  const float beta = k == 0 ? 0.f : (float)s.beta[si];
  const float *rr = s.r + S.base;
  const float *pp = pin + S.base;
  auto pn = [&](int c) { return k == 0 ? rr[c] : rr[c] + beta * pp[c]; };
  const int c0 = (tile - S.tile0) * kTileCells + threadIdx.x * kCells;
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < kCells; ++q) {
    const int c = c0 + q;
    if (c < n) {
      const int x = c % R, y = (c / R) % R, z = c / (R * R);
      const float vc = pn(c);
      const float av = apply_A(pn, vc, x, y, z, R, c, S.lam);
      pout[S.base + c] = vc;
      acc += (double)vc * (double)av;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) s.pq_part[tile] = t;
}

__global__ __launch_bounds__(kThreads) void cg_b_kernel(const CGSys *__restrict__ sys, int nsys,
                                                        int ntiles, int k, CGState s,
                                                        const float *__restrict__ pcur) {
  __shared__ double sh[kThreads / 64];
  const int tile = tile_of_block(ntiles);
  if (tile >= ntiles) return;
  const int si = find_sys(sys, nsys, tile);
  const CGSys S = sys[si];
  if (k >= S.iters) return;
  const int R = S.R;
  const int n = R * R * R;
  const float alpha = (float)s.alpha[si];
  const float *pp = pcur + S.base;
  auto pv = [&](int c) { return pp[c]; };
  const int c0 = (tile - S.tile0) * kTileCells + threadIdx.x * kCells;
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < kCells; ++q) {
    const int c = c0 + q;
    if (c < n) {
      const int x = c % R, y = (c / R) % R, z = c / (R * R);
      const float vc = pp[c];
      const float av = apply_A(pv, vc, x, y, z, R, c, S.lam);
      const long long a = S.base + c;
      s.x[a] += alpha * vc;
      const float rn = s.r[a] - alpha * av;
      s.r[a] = rn;
      acc += (double)rn * (double)rn;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) s.rr_part[tile] = t;
}

__device__ __forceinline__ int tiles_of(const CGSys &S) {
  const long long n = (long long)S.R * S.R * S.R;
  return (int)((n + kTileCells - 1) / kTileCells);
}

// mode 0: rr = sum rr_part (after init); mode 1: alpha = rr / sum pq_part;
// mode 2: rr' = sum rr_part, beta = rr'/rr, rr = rr'.
__global__ __launch_bounds__(kThreads) void cg_reduce_kernel(const CGSys *__restrict__ sys, int k,
                                                             int mode, CGState s) {
  __shared__ double sh[kThreads / 64];
  const int si = blockIdx.x;
  const CGSys S = sys[si];
  if (mode != 0 && k >= S.iters) return;
  const double *part = mode == 1 ? s.pq_part : s.rr_part;
  const int nt = tiles_of(S);
  double acc = 0.0;
  for (int i = threadIdx.x; i < nt; i += kThreads) acc += part[S.tile0 + i];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    if (mode == 0) {
      s.rr[si] = t;
    } else if (mode == 1) {
      s.alpha[si] = t > 0.0 ? s.rr[si] / t : 0.0;
    } else {
      const double old = s.rr[si];
      s.beta[si] = old > 0.0 ? t / old : 0.0;
      s.rr[si] = t;
    }
  }
}

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t cg_bytes(long long floats, int nsys, int ntiles) {
  return 4 * a256((size_t)floats * 4) + 2 * a256((size_t)ntiles * 8) + 3 * a256((size_t)nsys * 8);
}

pdg_status run_cg(const CGSys *sys, int nsys, int ntiles, int kmax, float *g, long long floats,
                  void *ws, hipStream_t st) {
  if (nsys <= 0 || ntiles <= 0) return PDG_OK;
  char *w = (char *)ws;
  CGState s;
  s.x = (float *)w;
  w += a256((size_t)floats * 4);
  s.r = (float *)w;
  w += a256((size_t)floats * 4);
  s.p0 = (float *)w;
  w += a256((size_t)floats * 4);
  s.p1 = (float *)w;
  w += a256((size_t)floats * 4);
  s.pq_part = (double *)w;
  w += a256((size_t)ntiles * 8);
  s.rr_part = (double *)w;
  w += a256((size_t)ntiles * 8);
  s.rr = (double *)w;
  w += a256((size_t)nsys * 8);
  s.alpha = (double *)w;
  w += a256((size_t)nsys * 8);
  s.beta = (double *)w;
  const unsigned nb = (unsigned)(((ntiles + 7) / 8) * 8);
  // solve 1: (I + lam L) y = g, y in s.x ; solve 2: (I + lam L) z = y, z in g
  for (int solve = 0; solve < 2; ++solve) {
    const float *src = solve == 0 ? g : s.x;
    float *xdst = solve == 0 ? s.x : g;
    // solve 2 starts from r = y: copy through cg_init with x = g
    CGState t = s;
    t.x = xdst;
    cg_init_kernel<<<nb, kThreads, 0, st>>>(sys, nsys, ntiles, src, t.r, t.x, t.rr_part);
    PDG_TRY(launched("cg_init"));
    cg_reduce_kernel<<<nsys, kThreads, 0, st>>>(sys, 0, 0, t);
    PDG_TRY(launched("cg_reduce"));
    for (int k = 0; k < kmax; ++k) {
      float *pin = (k & 1) ? t.p1 : t.p0;
      float *pout = (k & 1) ? t.p0 : t.p1;
      cg_a_kernel<<<nb, kThreads, 0, st>>>(sys, nsys, ntiles, k, t, pin, pout);
      PDG_TRY(launched("cg_a"));
      cg_reduce_kernel<<<nsys, kThreads, 0, st>>>(sys, k, 1, t);
      PDG_TRY(launched("cg_reduce"));
      cg_b_kernel<<<nb, kThreads, 0, st>>>(sys, nsys, ntiles, k, t, pout);
      PDG_TRY(launched("cg_b"));
      cg_reduce_kernel<<<nsys, kThreads, 0, st>>>(sys, k, 2, t);
      PDG_TRY(launched("cg_reduce"));
    }
  }
  return PDG_OK;
}

}  // namespace pdg
