// Mesh-vertex preconditioner (paper Sec. 3.2 applied to the vertices of X_0,
// Sec. 3.6): out = (I + lambda L)^{-2} g per coordinate channel, with L = D - A
// the combinatorial Laplacian of the mesh's edge graph.
//
// The adjacency is built on the device: both directions of every edge sorted
// by source vertex (radix sort) and a row table by binary search.  Each of the
// two solves is a Chebyshev iteration on the spectrum bound [1, 1 + 2 lambda
// d_max] of I + lambda L (Gershgorin), so it needs no inner products: one
// launch per iteration computes q = (I + lambda L) p from the neighbours of
// every vertex and updates x, r and the next direction, in float64.
#include "common.h"

namespace pdg {
namespace {

// Directed entries (src, dst) of every edge, both directions; entries of
// edges with an endpoint outside [0, V) get the key V (sorted past the rows).
__global__ __launch_bounds__(256) void mesh_keys_kernel(const int *__restrict__ edges, long long E,
                                                        long long V, uint32_t *__restrict__ keys,
                                                        uint32_t *__restrict__ vals) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int a = edges[e], b = edges[E + e];
  const bool ok = a >= 0 && b >= 0 && a < V && b < V;
  keys[2 * e] = ok ? (uint32_t)a : (uint32_t)V;
  vals[2 * e] = ok ? (uint32_t)b : 0u;
  keys[2 * e + 1] = ok ? (uint32_t)b : (uint32_t)V;
  vals[2 * e + 1] = ok ? (uint32_t)a : 0u;
}

// off[v] = first sorted entry with key >= v, v = 0..V.
__global__ __launch_bounds__(256) void mesh_rows_kernel(const uint32_t *__restrict__ keys,
                                                        long long nent, long long V,
                                                        int *__restrict__ off) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v > V) return;
  long long lo = 0, hi = nent;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if ((long long)keys[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  off[v] = (int)lo;
}

// x = 0, r = p = b (b float32 or float64 SoA [3][V]).  The second solve
// passes the first solve's result as b and x at once, so b and x may alias
// (no restrict on either: the compiler keeps the store of x[i] after the
// load of b[i]).
template <typename T>
__global__ __launch_bounds__(256) void cheb_init_kernel(const T *b, long long n, double *x,
                                                        double *__restrict__ r,
                                                        double *__restrict__ p) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = (double)b[i];
  x[i] = 0.0;
  r[i] = v;
  p[i] = v;
}

// One Chebyshev step: q = (I + lam L) p, x += alpha p, r -= alpha q,
// pn = r + beta p (beta of the next step).
__global__ __launch_bounds__(256) void cheb_step_kernel(const int *__restrict__ off,
                                                        const uint32_t *__restrict__ nbr,
                                                        long long V, double lam, double alpha,
                                                        double beta, const double *__restrict__ p,
                                                        double *__restrict__ x,
                                                        double *__restrict__ r,
                                                        double *__restrict__ pn) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int a = off[v], b = off[v + 1];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int k = a; k < b; ++k) {
    const long long u = nbr[k];
    s0 += p[u];
    s1 += p[V + u];
    s2 += p[2 * V + u];
  }
  const double dg = 1.0 + lam * (double)(b - a);
  const double p0 = p[v], p1 = p[V + v], p2 = p[2 * V + v];
  const double q[3] = {dg * p0 - lam * s0, dg * p1 - lam * s1, dg * p2 - lam * s2};
  const double pv[3] = {p0, p1, p2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const long long i = c * V + v;
    x[i] += alpha * pv[c];
    const double rr = r[i] - alpha * q[c];
    r[i] = rr;
    pn[i] = rr + beta * pv[c];
  }
}

__global__ __launch_bounds__(256) void to_float_kernel(const double *__restrict__ a, long long n,
                                                       float *__restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)a[i];
}

}  // namespace

struct MeshWs {
  uint32_t *keys, *vals;
  int *off;
  double *x, *r, *p0, *p1;
  void *sort;
};

namespace {
MeshWs mesh_layout(Carve &c, long long V, long long E) {
  MeshWs w;
  const long long ne = 2 * E;
  w.keys = c.take<uint32_t>(ne > 0 ? ne : 1);
  w.vals = c.take<uint32_t>(ne > 0 ? ne : 1);
  w.off = c.take<int>(V + 1);
  w.x = c.take<double>(3 * V);
  w.r = c.take<double>(3 * V);
  w.p0 = c.take<double>(3 * V);
  w.p1 = c.take<double>(3 * V);
  w.sort = c.take<char>((long long)radix_sort_bytes(ne > 0 ? ne : 1));
  return w;
}
}  // namespace

size_t mesh_precond_bytes(long long V, long long E) {
  Carve c(nullptr);
  mesh_layout(c, V, E);
  return c.off;
}

int cheb_iterations(double kappa, double tol) {
  const double sq = sqrt(kappa);
  const double rho = (sq - 1.0) / (sq + 1.0);
  if (rho <= 0.0) return 1;
  const double k = ceil(log(2.0 / tol) / -log(rho));
  return k < 1.0 ? 1 : (int)k;
}

pdg_status launch_mesh_adjacency(long long V, const int *edges, long long E, void *ws,
                                 hipStream_t st) {
  Carve c(ws);
  MeshWs w = mesh_layout(c, V, E);
  const long long ne = 2 * E;
  if (ne > 0) {
    mesh_keys_kernel<<<div_up(E, 256), 256, 0, st>>>(edges, E, V, w.keys, w.vals);
    PDG_TRY(launched("mesh_keys"));
    int bits = 1;
    while (bits < 32 && (1ull << bits) <= (unsigned long long)V) ++bits;
    PDG_TRY(radix_sort(w.keys, w.vals, ne, bits, w.sort, st));
  }
  mesh_rows_kernel<<<div_up(V + 1, 256), 256, 0, st>>>(w.keys, ne, V, w.off);
  return launched("mesh_rows");
}

pdg_status launch_mesh_precondition(long long V, const int *edges, long long E, float lambda,
                                    int max_degree, int iters, const float *g, float *out,
                                    void *ws, hipStream_t st) {
  PDG_TRY(launch_mesh_adjacency(V, edges, E, ws, st));
  return launch_mesh_solve(V, E, lambda, max_degree, iters, g, out, ws, st);
}

pdg_status launch_mesh_solve(long long V, long long E, float lambda, int max_degree, int iters,
                             const float *g, float *out, void *ws, hipStream_t st) {
  Carve c(ws);
  MeshWs w = mesh_layout(c, V, E);
  // Chebyshev coefficients on [lmin, lmax] = [1, 1 + 2 lambda d_max]
  const double lam = lambda, lmin = 1.0, lmax = 1.0 + 2.0 * lam * (double)max_degree;
  const double d = 0.5 * (lmax + lmin), cc = 0.5 * (lmax - lmin);
  const long long n = 3 * V;
  for (int solve = 0; solve < 2; ++solve) {
    if (solve == 0)
      cheb_init_kernel<float><<<div_up(n, 256), 256, 0, st>>>(g, n, w.x, w.r, w.p0);
    else
      cheb_init_kernel<double><<<div_up(n, 256), 256, 0, st>>>(w.x, n, w.x, w.r, w.p0);
    PDG_TRY(launched("cheb_init"));
    double alpha = 1.0 / d;
    double *p = w.p0, *pn = w.p1;
    for (int i = 1; i <= iters; ++i) {
      // beta and alpha of step i + 1 (Chebyshev recurrence)
      const double beta = i == 1 ? 0.5 * (cc * alpha) * (cc * alpha)
                                 : (0.5 * cc * alpha) * (0.5 * cc * alpha);
      const double alpha_next = 1.0 / (d - beta / alpha);
      cheb_step_kernel<<<div_up(V, 256), 256, 0, st>>>(w.off, w.vals, V, lam, alpha, beta, p, w.x,
                                                       w.r, pn);
      PDG_TRY(launched("cheb_step"));
      double *t = p;
      p = pn;
      pn = t;
      alpha = alpha_next;
    }
  }
  to_float_kernel<<<div_up(n, 256), 256, 0, st>>>(w.x, n, out);
  return launched("mesh_out");
}

}  // namespace pdg
