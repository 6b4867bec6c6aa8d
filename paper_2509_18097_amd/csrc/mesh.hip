// Mesh-vertex preconditioner (paper Sec. 3.2 applied to the vertices of X_0,
// Sec. 3.6): out = (I + lambda L)^{-2} g per coordinate channel, with L = D - A
// the combinatorial Laplacian of the mesh's edge graph.
//
// With A = I + lambda L, whose spectrum lies in [1, kappa], kappa =
// 1 + 2 lambda d_max (Gershgorin), the operator is f(A) for f(t) = t^-2, and
// one Chebyshev series of f on [1, kappa] gives it without inner products:
//   out = sum_j c_j T_j(B) g,   B = (2 A - (kappa + 1) I) / (kappa - 1),
// with the coefficients c_j from f at Chebyshev nodes (float64, on the host)
// and the series truncated where the sum of the dropped |c_j| -- a bound on
// the operator-norm error, since |T_j| <= 1 on the spectrum -- is below tol.
// The vectors v_j = T_j(B) g follow the three-term recurrence
// v_{j+1} = 2 B v_j - v_{j-1}, one neighbour gather per term, in float64
// (random inputs give outputs some 30 times smaller than g while the v_j stay
// at the scale of g, so float32 terms would leave errors near 1e-5 of the
// result).  For f = t^-2 at lambda = 16 on a valence-6 mesh this is about 146
// terms where two Chebyshev solves of A need twice 117 steps.
//
// Communication avoiding: the vertices are split into parts grown by
// breadth-first search (about 256 each); a part's block of 1024 threads holds
// in LDS the part and every vertex within k = 10 edges of it (about 1,300 on
// a valence-6 mesh), runs k recurrence steps there (a vertex at distance d
// from the part is updated in the first k - d steps, whose inputs it has),
// then writes the part's v_j, v_{j-1} and the series sum.  A launch thus
// advances k terms, with reads from the other launch's buffers only.  The
// plan (parts, their k-edge neighbourhoods, local adjacency) is built on the
// host from the edge list; a graph whose neighbourhoods do not fit the LDS
// runs one term per launch instead.  (Measured on the 40,962-vertex
// template: parts of 1024 with k = 8 take 0.54 ms, 256 with k = 10 0.32 ms,
// one term per launch 0.93 ms.)
#include "common.h"

#include <algorithm>
#include <vector>

namespace pdg {
namespace {

#ifndef PDG_MESH_THREADS
#define PDG_MESH_THREADS 1024
#define PDG_MESH_STEPS 10
#define PDG_MESH_LOCAL 1536
#define PDG_MESH_CORE 256
#endif
constexpr int kMeshThreads = PDG_MESH_THREADS;
constexpr int kMeshSteps = PDG_MESH_STEPS;      // recurrence terms per block launch (halo depth)
constexpr int kMeshLocalMax = PDG_MESH_LOCAL;   // local vertices of a part (LDS: 48 B each)
constexpr int kMeshOwn = (kMeshLocalMax + kMeshThreads - 1) / kMeshThreads;
constexpr int kMeshCore = PDG_MESH_CORE;        // target part size
constexpr int kRegNbr = 8;                      // neighbours held in registers
constexpr int kCoefNodes = 1024;       // Chebyshev nodes of the coefficient sums
constexpr int kMeshMaxTerms = kCoefNodes - 1;

struct MeshDev {
  long long V;
  double lam, b1, b0;                  // B = b1 A + b0 I
  const double *coef;                  // [terms]
  // parts
  const int *part_off;                 // [npart + 1] first local vertex of each part
  const int *part_core;                // [npart] vertices of the part proper
  const int *lglob;                    // [nloc] global index of a local vertex
  const int *ldist;                    // [nloc] distance from the part (0: in it)
  const int *ladj_off;                 // [nloc + 1] local adjacency (vertices with d < k)
  const unsigned short *ladj;          // local neighbour index
  // one-term path
  const int *off;                      // [V + 1] global adjacency
  const int *nbr;
};

// v_0 = g (float64 copy), y = c_0 g.
__global__ __launch_bounds__(256) void mesh_init_kernel(MeshDev M, const float *__restrict__ g,
                                                        double *__restrict__ v0,
                                                        double *__restrict__ y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * M.V) return;
  const double v = (double)g[i];
  v0[i] = v;
  y[i] = M.coef[0] * v;
}

// B v at vertex i from its own value and its neighbours' sum.
__device__ __forceinline__ double apply_b(const MeshDev &M, double v, double s, int deg) {
  const double av = (1.0 + M.lam * (double)deg) * v - M.lam * s;
  return M.b1 * av + M.b0 * v;
}

// Terms j0 + 1 .. j0 + ks of one part: v_{j0} (all local vertices) and
// v_{j0-1} (own) from (cur, prev), the part's v_{j0+ks}, v_{j0+ks-1} to
// (ncur, nprev), its series sum y updated in place; with `out` set (the last
// launch) the sum is written there in float32 instead.
__global__ __launch_bounds__(kMeshThreads) void mesh_block_kernel(
    MeshDev M, int j0, int ks, const double *__restrict__ cur, const double *__restrict__ prev,
    double *__restrict__ ncur, double *__restrict__ nprev, double *__restrict__ y,
    float *__restrict__ out) {
  extern __shared__ double lv[];       // [2][3][nloc]
  const int part = blockIdx.x;
  const int base = M.part_off[part];
  const int nloc = M.part_off[part + 1] - base;
  const int ncore = M.part_core[part];
  const long long V = M.V;
  const int t = threadIdx.x;
  for (int i = t; i < nloc; i += kMeshThreads) {
    const long long gi = M.lglob[base + i];
#pragma unroll
    for (int c = 0; c < 3; ++c) lv[c * nloc + i] = cur[c * V + gi];
  }
  double vp[kMeshOwn][3], ys[kMeshOwn][3];
  int dist[kMeshOwn], a0[kMeshOwn], deg[kMeshOwn];
  unsigned nb[kMeshOwn][kRegNbr / 2];   // the first kRegNbr neighbours, two per register
#pragma unroll
  for (int m = 0; m < kMeshOwn; ++m) {
    const int i = t + m * kMeshThreads;
    dist[m] = i < nloc ? M.ldist[base + i] : kMeshSteps + 1;
    a0[m] = deg[m] = 0;
#pragma unroll
    for (int q = 0; q < kRegNbr / 2; ++q) nb[m][q] = 0u;
#pragma unroll
    for (int c = 0; c < 3; ++c) vp[m][c] = ys[m][c] = 0.0;
    if (i < nloc && dist[m] < ks) {
      a0[m] = M.ladj_off[base + i];
      deg[m] = M.ladj_off[base + i + 1] - a0[m];
#pragma unroll
      for (int q = 0; q < kRegNbr; ++q)
        if (q < deg[m]) nb[m][q / 2] |= (unsigned)M.ladj[a0[m] + q] << (16 * (q & 1));
      const long long gi = M.lglob[base + i];
#pragma unroll
      for (int c = 0; c < 3; ++c) vp[m][c] = j0 > 0 ? prev[c * V + gi] : 0.0;
      if (i < ncore)
#pragma unroll
        for (int c = 0; c < 3; ++c) ys[m][c] = y[c * V + gi];
    }
  }
  __syncthreads();
  for (int s = 1; s <= ks; ++s) {
    const int j = j0 + s - 1;                        // this step forms v_{j+1}
    const double *src = lv + ((s - 1) & 1) * 3 * nloc;
    double *dst = lv + (s & 1) * 3 * nloc;
    const double cj = M.coef[j + 1];
#pragma unroll
    for (int m = 0; m < kMeshOwn; ++m) {
      const int i = t + m * kMeshThreads;
      if (dist[m] > ks - s) continue;              // its inputs are not current any more
      // all register-held neighbours' loads issued together (index 0 stands
      // in for absent ones and is not added)
      double g0[kRegNbr], g1[kRegNbr], g2[kRegNbr];
#pragma unroll
      for (int q = 0; q < kRegNbr; ++q) {
        const int u = (int)((nb[m][q / 2] >> (16 * (q & 1))) & 0xffffu);
        g0[q] = src[u];
        g1[q] = src[nloc + u];
        g2[q] = src[2 * nloc + u];
      }
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int q = 0; q < kRegNbr; ++q)
        if (q < deg[m]) {
          s0 += g0[q];
          s1 += g1[q];
          s2 += g2[q];
        }
      for (int k = a0[m] + kRegNbr; k < a0[m] + deg[m]; ++k) {   // degrees above kRegNbr
        const int u = M.ladj[k];
        s0 += src[u];
        s1 += src[nloc + u];
        s2 += src[2 * nloc + u];
      }
      const double sum[3] = {s0, s1, s2};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double v = src[c * nloc + i];
        const double bv = apply_b(M, v, sum[c], deg[m]);
        const double vn = j == 0 ? bv : 2.0 * bv - vp[m][c];
        dst[c * nloc + i] = vn;
        vp[m][c] = v;
        ys[m][c] += cj * vn;
      }
    }
    __syncthreads();
  }
  const double *fin = lv + (ks & 1) * 3 * nloc;
#pragma unroll
  for (int m = 0; m < kMeshOwn; ++m) {
    const int i = t + m * kMeshThreads;
    if (i >= ncore) continue;
    const long long gi = M.lglob[base + i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (out) {
        out[c * V + gi] = (float)ys[m][c];
      } else {
        ncur[c * V + gi] = fin[c * nloc + i];
        nprev[c * V + gi] = vp[m][c];
        y[c * V + gi] = ys[m][c];
      }
    }
  }
}

// One term on the global adjacency (graphs whose neighbourhoods exceed the
// LDS): v_{j+1} = 2 B v_j - v_{j-1} (B v_0 for j = 0), y += c_{j+1} v_{j+1}.
__global__ __launch_bounds__(256) void mesh_term_kernel(MeshDev M, int j,
                                                        const double *__restrict__ cur,
                                                        const double *__restrict__ prev,
                                                        double *__restrict__ next,
                                                        double *__restrict__ y) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long V = M.V;
  if (v >= V) return;
  const int a = M.off[v], b = M.off[v + 1];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int k = a; k < b; ++k) {
    const long long u = M.nbr[k];
    s0 += cur[u];
    s1 += cur[V + u];
    s2 += cur[2 * V + u];
  }
  const double sum[3] = {s0, s1, s2};
  const double cj = M.coef[j + 1];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const long long i = c * V + v;
    const double bv = apply_b(M, cur[i], sum[c], b - a);
    const double vn = j == 0 ? bv : 2.0 * bv - prev[i];
    next[i] = vn;
    y[i] += cj * vn;
  }
}

__global__ __launch_bounds__(256) void mesh_out_kernel(const double *__restrict__ y, long long n,
                                                       float *__restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)y[i];
}

// Workspace: global adjacency, four float64 vector sets, the series sum, the
// coefficients and the part tables (capacity fixed by V and E; a plan that
// needs more runs one term per launch).
struct MeshWs {
  int *off, *nbr;
  double *vec[4], *y, *coef;
  int *part_off, *part_core, *lglob, *ldist, *ladj_off;
  unsigned short *ladj;
  long long slots, adj_slots, parts;
};

MeshWs mesh_layout(Carve &c, long long V, long long E) {
  MeshWs w;
  w.off = c.take<int>(V + 1);
  w.nbr = c.take<int>(2 * E > 0 ? 2 * E : 1);
  for (double *&p : w.vec) p = c.take<double>(3 * V > 0 ? 3 * V : 1);
  w.y = c.take<double>(3 * V > 0 ? 3 * V : 1);
  w.coef = c.take<double>(kMeshMaxTerms);
  w.parts = V / 16 + 1;
  w.slots = 12 * V + kMeshLocalMax;
  w.adj_slots = 24 * E + 8 * kMeshLocalMax;
  w.part_off = c.take<int>(w.parts + 1);
  w.part_core = c.take<int>(w.parts);
  w.lglob = c.take<int>(w.slots);
  w.ldist = c.take<int>(w.slots);
  w.ladj_off = c.take<int>(w.slots + 1);
  w.ladj = c.take<unsigned short>(w.adj_slots);
  return w;
}

// Chebyshev coefficients of t^-2 on [1, kappa] from kCoefNodes nodes; returns
// the number of terms whose dropped tail sums below tol (0: more than the cap).
int mesh_coefficients(double kappa, double tol, int terms, std::vector<double> &c) {
  const int N = kCoefNodes;
  std::vector<double> f(N), th(N);
  for (int m = 0; m < N; ++m) {
    th[m] = M_PI * (m + 0.5) / N;
    const double tt = 0.5 * ((kappa - 1.0) * cos(th[m]) + (kappa + 1.0));
    f[m] = 1.0 / (tt * tt);
  }
  c.assign(N, 0.0);
  for (int j = 0; j < N; ++j) {
    double s = 0.0;
    for (int m = 0; m < N; ++m) s += f[m] * cos(j * th[m]);
    c[j] = (j == 0 ? 1.0 : 2.0) * s / N;
  }
  if (terms > 0) return terms <= kMeshMaxTerms ? terms : 0;
  double tail = 0.0;
  int n = N;
  for (int j = N - 1; j >= 1; --j) {       // smallest n with sum_{j >= n} |c_j| <= tol
    tail += fabs(c[j]);
    if (tail > tol) break;
    n = j;
  }
  return n <= kMeshMaxTerms ? n : 0;       // n = N: not resolved by the nodes
}

// Parts of the vertex set for the LDS path: each grown by breadth-first
// search from the lowest unassigned vertex within its piece of the unassigned
// vertices (about kMeshCore vertices), with every vertex within kMeshSteps
// edges of it, ordered by distance (the part first); local adjacency for the
// vertices closer than kMeshSteps.  ok = false when a part cannot be made to
// fit kMeshLocalMax or the capacities.
struct MeshParts {
  std::vector<int> part_off{0}, part_core, lglob, ldist, ladj_off;
  std::vector<unsigned short> ladj;
  int lmax = 0;
  bool ok = false;
};

void mesh_partition(long long V, const std::vector<int> &off, const std::vector<int> &nbr,
                    long long parts_cap, long long slots_cap, long long adj_cap, MeshParts &P) {
  std::vector<int> owner(V, -1), stamp(V, -1), lidx(V, 0), queue;
  long long next_seed = 0;
  int np = 0;
  P.ok = true;
  while (true) {
    while (next_seed < V && owner[next_seed] >= 0) ++next_seed;
    if (next_seed >= V) break;
    int want = kMeshCore;
    bool placed = false;
    while (!placed && want >= 16) {
      // the part: up to `want` unassigned vertices in breadth-first order
      // from the seed, within the seed's piece of the unassigned vertices (a
      // part never joins pieces that lie apart: its neighbourhood would not
      // fit)
      std::vector<int> core(1, (int)next_seed);
      owner[next_seed] = np;
      for (size_t h = 0; h < core.size() && (int)core.size() < want; ++h) {
        const int v = core[h];
        for (int k = off[v]; k < off[v + 1] && (int)core.size() < want; ++k) {
          const int u = nbr[k];
          if (owner[u] < 0) {
            owner[u] = np;
            core.push_back(u);
          }
        }
      }
      // its neighbourhood, by distance (stamps are -1 outside an attempt)
      queue.assign(core.begin(), core.end());
      std::vector<int> dl(core.size(), 0);
      for (int v : core) stamp[v] = 1;
      for (size_t h = 0; h < queue.size() && (int)queue.size() <= kMeshLocalMax; ++h) {
        if (dl[h] >= kMeshSteps) continue;
        for (int k = off[queue[h]]; k < off[queue[h] + 1]; ++k) {
          const int u = nbr[k];
          if (stamp[u] != 1) {
            stamp[u] = 1;
            queue.push_back(u);
            dl.push_back(dl[h] + 1);
          }
        }
      }
      if ((int)queue.size() > kMeshLocalMax) {   // too large: a smaller part
        for (int v : core) owner[v] = -1;
        for (int v : queue) stamp[v] = -1;
        want = want * 3 / 4;
        continue;
      }
      const int base = (int)P.lglob.size();
      for (size_t h = 0; h < queue.size(); ++h) lidx[queue[h]] = (int)h;
      for (size_t h = 0; h < queue.size(); ++h) {
        P.lglob.push_back(queue[h]);
        P.ldist.push_back(dl[h]);
        P.ladj_off.push_back((int)P.ladj.size());
        if (dl[h] < kMeshSteps)
          for (int k = off[queue[h]]; k < off[queue[h] + 1]; ++k)
            P.ladj.push_back((unsigned short)lidx[nbr[k]]);
      }
      for (int v : queue) stamp[v] = -1;
      P.part_core.push_back((int)core.size());
      P.part_off.push_back(base + (int)queue.size());
      P.lmax = std::max(P.lmax, (int)queue.size());
      placed = true;
    }
    if (!placed || (long long)P.part_core.size() > parts_cap ||
        (long long)P.lglob.size() > slots_cap || (long long)P.ladj.size() > adj_cap) {
      P.ok = false;
      break;
    }
    ++np;
  }
  P.ladj_off.push_back((int)P.ladj.size());
}

// Adjacency with multiplicity, both directions, neighbours in edge order;
// edges with an endpoint outside [0, V) are left out.
void mesh_adjacency_host(long long V, const int *eh, long long E, std::vector<int> &off,
                         std::vector<int> &nbr) {
  off.assign(V + 1, 0);
  for (long long k = 0; k < E; ++k) {
    const int a = eh[k], b = eh[E + k];
    if (a < 0 || b < 0 || a >= V || b >= V) continue;
    ++off[a + 1];
    ++off[b + 1];
  }
  for (long long v = 0; v < V; ++v) off[v + 1] += off[v];
  nbr.assign(off[V] > 0 ? off[V] : 1, 0);
  std::vector<int> fill(off.begin(), off.end() - 1);
  for (long long k = 0; k < E; ++k) {
    const int a = eh[k], b = eh[E + k];
    if (a < 0 || b < 0 || a >= V || b >= V) continue;
    nbr[fill[a]++] = b;
    nbr[fill[b]++] = a;
  }
}

}  // namespace

struct MeshPlan {
  long long V = 0, E = 0;
  int terms = 0;           // series terms; 1: the identity (L = 0 or lambda = 0)
  int npart = 0;           // 0: one term per launch
  int lmax = 0;            // largest part with its neighbourhood
  MeshDev dev;
  MeshWs w;
};

size_t mesh_precond_bytes(long long V, long long E) {
  Carve c(nullptr);
  mesh_layout(c, V, E);
  return c.off;
}

void mesh_plan_free(MeshPlan *p) { delete p; }   // null: nothing

// Host side: adjacency, coefficients and parts from the edge list (device,
// copied here), uploaded into ws.  Synchronises `st`.
pdg_status mesh_plan_build(long long V, const int *edges, long long E, float lambda,
                           int max_degree, int terms, double tol, void *ws, hipStream_t st,
                           MeshPlan **out) {
  MeshPlan *p = new (std::nothrow) MeshPlan;
  if (!p) {
    set_error("host allocation failed");
    return PDG_ENOMEM;
  }
  p->V = V;
  p->E = E;
  Carve c(ws);
  p->w = mesh_layout(c, V, E);
  MeshWs &w = p->w;
  std::vector<int> eh(2 * E);
  hipError_t e = hipSuccess;
  if (E > 0) {
    e = hipMemcpyAsync(eh.data(), edges, eh.size() * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "mesh plan: edge copy");
  }
  std::vector<int> off, nbr;
  mesh_adjacency_host(V, eh.data(), E, off, nbr);
  int dmax = 0;
  for (long long v = 0; v < V; ++v) dmax = std::max(dmax, off[v + 1] - off[v]);
  if (dmax > max_degree) {
    delete p;
    set_error("mesh plan: a vertex has degree %d above max_degree %d", dmax, max_degree);
    return PDG_EINVAL;
  }
  const double lam = lambda, kappa = 1.0 + 2.0 * lam * (double)max_degree;
  std::vector<double> coef;
  if (lam == 0.0 || max_degree == 0 || off[V] == 0) {
    p->terms = 1;                           // (I + lambda L) = I
    coef.assign(1, 1.0);
  } else {
    p->terms = mesh_coefficients(kappa, tol, terms, coef);
    if (p->terms == 0) {
      delete p;
      set_error("mesh plan: the series needs more than %d terms (raise tol)", kMeshMaxTerms);
      return PDG_EINVAL;
    }
  }
  MeshDev &d = p->dev;
  d.V = V;
  d.lam = lam;
  d.b1 = kappa > 1.0 ? 2.0 / (kappa - 1.0) : 0.0;
  d.b0 = kappa > 1.0 ? -(kappa + 1.0) / (kappa - 1.0) : 0.0;
  d.coef = w.coef;
  d.off = w.off;
  d.nbr = w.nbr;
  d.part_off = w.part_off;
  d.part_core = w.part_core;
  d.lglob = w.lglob;
  d.ldist = w.ldist;
  d.ladj_off = w.ladj_off;
  d.ladj = w.ladj;
  MeshParts parts;
  if (p->terms > 1) mesh_partition(V, off, nbr, w.parts, w.slots, w.adj_slots, parts);
  p->npart = parts.ok ? (int)parts.part_core.size() : 0;
  p->lmax = parts.ok ? parts.lmax : 0;
  std::vector<int> &part_off = parts.part_off, &part_core = parts.part_core,
                   &lglob = parts.lglob, &ldist = parts.ldist, &ladj_off = parts.ladj_off;
  std::vector<unsigned short> &ladj = parts.ladj;
  auto up = [&](void *dst, const void *src, size_t bytes) {
    if (e == hipSuccess && bytes > 0) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
  };
  up(w.off, off.data(), off.size() * sizeof(int));
  up(w.nbr, nbr.data(), nbr.size() * sizeof(int));
  up(w.coef, coef.data(), (size_t)p->terms * sizeof(double));
  if (p->npart > 0) {
    up(w.part_off, part_off.data(), part_off.size() * sizeof(int));
    up(w.part_core, part_core.data(), part_core.size() * sizeof(int));
    up(w.lglob, lglob.data(), lglob.size() * sizeof(int));
    up(w.ldist, ldist.data(), ldist.size() * sizeof(int));
    up(w.ladj_off, ladj_off.data(), ladj_off.size() * sizeof(int));
    up(w.ladj, ladj.data(), ladj.size() * sizeof(unsigned short));
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host vectors go out of scope
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "mesh plan: upload");
  }
  *out = p;
  return PDG_OK;
}

pdg_status mesh_plan_apply(const MeshPlan &p, const float *g, float *out, hipStream_t st) {
  const long long V = p.V, n = 3 * V;
  if (V == 0) return PDG_OK;
  if (p.terms == 1) return launch_copy(out, g, n, st);   // the identity, exactly
  const MeshWs &w = p.w;
  const MeshDev &d = p.dev;
  mesh_init_kernel<<<div_up(n, 256), 256, 0, st>>>(d, g, w.vec[0], w.y);
  PDG_TRY(launched("mesh_init"));
  const int steps = p.terms - 1;              // v_1 .. v_{terms-1}
  if (p.npart > 0) {
    const size_t lds = (size_t)2 * 3 * p.lmax * sizeof(double);
    static PerDevice attr;
    int dev = 0;
    PDG_TRY_HIP(hipGetDevice(&dev));
    if (!attr.done(dev)) {
      PDG_TRY_HIP(hipFuncSetAttribute((const void *)mesh_block_kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)(2 * 3 * kMeshLocalMax * sizeof(double))));
      attr.mark(dev);
    }
    // (cur, prev) in vec[0], vec[1]; the launch writes vec[2], vec[3]; swap
    const double *cur = w.vec[0], *prev = w.vec[1];
    double *ncur = w.vec[2], *nprev = w.vec[3];
    for (int j0 = 0; j0 < steps; j0 += kMeshSteps) {
      const int ks = steps - j0 < kMeshSteps ? steps - j0 : kMeshSteps;
      const bool last = j0 + ks == steps;
      mesh_block_kernel<<<p.npart, kMeshThreads, lds, st>>>(d, j0, ks, cur, prev, ncur, nprev,
                                                           w.y, last ? out : nullptr);
      PDG_TRY(launched("mesh_block"));
      const double *t0 = cur, *t1 = prev;
      cur = ncur;
      prev = nprev;
      ncur = const_cast<double *>(t0);
      nprev = const_cast<double *>(t1);
    }
    return PDG_OK;
  }
  // one term per launch: v_{j-1}, v_j, v_{j+1} rotate through three buffers
  double *b[3] = {w.vec[1], w.vec[0], w.vec[2]};   // prev, cur, next
  for (int j = 0; j < steps; ++j) {
    mesh_term_kernel<<<div_up(V, 256), 256, 0, st>>>(d, j, b[1], b[0], b[2], w.y);
    PDG_TRY(launched("mesh_term"));
    double *t = b[0];
    b[0] = b[1];
    b[1] = b[2];
    b[2] = t;
  }
  mesh_out_kernel<<<div_up(n, 256), 256, 0, st>>>(w.y, n, out);
  return launched("mesh_out");
}

pdg_status mesh_partition_query(long long V, const int *edges_host, long long E, int *part_off,
                                int *part_core, int *lglob, int *ldist, long long *sizes) {
  std::vector<int> off, nbr;
  mesh_adjacency_host(V, edges_host, E, off, nbr);
  Carve c(nullptr);
  const MeshWs w = mesh_layout(c, V, E);
  MeshParts P;
  mesh_partition(V, off, nbr, w.parts, w.slots, w.adj_slots, P);
  const long long np = P.ok ? (long long)P.part_core.size() : 0;
  sizes[0] = np;
  sizes[1] = P.ok ? (long long)P.lglob.size() : 0;
  sizes[2] = kMeshSteps;
  sizes[3] = kMeshLocalMax;
  if (np > 0) {
    if (part_off) std::copy(P.part_off.begin(), P.part_off.end(), part_off);
    if (part_core) std::copy(P.part_core.begin(), P.part_core.end(), part_core);
    if (lglob) std::copy(P.lglob.begin(), P.lglob.end(), lglob);
    if (ldist) std::copy(P.ldist.begin(), P.ldist.end(), ldist);
  }
  return PDG_OK;
}

int mesh_plan_terms(const MeshPlan &p) { return p.terms; }
long long mesh_plan_vertices(const MeshPlan &p) { return p.V; }
int mesh_plan_parts(const MeshPlan &p) { return p.npart; }

}  // namespace pdg
