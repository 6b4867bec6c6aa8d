// Adam (paper Sec. 3.6), the isometry loss (Eq. 18) with its adjoint, and
// the loss assembly with confidence weights (Eq. 9, 14-17).
#include "common.h"

namespace pdg {
namespace {

__device__ __forceinline__ int level_of(const AdamLevels &lv, long long w) {
  int l = 0;
  while (l + 1 < lv.levels && w >= lv.off[l + 1]) ++l;
  return l;
}

// Kept bit of value w of stack b (pruned grids; 1 without a mask).
__device__ __forceinline__ unsigned kept_of(const AdamLevels &lv, long long b, long long w) {
  if (!lv.mask) return 1u;
  const int l = level_of(lv, w);
  const long long cell = (w - lv.off[l]) % lv.r3[l];
  return (lv.mask[b * lv.mstack + lv.moff[l] + (cell >> 5)] >> (cell & 31)) & 1u;
}

// Whether any of values w .. w + 3 (w % 4 == 0) is kept: one lookup when the
// four lie in one level's channel block (its offset and R^3 multiples of 4,
// so they share a mask word), else one per value.
__device__ __forceinline__ bool kept_any4(const AdamLevels &lv, long long b, long long w) {
  if (!lv.mask) return true;
  const int l = level_of(lv, w);
  if (w + 3 < lv.off[l + 1] && (lv.off[l] & 3) == 0 && (lv.r3[l] & 3) == 0 &&
      lv.r3[l] < (1ll << 32)) {
    const unsigned cell = (unsigned)(w - lv.off[l]) % (unsigned)lv.r3[l];
    return ((lv.mask[b * lv.mstack + lv.moff[l] + (cell >> 5)] >> (cell & 31)) & 15u) != 0u;
  }
  return (kept_of(lv, b, w) | kept_of(lv, b, w + 1) | kept_of(lv, b, w + 2) |
          kept_of(lv, b, w + 3)) != 0u;
}

// Adam's streams are read or written once: past the caches (non-temporal
// accesses)
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 nt_load4(const float *p) {
  const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void nt_store4(float *p, float4 x) {
  const nt_f4 v = {x.x, x.y, x.z, x.w};
  __builtin_nontemporal_store(v, reinterpret_cast<nt_f4 *>(p));
}

// kAdamGroups groups of four consecutive values of stack blockIdx.y per thread (all
// loads issued before the arithmetic); stack % 4 == 0 and 16-byte aligned arrays.
constexpr int kAdamGroups = 1;
__global__ __launch_bounds__(256) void adam4_kernel(AdamLevels lv, long long stack, long long c0,
                                                    long long c1, float b1, float b2, float eps,
                                                    const int *__restrict__ step_dev, int step_host,
                                                    float *__restrict__ th, float *__restrict__ m,
                                                    float *__restrict__ v,
                                                    const float *__restrict__ g) {
  __shared__ float sbc[2];
  adam_bias(b1, b2, step_dev, step_host, sbc);
  const float bc1 = sbc[0], bc2 = sbc[1];
  const long long w0 = c0 + (long long)blockIdx.x * blockDim.x * 4 * kAdamGroups + threadIdx.x * 4;
  const long long base = (long long)blockIdx.y * stack;
  float4 gi[kAdamGroups], mi[kAdamGroups], vi[kAdamGroups], ti[kAdamGroups];
  bool live[kAdamGroups];
#pragma unroll
  for (int q = 0; q < kAdamGroups; ++q) {
    const long long w = w0 + (long long)q * blockDim.x * 4;
    // a group of four pruned values is left as it is (no loads, no stores)
    live[q] = w < c1 && kept_any4(lv, blockIdx.y, w);
    if (live[q]) {
      gi[q] = nt_load4(g + base + w);
      mi[q] = nt_load4(m + base + w);
      vi[q] = nt_load4(v + base + w);
      ti[q] = nt_load4(th + base + w);
    }
  }
#pragma unroll
  for (int q = 0; q < kAdamGroups; ++q) {
    const long long w = w0 + (long long)q * blockDim.x * 4;
    if (!live[q]) continue;
    ti[q].x = adam_one(b1, b2, eps, lv.lr[level_of(lv, w)], bc1, bc2, gi[q].x, mi[q].x, vi[q].x, ti[q].x);
    ti[q].y = adam_one(b1, b2, eps, lv.lr[level_of(lv, w + 1)], bc1, bc2, gi[q].y, mi[q].y, vi[q].y, ti[q].y);
    ti[q].z = adam_one(b1, b2, eps, lv.lr[level_of(lv, w + 2)], bc1, bc2, gi[q].z, mi[q].z, vi[q].z, ti[q].z);
    ti[q].w = adam_one(b1, b2, eps, lv.lr[level_of(lv, w + 3)], bc1, bc2, gi[q].w, mi[q].w, vi[q].w, ti[q].w);
    nt_store4(m + base + w, mi[q]);
    nt_store4(v + base + w, vi[q]);
    nt_store4(th + base + w, ti[q]);
  }
}

// One value per thread (any layout).
__global__ __launch_bounds__(256) void adam_kernel(AdamLevels lv, long long stack, long long c0,
                                                   long long c1, float b1, float b2, float eps,
                                                   const int *__restrict__ step_dev, int step_host,
                                                   float *__restrict__ th, float *__restrict__ m,
                                                   float *__restrict__ v,
                                                   const float *__restrict__ g) {
  __shared__ float sbc[2];
  adam_bias(b1, b2, step_dev, step_host, sbc);
  const long long w = c0 + (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= c1 || !kept_of(lv, blockIdx.y, w)) return;   // pruned values stay as they are
  const long long i = (long long)blockIdx.y * stack + w;
  float mi = m[i], vi = v[i];
  th[i] = adam_one(b1, b2, eps, lv.lr[level_of(lv, w)], sbc[0], sbc[1], g[i], mi, vi, th[i]);
  m[i] = mi;
  v[i] = vi;
}

__global__ void set_int_kernel(int *p, int v) { *p = v; }

__device__ __forceinline__ double block_sum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  return t;
}

// Per (frame t = 1..T, edge e): sign of the length change and the unit edge
// vector at t; float64 partial sums of |l_t - l_{t-1}|.
__global__ __launch_bounds__(256) void iso_edge_kernel(IsoArgs a) {
#pragma clang fp contract(off)
  __shared__ double sh[4];
  const long long total = (long long)a.T * a.E;
  const long long V = a.V, E = a.E;
  double acc = 0.0;
  for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < total;
       k += (long long)gridDim.x * 256) {
    const int t = (int)(k / E) + 1;
    const int e = (int)(k % E);
    const int i = a.edges[e], j = a.edges[E + e];
    const float *xc = a.xhat + (long long)t * 3 * V;
    const float *xp = xc - 3 * V;
    const double cx = (double)xc[i] - (double)xc[j];
    const double cy = (double)xc[V + i] - (double)xc[V + j];
    const double cz = (double)xc[2 * V + i] - (double)xc[2 * V + j];
    const double px = (double)xp[i] - (double)xp[j];
    const double py = (double)xp[V + i] - (double)xp[V + j];
    const double pz = (double)xp[2 * V + i] - (double)xp[2 * V + j];
    const double lc = sqrt((cx * cx + cy * cy) + cz * cz);
    const double lp = sqrt((px * px + py * py) + pz * pz);
    const double d = lc - lp;
    acc += fabs(d);
    const long long o = (long long)(t - 1) * E + e;
    a.sig[o] = d > 0.0 ? 1.0f : (d < 0.0 ? -1.0f : 0.0f);
    const double inv = lc > 0.0 ? 1.0 / lc : 0.0;
    const long long ou = (long long)(t - 1) * 3 * E + e;
    a.u[ou] = (float)(cx * inv);
    a.u[ou + E] = (float)(cy * inv);
    a.u[ou + 2 * E] = (float)(cz * inv);
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) a.partials[blockIdx.x] = t;
}

// Per (frame t = 1..T, vertex v): gather over the incident edges (sorted by
// edge id) coef * (sig_t - sig_{t+1}) * (+-u_t) and add to the direct
// gradient of X_t.
__global__ __launch_bounds__(256) void iso_vertex_kernel(IsoArgs a) {
  const long long V = a.V, E = a.E;
  const long long k = (long long)blockIdx.x * 256 + threadIdx.x;
  if (k >= (long long)a.T * V) return;
  const int t = (int)(k / V) + 1;
  const int v = (int)(k % V);
  const float coef = (float)a.coef;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f;
  for (int q = a.inc_off[v]; q < a.inc_off[v + 1]; ++q) {
    const uint32_t code = a.inc[q];
    const int e = (int)(code >> 1);
    const float side = (code & 1u) ? -1.0f : 1.0f;
    float s = a.sig[(long long)(t - 1) * E + e];
    if (t < a.T) s -= a.sig[(long long)t * E + e];
    if (s == 0.0f) continue;
    const long long ou = (long long)(t - 1) * 3 * E + e;
    const float c = coef * s * side;
    s0 += c * a.u[ou];
    s1 += c * a.u[ou + E];
    s2 += c * a.u[ou + 2 * E];
  }
  float *gx = a.gx + (long long)(t - 1) * 3 * V;
  gx[v] += s0;
  gx[V + v] += s1;
  gx[2 * V + v] += s2;
}

__global__ void incidence_keys_kernel(const int *__restrict__ edges, int E, uint32_t *keys,
                                      uint32_t *vals) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  keys[2 * e] = (uint32_t)edges[e];
  vals[2 * e] = 2u * e;
  keys[2 * e + 1] = (uint32_t)edges[E + e];
  vals[2 * e + 1] = 2u * e + 1u;
}

__global__ void incidence_off_kernel(const uint32_t *__restrict__ keys, int n2, int V,
                                     int *__restrict__ off) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v > V) return;
  int lo = 0, hi = n2;  // first position with key >= v
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (keys[mid] < (uint32_t)v) lo = mid + 1; else hi = mid;
  }
  off[v] = lo;
}

// Lane-strided partials summed in lane order (the result on lane 0).
__device__ __forceinline__ double lane_ordered_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < 64; ++i) s += sh[i];
  __syncthreads();
  return s;
}

// One wave: the loads and the confidence factors lane-parallel, the
// cumulative product and the sums in a fixed order.
__global__ __launch_bounds__(64) void assemble_kernel(AssembleArgs a) {
  __shared__ double sh[64], fac[64], cc[64];
  const int lane = threadIdx.x;
  const int E = a.E, T = a.T, Tn = a.Tn;
  double cm = -1.0, sp = 0.0;
  for (int t = lane; t < T; t += 64) {
    const double c = a.losses[2 * t] + a.losses[2 * t + 1];
    cm = c > cm ? c : cm;
    sp += c;
    a.w[2 * t] = 1.0 / Tn;
    a.w[2 * t + 1] = 1.0 / Tn;
  }
  for (int t = lane; t < a.partner_T; t += 64) {   // the other chain's point terms (Eq. 17)
    const double c = a.partner_losses[2 * t] + a.partner_losses[2 * t + 1];
    cm = c > cm ? c : cm;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double u = __shfl_xor(cm, o, 64);
    cm = u > cm ? u : cm;
  }
  const double cd_max = cm;
  const double sum_pt = lane_ordered_sum(sp, sh);
  const int e = *a.epoch;
  const double delta = 1.0 - sqrt((double)e / (double)a.e_max);
  double wc = 1.0, sum_tm = 0.0, l_iso = 0.0;
  if (a.has_tm) {
    for (int t0 = 0; t0 < T; t0 += 64) {
      const int t = t0 + lane;
      if (t < T) {
        const double c = a.losses[2 * (T + t)] + a.losses[2 * (T + t) + 1];
        const double ex = c - cd_max > 0.0 ? c - cd_max : 0.0;
        fac[lane] = pow(1.0 / (1.0 + ex), delta);
        cc[lane] = c;
      }
      __syncthreads();
      if (lane == 0) {
        const int n = T - t0 < 64 ? T - t0 : 64;
        for (int j = 0; j < n; ++j) {
          wc *= fac[j];
          a.wconf[t0 + j] = wc;
          sum_tm += wc * cc[j];
        }
      }
      __syncthreads();
    }
    // Gradient weight of each template term: w_conf(tau) itself plus the
    // change of every later weight through factor tau (Eq. 15), cd_max held
    // constant (Eq. 17): when CD_tau > cd_max,
    //   - delta / (1 + CD_tau - cd_max) * sum_{t >= tau} w_conf(t) CD_t.
    if (lane == 0) {
      double later = 0.0;
      for (int t = T - 1; t >= 0; --t) {
        const double c = a.losses[2 * (T + t)] + a.losses[2 * (T + t) + 1];
        const double w = a.wconf[t];
        later += w * c;
        const double g = c - cd_max > 0.0 ? w - delta / (1.0 + (c - cd_max)) * later : w;
        a.w[2 * (T + t)] = g / Tn;
        a.w[2 * (T + t) + 1] = g / Tn;
      }
    }
    if (E > 0) {
      double s = 0.0;
      for (int b = lane; b < kIsoBlocks; b += 64) s += a.iso_partials[b];
      s = lane_ordered_sum(s, sh);
      l_iso = (double)a.w_iso * s / ((double)Tn * (double)E);
    }
  } else {
    for (int t = lane; t < T; t += 64) a.wconf[t] = 1.0;
  }
  if (lane != 0) return;
  const double l_tr = (sum_tm + sum_pt) / Tn;
  double terms[kTerms] = {l_tr + l_iso, l_tr, l_iso, cd_max, sum_pt / Tn, sum_tm / Tn, wc,
                          (double)e, 0.0};
  for (int i = 0; i < kTerms; ++i) {
    a.terms[i] = terms[i];
    if (a.user_terms) a.user_terms[i] = terms[i];
  }
}

__global__ void joint_terms_kernel(const double *tb, const double *tf, double *out,
                                   double *user) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double *last = tf ? tf : tb;
  double t[kTerms];
  for (int i = 0; i < kTerms; ++i) t[i] = (tb ? tb[i] : 0.0) + (tf ? tf[i] : 0.0);
  t[3] = last[3];   // cd_max: the same in both chains
  t[6] = last[6];
  t[7] = last[7];
  for (int i = 0; i < kTerms; ++i) {
    out[i] = t[i];
    if (user) user[i] = t[i];
  }
}

__global__ void mesh_terms_kernel(double *terms, double *user, const double *loss0) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double lm = loss0[0] + loss0[1];
  terms[8] = lm;
  terms[0] = terms[1] + terms[2] + lm;
  if (user) {
    user[8] = lm;
    user[0] = terms[0];
  }
}

}  // namespace

pdg_status launch_joint_terms(const double *tb, const double *tf, double *out, double *user,
                              hipStream_t st) {
  joint_terms_kernel<<<1, 64, 0, st>>>(tb, tf, out, user);
  return launched("joint_terms");
}

pdg_status launch_mesh_terms(double *terms, double *user, const double *loss0, hipStream_t st) {
  mesh_terms_kernel<<<1, 64, 0, st>>>(terms, user, loss0);
  return launched("mesh_terms");
}

namespace {
// Adam over columns [c0, c1) of every stack.
pdg_status adam_cols(const AdamLevels &lv, long long stack, long long c0, long long c1, int batch,
                     float b1, float b2, float eps, const int *step_dev, int step_host,
                     float *theta, float *m, float *v, const float *g, hipStream_t st) {
  if (c1 <= c0 || batch <= 0) return PDG_OK;
  const bool vec = stack % 4 == 0 && c0 % 4 == 0 && c1 % 4 == 0 &&
                   ((uintptr_t)theta | (uintptr_t)m | (uintptr_t)v | (uintptr_t)g) % 16 == 0;
  const long long cols = c1 - c0;
  for (int b0 = 0; b0 < batch; b0 += 65535) {      // grid.y limit
    const int nb = batch - b0 < 65535 ? batch - b0 : 65535;
    const long long o = (long long)b0 * stack;
    AdamLevels lb = lv;                 // this chunk's stacks' mask words
    if (lb.mask) lb.mask += (long long)b0 * lb.mstack;
    if (vec) {
      dim3 grid(div_up(cols / 4, 256 * kAdamGroups), nb);
      adam4_kernel<<<grid, 256, 0, st>>>(lb, stack, c0, c1, b1, b2, eps, step_dev, step_host,
                                         theta + o, m + o, v + o, g + o);
    } else {
      dim3 grid(div_up(cols, 256), nb);
      adam_kernel<<<grid, 256, 0, st>>>(lb, stack, c0, c1, b1, b2, eps, step_dev, step_host,
                                        theta + o, m + o, v + o, g + o);
    }
    PDG_TRY(launched("adam"));
  }
  return PDG_OK;
}
}  // namespace

pdg_status launch_adam(const AdamLevels &lv, long long stack, int batch, float b1, float b2,
                       float eps, const int *step_dev, int step_host, float *theta, float *m,
                       float *v, const float *g, hipStream_t st) {
  if (stack <= 0 || batch <= 0) return PDG_OK;
  return adam_cols(lv, stack, 0, stack, batch, b1, b2, eps, step_dev, step_host, theta, m, v, g,
                   st);
}

pdg_status launch_adam_levels(const AdamLevels &lv, unsigned skip, long long stack, int batch,
                              float b1, float b2, float eps, const int *step_dev, int step_host,
                              float *theta, float *m, float *v, const float *g, hipStream_t st) {
  // one launch per maximal run of levels that are not skipped
  for (int l = 0; l < lv.levels;) {
    if ((skip >> l) & 1u) {
      ++l;
      continue;
    }
    int e = l;
    while (e < lv.levels && !((skip >> e) & 1u)) ++e;
    PDG_TRY(adam_cols(lv, stack, lv.off[l], lv.off[e], batch, b1, b2, eps, step_dev, step_host,
                      theta, m, v, g, st));
    l = e;
  }
  return PDG_OK;
}

pdg_status launch_set_int(int *p, int value, hipStream_t st) {
  set_int_kernel<<<1, 1, 0, st>>>(p, value);
  return launched("set_int");
}

pdg_status launch_iso_edges(const IsoArgs &a, hipStream_t st) {
  if (a.T <= 0 || a.E <= 0) return PDG_OK;
  iso_edge_kernel<<<kIsoBlocks, 256, 0, st>>>(a);
  return launched("iso_edge");
}

pdg_status launch_iso_vertices(const IsoArgs &a, hipStream_t st) {
  if (a.T <= 0 || a.E <= 0 || a.V <= 0) return PDG_OK;
  iso_vertex_kernel<<<div_up((long long)a.T * a.V, 256), 256, 0, st>>>(a);
  return launched("iso_vertex");
}

pdg_status launch_incidence(const int *edges, int E, int V, uint32_t *keys, uint32_t *vals,
                            int *inc_off, void *sort_scratch, hipStream_t st) {
  if (E > 0) {
    incidence_keys_kernel<<<div_up(E, 256), 256, 0, st>>>(edges, E, keys, vals);
    PDG_TRY(launched("incidence_keys"));
    int bits = 1;
    while ((1ll << bits) <= (long long)V) ++bits;
    PDG_TRY(radix_sort(keys, vals, 2ll * E, bits, sort_scratch, st));
  }
  incidence_off_kernel<<<div_up(V + 1, 256), 256, 0, st>>>(keys, 2 * E, V, inc_off);
  return launched("incidence_off");
}

pdg_status launch_assemble(const AssembleArgs &a, hipStream_t st) {
  assemble_kernel<<<1, 64, 0, st>>>(a);
  return launched("assemble");
}

}  // namespace pdg
