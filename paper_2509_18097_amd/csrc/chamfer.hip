// Robust Chamfer distance (paper Sec. 3.4, Eq. 11-13): exact float32
// nearest-neighbour tiles, float64 loss reduction and the adjoint.
//
// Neighbour contract (shared with every mode of the library): the squared
// distance is evaluated in float32 in difference form without fused
// multiply-add, d2 = (dx*dx + dy*dy) + dz*dz with dx = q_x - c_x, and the
// lowest index wins ties.  Candidates are scanned in increasing index order
// with a strict comparison, which realises the tie rule.
#include "common.h"

namespace pdg {
namespace {

constexpr int kNNThreads = 256;
constexpr int kQPT = 4;                       // queries per thread
constexpr int kQTile = kNNThreads * kQPT;     // queries per workgroup
constexpr int kCTile = 1024;                  // candidates staged in LDS per round

__device__ __forceinline__ float d2_contract(float qx, float qy, float qz, float cx, float cy,
                                             float cz) {
#pragma clang fp contract(off)
  const float dx = qx - cx;
  const float dy = qy - cy;
  const float dz = qz - cz;
  return (dx * dx + dy * dy) + dz * dz;
}

__global__ __launch_bounds__(kNNThreads) void nn_exact_kernel(const NNJob *__restrict__ jobs) {
  const NNJob J = jobs[blockIdx.y];
  const int q0 = blockIdx.x * kQTile;
  if (q0 >= J.nq) return;
  __shared__ float4 sc[kCTile];
  const int tid = threadIdx.x;
  float qx[kQPT], qy[kQPT], qz[kQPT], best[kQPT];
  int bi[kQPT];
#pragma unroll
  for (int k = 0; k < kQPT; ++k) {
    const int qi = q0 + k * kNNThreads + tid;
    const bool ok = qi < J.nq;
    qx[k] = ok ? J.q[qi] : 0.f;
    qy[k] = ok ? J.q[(long long)J.nq + qi] : 0.f;
    qz[k] = ok ? J.q[2ll * J.nq + qi] : 0.f;
    best[k] = __builtin_huge_valf();
    bi[k] = 0;
  }
  const long long nc = J.nc;
  for (int c0 = 0; c0 < J.nc; c0 += kCTile) {
    const int cnt = (J.nc - c0) < kCTile ? (J.nc - c0) : kCTile;
    __syncthreads();
    for (int j = tid; j < cnt; j += kNNThreads)
      sc[j] = make_float4(J.c[c0 + j], J.c[nc + c0 + j], J.c[2 * nc + c0 + j], 0.f);
    __syncthreads();
    int j = 0;
    for (; j + 4 <= cnt; j += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float4 p = sc[j + u];
#pragma unroll
        for (int k = 0; k < kQPT; ++k) {
          const float d = d2_contract(qx[k], qy[k], qz[k], p.x, p.y, p.z);
          if (d < best[k]) {
            best[k] = d;
            bi[k] = c0 + j + u;
          }
        }
      }
    }
    for (; j < cnt; ++j) {
      const float4 p = sc[j];
#pragma unroll
      for (int k = 0; k < kQPT; ++k) {
        const float d = d2_contract(qx[k], qy[k], qz[k], p.x, p.y, p.z);
        if (d < best[k]) {
          best[k] = d;
          bi[k] = c0 + j;
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kQPT; ++k) {
    const int qi = q0 + k * kNNThreads + tid;
    if (qi < J.nq) J.nn[qi] = bi[k];
  }
}

__device__ __forceinline__ double block_sum_f64(double v, double *sh) {
  // fixed-order reduction: butterfly inside each wave, then waves in order
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(256) void chamfer_loss_kernel(const ChSeg *__restrict__ segs,
                                                           double alpha,
                                                           double *__restrict__ partials) {
  __shared__ double sh[4];
  const ChSeg S = segs[blockIdx.y];
  const int dir = blockIdx.z;
  const float *q = dir == 0 ? S.a : S.b;
  const float *c = dir == 0 ? S.b : S.a;
  const int nq = dir == 0 ? S.n : S.m;
  const long long nc = dir == 0 ? S.m : S.n;
  const int *nn = dir == 0 ? S.nn_a : S.nn_b;
  double acc = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nq; i += kLossBlocks * 256) {
    const int j = nn[i];
    const double dx = (double)q[i] - (double)c[j];
    const double dy = (double)q[nq + i] - (double)c[nc + j];
    const double dz = (double)q[2ll * nq + i] - (double)c[2 * nc + j];
    const double s = dx * dx + dy * dy + dz * dz;
    acc += exp(-alpha * s) * s;
  }
  double t = block_sum_f64(acc, sh);
  if (threadIdx.x == 0)
    partials[((long long)blockIdx.y * 2 + dir) * kLossBlocks + blockIdx.x] = t;
}

__global__ void chamfer_loss_final_kernel(const ChSeg *__restrict__ segs, int nseg,
                                          const double *__restrict__ partials,
                                          double *__restrict__ losses) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 2 * nseg) return;
  double t = 0.0;
  for (int b = 0; b < kLossBlocks; ++b) t += partials[(long long)k * kLossBlocks + b];
  const ChSeg S = segs[k >> 1];
  losses[k] = t / (double)((k & 1) ? S.m : S.n);
}

__global__ __launch_bounds__(256) void chamfer_grad_fwd_kernel(const ChSeg *__restrict__ segs,
                                                               float alpha,
                                                               const double *__restrict__ w) {
  const int seg = blockIdx.y;
  const ChSeg S = segs[seg];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= S.n || S.ga == nullptr) return;
  const long long m = S.m, n = S.n;
  const int j = S.nn_a[i];
  const float dx = S.a[i] - S.b[j];
  const float dy = S.a[n + i] - S.b[m + j];
  const float dz = S.a[2 * n + i] - S.b[2 * m + j];
  const float s = dx * dx + dy * dy + dz * dz;
  const float coef = (float)(w[2 * seg] / (double)S.n) * expf(-alpha * s) * (1.0f - alpha * s) * 2.0f;
  S.ga[i] = coef * dx;
  S.ga[n + i] = coef * dy;
  S.ga[2 * n + i] = coef * dz;
}

__global__ __launch_bounds__(256) void chamfer_rev_keys_kernel(const ChSeg *__restrict__ segs,
                                                               const unsigned *__restrict__ b_base,
                                                               uint32_t *__restrict__ keys,
                                                               uint32_t *__restrict__ vals) {
  const int seg = blockIdx.y;
  const ChSeg S = segs[seg];
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= S.m) return;
  const unsigned g = b_base[seg] + (unsigned)j;
  keys[g] = S.a_base + (unsigned)S.nn_b[j];
  vals[g] = g;
}

__global__ __launch_bounds__(256) void chamfer_rev_scatter_kernel(
    const ChSeg *__restrict__ segs, int nseg, const unsigned *__restrict__ b_base,
    const uint32_t *__restrict__ keys, const uint32_t *__restrict__ vals, long long nent,
    float alpha, const double *__restrict__ w) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nent) return;
  const uint32_t key = keys[i];
  if (i > 0 && keys[i - 1] == key) return;
  // segment of this run: the b index determines it (b_base is increasing)
  const unsigned g0 = vals[i];
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b_base[mid] <= g0) lo = mid; else hi = mid - 1;
  }
  const ChSeg S = segs[lo];
  if (S.ga == nullptr) return;
  const long long n = S.n, m = S.m;
  const int ai = (int)(key - S.a_base);
  const float ax = S.a[ai], ay = S.a[n + ai], az = S.a[2 * n + ai];
  const float cw = (float)(w[2 * lo + 1] / (double)S.m);
  float s0 = 0.f, s1 = 0.f, s2 = 0.f;
  for (long long k = i; k < nent && keys[k] == key; ++k) {
    const int j = (int)(vals[k] - b_base[lo]);
    const float dx = ax - S.b[j];
    const float dy = ay - S.b[m + j];
    const float dz = az - S.b[2 * m + j];
    const float s = dx * dx + dy * dy + dz * dz;
    const float coef = cw * expf(-alpha * s) * (1.0f - alpha * s) * 2.0f;
    s0 += coef * dx;
    s1 += coef * dy;
    s2 += coef * dz;
  }
  S.ga[ai] += s0;
  S.ga[n + ai] += s1;
  S.ga[2 * n + ai] += s2;
}

}  // namespace

pdg_status launch_nn_exact(const NNJob *jobs, int njobs, int max_nq, hipStream_t st) {
  if (njobs <= 0 || max_nq <= 0) return PDG_OK;
  dim3 grid(div_up(max_nq, kQTile), njobs);
  nn_exact_kernel<<<grid, kNNThreads, 0, st>>>(jobs);
  return launched("nn_exact");
}

pdg_status launch_chamfer_loss(const ChSeg *segs, int nseg, double alpha, double *partials,
                               double *losses, hipStream_t st) {
  if (nseg <= 0) return PDG_OK;
  dim3 grid(kLossBlocks, nseg, 2);
  chamfer_loss_kernel<<<grid, 256, 0, st>>>(segs, alpha, partials);
  PDG_TRY(launched("chamfer_loss"));
  chamfer_loss_final_kernel<<<div_up(2 * nseg, 64), 64, 0, st>>>(segs, nseg, partials, losses);
  return launched("chamfer_loss_final");
}

pdg_status launch_chamfer_grad_fwd(const ChSeg *segs, int nseg, int max_n, float alpha,
                                   const double *w, hipStream_t st) {
  if (nseg <= 0 || max_n <= 0) return PDG_OK;
  dim3 grid(div_up(max_n, 256), nseg);
  chamfer_grad_fwd_kernel<<<grid, 256, 0, st>>>(segs, alpha, w);
  return launched("chamfer_grad_fwd");
}

pdg_status launch_chamfer_rev_keys(const ChSeg *segs, int nseg, int max_m, const unsigned *b_base,
                                   uint32_t *keys, uint32_t *vals, hipStream_t st) {
  if (nseg <= 0 || max_m <= 0) return PDG_OK;
  dim3 grid(div_up(max_m, 256), nseg);
  chamfer_rev_keys_kernel<<<grid, 256, 0, st>>>(segs, b_base, keys, vals);
  return launched("chamfer_rev_keys");
}

pdg_status launch_chamfer_rev_scatter(const ChSeg *segs, int nseg, const unsigned *b_base,
                                      const unsigned * /*unused*/, const uint32_t *keys,
                                      const uint32_t *vals, long long nent, float alpha,
                                      const double *w, hipStream_t st) {
  if (nent <= 0) return PDG_OK;
  chamfer_rev_scatter_kernel<<<div_up(nent, 256), 256, 0, st>>>(segs, nseg, b_base, keys, vals,
                                                                nent, alpha, w);
  return launched("chamfer_rev_scatter");
}

}  // namespace pdg
