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
  const PDG_GLOBAL float *jq = glb(J.q), *jc = glb(J.c);
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
    qx[k] = ok ? jq[qi] : 0.f;
    qy[k] = ok ? jq[(long long)J.nq + qi] : 0.f;
    qz[k] = ok ? jq[2ll * J.nq + qi] : 0.f;
    best[k] = __builtin_huge_valf();
    bi[k] = 0;
  }
  const long long nc = J.nc;
  for (int c0 = 0; c0 < J.nc; c0 += kCTile) {
    const int cnt = (J.nc - c0) < kCTile ? (J.nc - c0) : kCTile;
    __syncthreads();
    for (int j = tid; j < cnt; j += kNNThreads)
      sc[j] = make_float4(jc[c0 + j], jc[nc + c0 + j], jc[2 * nc + c0 + j], 0.f);
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
    if (qi < J.nq) glb(J.nn)[qi] = bi[k];
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

// The kLossBlocks workgroups of one (segment, direction) job run on one XCD
// (job_block), so its L2 holds the job's candidate set once.
__global__ __launch_bounds__(256) void chamfer_loss_kernel(const ChSeg *__restrict__ segs,
                                                           int njobs, double alpha) {
  __shared__ double sh[4];
  unsigned job, blk;
  if (!job_block(blockIdx.x, (unsigned)njobs, kLossBlocks, job, blk)) return;
  const int seg = (int)job >> 1;
  const ChSeg S = segs[seg];
  const int dir = (int)job & 1;
  const PDG_GLOBAL float *q = glb(dir == 0 ? S.a : S.b);
  const PDG_GLOBAL float *c = glb(dir == 0 ? S.b : S.a);
  const int nq = dir == 0 ? S.n : S.m;
  const long long nc = dir == 0 ? S.m : S.n;
  const PDG_GLOBAL int *nn = glb(dir == 0 ? S.nn_a : S.nn_b);
  double acc = 0.0;
  for (int i = (int)blk * 256 + threadIdx.x; i < nq; i += kLossBlocks * 256) {
    const int j = nn[i];
    const double dx = (double)q[i] - (double)c[j];
    const double dy = (double)q[nq + i] - (double)c[nc + j];
    const double dz = (double)q[2ll * nq + i] - (double)c[2 * nc + j];
    const double s = dx * dx + dy * dy + dz * dz;
    acc += exp(-alpha * s) * s;
  }
  double t = block_sum_f64(acc, sh);
  if (threadIdx.x == 0) S.part[dir * kLossBlocks + blk] = t;
}

__global__ void chamfer_loss_final_kernel(const ChSeg *__restrict__ segs, int nseg) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 2 * nseg) return;
  const ChSeg S = segs[k >> 1];
  const int dir = k & 1;
  double t = 0.0;
  for (int b = 0; b < kLossBlocks; ++b) t += S.part[dir * kLossBlocks + b];
  S.loss[dir] = t / (double)(dir ? S.m : S.n);
}

// One segment's nb workgroups on one XCD, as for the loss.
__global__ __launch_bounds__(256) void chamfer_grad_fwd_kernel(const ChSeg *__restrict__ segs,
                                                               int nseg, unsigned nb, float alpha) {
  unsigned job, blk;
  if (!job_block(blockIdx.x, (unsigned)nseg, nb, job, blk)) return;
  const int seg = (int)job;
  const ChSeg S = segs[seg];
  const PDG_GLOBAL float *Sa = glb(S.a), *Sb = glb(S.b);
  const PDG_GLOBAL int *Snn = glb(S.nn_a);
  PDG_GLOBAL float *Sga = glb(S.ga);
  const int i = (int)blk * 256 + threadIdx.x;
  if (i >= S.n || S.ga == nullptr) return;
  const long long m = S.m, n = S.n;
  const int j = Snn[i];
  const float dx = Sa[i] - Sb[j];
  const float dy = Sa[n + i] - Sb[m + j];
  const float dz = Sa[2 * n + i] - Sb[2 * m + j];
  const float s = dx * dx + dy * dy + dz * dz;
  const float coef = (float)(S.w[0] / (double)S.n) * expf(-alpha * s) * (1.0f - alpha * s) * 2.0f;
  Sga[i] = coef * dx;
  Sga[n + i] = coef * dy;
  Sga[2 * n + i] = coef * dz;
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
  keys[g] = S.a_base + (unsigned)glb(S.nn_b)[j];
  vals[g] = g;
}

// Global segment of b index g0 (b_base is increasing).
__device__ __forceinline__ int rev_segment(const unsigned *__restrict__ b_base, int nseg,
                                           unsigned g0) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b_base[mid] <= g0)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

constexpr int kRevThreads = 256;

// Reverse direction of the adjoint: sorted entry i (key = a index, value = b
// index) contributes coef * (a - b) to ga[key].  One workgroup per 256
// entries: a segmented scan over equal keys sums each run inside the block;
// a run that starts and ends in the block is added to ga by its last thread,
// the part of a run that entered from an earlier block goes to head[block],
// and the part of a run that leaves the block goes to tail[block] (joined by
// rev_join_kernel in block order).
__global__ __launch_bounds__(kRevThreads) void chamfer_rev_scatter_kernel(
    const ChSeg *__restrict__ segs, int nseg, const unsigned *__restrict__ b_base,
    const uint32_t *__restrict__ keys, const uint32_t *__restrict__ vals, long long nent,
    float alpha, float4 *__restrict__ head, float4 *__restrict__ tail) {
  __shared__ uint32_t skey[kRevThreads + 1];
  __shared__ float wtail[kRevThreads / 64][3];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  // consecutive blocks (one segment's sorted entries) on one XCD
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  if ((long long)blk * kRevThreads >= nent) return;
  const long long b0 = (long long)blk * kRevThreads;
  const long long i = b0 + t;
  const bool valid = i < nent;
  const uint32_t key = valid ? keys[i] : 0xffffffffu;
  float v[3] = {0.f, 0.f, 0.f};
  int sg = 0;
  if (valid) {
    const unsigned g0 = vals[i];
    sg = rev_segment(b_base, nseg, g0);
    const ChSeg S = segs[sg];
    if (S.ga != nullptr) {
      const PDG_GLOBAL float *Sa = glb(S.a), *Sb = glb(S.b);
      const long long n = S.n, m = S.m;
      const int ai = (int)(key - S.a_base);
      const int j = (int)(g0 - b_base[sg]);
      const float cw = (float)(S.w[1] / (double)S.m);
      const float dx = Sa[ai] - Sb[j];
      const float dy = Sa[n + ai] - Sb[m + j];
      const float dz = Sa[2 * n + ai] - Sb[2 * m + j];
      const float d2 = dx * dx + dy * dy + dz * dz;
      const float coef = cw * expf(-alpha * d2) * (1.0f - alpha * d2) * 2.0f;
      v[0] = coef * dx;
      v[1] = coef * dy;
      v[2] = coef * dz;
    }
  }
  skey[t] = key;
  if (t == 0) skey[kRevThreads] = b0 + kRevThreads < nent ? keys[b0 + kRevThreads] : 0xffffffffu;
  // segmented inclusive scan within the wave (equal keys are contiguous)
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t ok = __shfl_up(key, off, 64);
    const bool same = lane >= off && ok == key;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float o = __shfl_up(v[c], off, 64);
      if (same) v[c] = o + v[c];
    }
  }
  if (lane == 63) {
#pragma unroll
    for (int c = 0; c < 3; ++c) wtail[wv][c] = v[c];
  }
  __syncthreads();
  // carry into this wave's leading run from the waves before it
  if (wv > 0 && key == skey[64 * wv]) {
    float cin[3] = {0.f, 0.f, 0.f};
    for (int j = wv - 1; j >= 0; --j) {
      if (skey[64 * j + 63] != key) break;
#pragma unroll
      for (int c = 0; c < 3; ++c) cin[c] += wtail[j][c];
      if (skey[64 * j] != key) break;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = cin[c] + v[c];
  }
  if (!valid || (skey[t + 1] == key && t + 1 < kRevThreads)) return;   // not the run's last here
  const bool ends = skey[t + 1] != key;                 // run ends inside this block
  const bool entered = blk > 0 && key == skey[0] && keys[b0 - 1] == key;
  if (entered) {
    head[blk] = make_float4(v[0], v[1], v[2], 0.f);
  } else if (!ends) {
    tail[blk] = make_float4(v[0], v[1], v[2], 0.f);
  } else {
    const ChSeg &S = segs[sg];
    if (S.ga == nullptr) return;
    const long long n = S.n;
    const int ai = (int)(key - S.a_base);
    PDG_GLOBAL float *ga = glb(S.ga);
    ga[ai] += v[0];
    ga[n + ai] += v[1];
    ga[2 * n + ai] += v[2];
  }
}

// Runs that cross block boundaries: for each block whose last run started in
// it and continues, tail[b] + head[b + 1] + ... in block order is added to ga.
__global__ __launch_bounds__(256) void rev_join_kernel(const ChSeg *__restrict__ segs, int nseg,
                                                       const unsigned *__restrict__ b_base,
                                                       const uint32_t *__restrict__ keys,
                                                       const uint32_t *__restrict__ vals,
                                                       long long nent, int nblocks,
                                                       const float4 *__restrict__ head,
                                                       const float4 *__restrict__ tail) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblocks) return;
  const long long b0 = (long long)b * kRevThreads;
  const long long last = b0 + kRevThreads - 1 < nent ? b0 + kRevThreads - 1 : nent - 1;
  const uint32_t key = keys[last];
  if (last + 1 >= nent || keys[last + 1] != key) return;   // the last run ends in block b
  if (b > 0 && keys[b0] == key && keys[b0 - 1] == key) return;   // started before block b
  float4 s = tail[b];
  for (int b2 = b + 1; b2 < nblocks; ++b2) {
    const float4 h = head[b2];
    s.x += h.x;
    s.y += h.y;
    s.z += h.z;
    const long long e2 = (long long)b2 * kRevThreads + kRevThreads - 1;
    if (e2 + 1 >= nent || keys[e2 + 1] != key) break;
  }
  const int sg = rev_segment(b_base, nseg, vals[last]);
  const ChSeg &S = segs[sg];
  if (S.ga == nullptr) return;
  const long long n = S.n;
  const int ai = (int)(key - S.a_base);
  PDG_GLOBAL float *ga = glb(S.ga);
  ga[ai] += s.x;
  ga[n + ai] += s.y;
  ga[2 * n + ai] += s.z;
}

}  // namespace

pdg_status launch_nn_exact(const NNJob *jobs, int njobs, int max_nq, hipStream_t st) {
  if (njobs <= 0 || max_nq <= 0) return PDG_OK;
  dim3 grid(div_up(max_nq, kQTile), njobs);
  nn_exact_kernel<<<grid, kNNThreads, 0, st>>>(jobs);
  return launched("nn_exact");
}

pdg_status launch_chamfer_loss(const ChSeg *segs, int nseg, double alpha, hipStream_t st) {
  if (nseg <= 0) return PDG_OK;
  const int njobs = 2 * nseg;
  chamfer_loss_kernel<<<(unsigned)job_grid(njobs, kLossBlocks), 256, 0, st>>>(segs, njobs, alpha);
  PDG_TRY(launched("chamfer_loss"));
  chamfer_loss_final_kernel<<<div_up(2 * nseg, 64), 64, 0, st>>>(segs, nseg);
  return launched("chamfer_loss_final");
}

pdg_status launch_chamfer_grad_fwd(const ChSeg *segs, int nseg, int max_n, float alpha,
                                   hipStream_t st) {
  if (nseg <= 0 || max_n <= 0) return PDG_OK;
  const unsigned nb = div_up(max_n, 256);
  chamfer_grad_fwd_kernel<<<(unsigned)job_grid(nseg, nb), 256, 0, st>>>(segs, nseg, nb, alpha);
  return launched("chamfer_grad_fwd");
}

pdg_status launch_chamfer_rev_keys(const ChSeg *segs, int nseg, int max_m, const unsigned *b_base,
                                   uint32_t *keys, uint32_t *vals, hipStream_t st) {
  if (nseg <= 0 || max_m <= 0) return PDG_OK;
  dim3 grid(div_up(max_m, 256), nseg);
  chamfer_rev_keys_kernel<<<grid, 256, 0, st>>>(segs, b_base, keys, vals);
  return launched("chamfer_rev_keys");
}

long long rev_part_count(long long nent) { return (nent + kRevThreads - 1) / kRevThreads; }

pdg_status launch_chamfer_rev_scatter(const ChSeg *segs, int nseg, const unsigned *b_base,
                                      const uint32_t *keys, const uint32_t *vals, long long nent,
                                      float alpha, float4 *part, hipStream_t st) {
  if (nent <= 0) return PDG_OK;
  const long long nb = rev_part_count(nent);
  if (nb >= (1ll << 31)) {
    set_error("chamfer reverse scatter: %lld entries exceed the launch limit", nent);
    return PDG_EINVAL;
  }
  chamfer_rev_scatter_kernel<<<xcd_pad(nb), kRevThreads, 0, st>>>(segs, nseg, b_base, keys, vals,
                                                                  nent, alpha, part, part + nb);
  PDG_TRY(launched("chamfer_rev_scatter"));
  rev_join_kernel<<<div_up(nb, 256), 256, 0, st>>>(segs, nseg, b_base, keys, vals, nent, (int)nb,
                                                   part, part + nb);
  return launched("chamfer_rev_join");
}

}  // namespace pdg
