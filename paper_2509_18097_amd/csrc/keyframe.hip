// Keyframe selection (paper Sec. 3.5, Eq. 19-20): the number of occupied
// voxels of a 128^3 grid over [-1, 1]^3 in every frame, weighted by
// exp(-gamma (t - T/2)^2) with T = frames - 1, and the first frame of largest
// weighted count.
//
// Occupancy is a bit per voxel and frame set with integer atomics (the result
// does not depend on their order), counted by population counts and a
// fixed-order block sum, so the counts are exact and reproducible.
#include "common.h"

namespace pdg {
namespace {

constexpr int kVoxGrid = 128;
constexpr long long kVoxWords = (long long)kVoxGrid * kVoxGrid * kVoxGrid / 32;   // per frame

// Voxel of coordinate s: floor((s + 1) * 64) in float32 (the product by 64 is
// exact), clamped to 0..127; a NaN coordinate falls in voxel 0.
__device__ __forceinline__ int voxel1(float s) {
  float u = (s + 1.0f) * (0.5f * (float)kVoxGrid);
  u = fminf(fmaxf(u, 0.0f), (float)(kVoxGrid - 1));
  return (int)floorf(u);
}

__global__ __launch_bounds__(256) void occupy_kernel(const float *__restrict__ points, long long n,
                                                     unsigned *__restrict__ bits) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long f = blockIdx.y;
  const float *P = points + f * 3 * n;
  const int ix = voxel1(P[i]), iy = voxel1(P[n + i]), iz = voxel1(P[2 * n + i]);
  const unsigned id = ((unsigned)iz * kVoxGrid + (unsigned)iy) * kVoxGrid + (unsigned)ix;
  atomicOr(&bits[f * kVoxWords + (id >> 5)], 1u << (id & 31u));
}

// counts[f] = number of set bits of frame f: one workgroup per frame.
__global__ __launch_bounds__(256) void occupancy_count_kernel(const unsigned *__restrict__ bits,
                                                              long long *__restrict__ counts) {
  __shared__ long long part[256];
  const long long f = blockIdx.x;
  const unsigned *B = bits + f * kVoxWords;
  long long c = 0;
  for (long long w = threadIdx.x; w < kVoxWords; w += blockDim.x) c += __popc(B[w]);
  part[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[f] = part[0];
}

// Eq. 19: first frame of largest exp(-gamma (t - T/2)^2) * count (float64).
__global__ void keyframe_select_kernel(const long long *__restrict__ counts, int frames,
                                       double gamma, int *__restrict__ key) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double mid = 0.5 * (double)(frames - 1);
  int best = 0;
  double bs = -1.0;
  for (int t = 0; t < frames; ++t) {
    const double d = (double)t - mid;
    const double s = exp(-gamma * d * d) * (double)counts[t];
    if (s > bs) {
      bs = s;
      best = t;
    }
  }
  key[0] = best;
}

}  // namespace

size_t keyframe_bytes(int frames) {
  return (size_t)frames * kVoxWords * sizeof(unsigned) + (size_t)frames * sizeof(long long) + 256;
}

pdg_status launch_keyframe(const float *points, int frames, long long n, double gamma,
                           long long *counts, int *key, void *ws, hipStream_t st) {
  unsigned *bits = (unsigned *)ws;
  long long *cnt = counts;
  if (!cnt) {
    const size_t off = ((size_t)frames * kVoxWords * sizeof(unsigned) + 255) & ~(size_t)255;
    cnt = (long long *)((char *)ws + off);
  }
  PDG_TRY(launch_fill((float *)bits, (long long)frames * kVoxWords, 0.f, st));
  if (n > 0) {
    dim3 grid(div_up(n, 256), frames);
    occupy_kernel<<<grid, 256, 0, st>>>(points, n, bits);
    PDG_TRY(launched("occupy"));
  }
  occupancy_count_kernel<<<frames, 256, 0, st>>>(bits, cnt);
  PDG_TRY(launched("occupancy_count"));
  keyframe_select_kernel<<<1, 64, 0, st>>>(cnt, frames, gamma, key);
  return launched("keyframe_select");
}

}  // namespace pdg
