// Stable LSD radix sort of (uint32 key, uint32 value) pairs for gfx950.
//
// Used wherever the step needs a scatter-add to be deterministic: entries are
// sorted by destination, then every run of equal keys is summed in entry
// order by one thread (no floating-point atomics anywhere).
//
// Per 8-bit digit pass:
//   hist    -- per 2048-entry tile, digit counts (LDS integer atomics: exact;
//              a wave whose entries share one digit, as on nearly sorted
//              input, adds its count with one atomic instead of 64);
//   scan    -- exclusive scan of the digit-major count table;
//   scatter -- each tile ranks its entries stably (round-major, then wave,
//              then lane order; the same ballot matching), stages them in LDS
//              in digit order and writes each digit's run of the tile to its
//              consecutive final slots (coalesced).
#include "common.h"

namespace pdg {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;
constexpr int kScanThreads = 1024;

// Lanes of the wave (valid ones) holding the same 8-bit digit d as this lane.
__device__ __forceinline__ unsigned long long digit_peers(uint32_t d, bool valid) {
  unsigned long long same = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const unsigned long long m = __ballot((d >> b) & 1u);
    same &= ((d >> b) & 1u) ? m : ~m;
  }
  return same;
}

__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const uint32_t *__restrict__ keys,
                                                              long long n, int shift,
                                                              uint32_t *__restrict__ hist,
                                                              int nblocks) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const long long base = (long long)blockIdx.x * kTile;
  const int lane = threadIdx.x & 63;
  uint32_t k[kItems];
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const long long i = base + r * kThreads + threadIdx.x;
    k[r] = i < n ? keys[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const bool valid = base + r * kThreads + threadIdx.x < n;
    const uint32_t d = (k[r] >> shift) & 255u;
    const unsigned long long live = __ballot(valid);
    if (live == 0ull) continue;
    const uint32_t d0 = (uint32_t)__shfl(d, __ffsll((long long)live) - 1, 64);
    if (__ballot(valid && d == d0) == live) {      // one digit in the whole wave
      if (lane == __ffsll((long long)live) - 1) atomicAdd(&cnt[d0], (uint32_t)__popcll(live));
    } else if (valid) {
      atomicAdd(&cnt[d], 1u);
    }
  }
  __syncthreads();
  hist[(long long)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of `total` entries in place, one workgroup: every thread owns
// a contiguous chunk; chunk sums are scanned in LDS.  Used for short arrays
// (the per-chunk sums of the multi-block scan below).
__global__ __launch_bounds__(kScanThreads) void scan_kernel(uint32_t *__restrict__ a,
                                                            long long total) {
  __shared__ uint32_t sh[kScanThreads];
  const int t = threadIdx.x;
  long long chunk = (total + kScanThreads - 1) / kScanThreads;
  long long lo = t * chunk;
  long long hi = lo + chunk < total ? lo + chunk : total;
  uint32_t s = 0;
  for (long long i = lo; i < hi; ++i) s += a[i];
  sh[t] = s;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {
    uint32_t v = t >= d ? sh[t - d] : 0u;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  uint32_t run = sh[t] - s;  // exclusive prefix of this chunk
  for (long long i = lo; i < hi; ++i) {
    uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
}

// Multi-block exclusive scan: chunks of kScanChunk entries; phase 1 sums each
// chunk, phase 2 scans the chunk sums (scan_kernel), phase 3 scans each chunk
// from its offset.  Thread t of a chunk owns 4 consecutive entries.
constexpr int kScanChunk = kScanThreads * 4;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

__global__ __launch_bounds__(kScanThreads) void scan_sums_kernel(const uint32_t *__restrict__ a,
                                                                 long long total,
                                                                 uint32_t *__restrict__ sums) {
  __shared__ uint32_t sh[kScanThreads / 64];
  const long long base = (long long)blockIdx.x * kScanChunk + 4ll * threadIdx.x;
  uint32_t v = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (base + k < total) v += a[base + k];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) t += sh[w];
    sums[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_chunks_kernel(uint32_t *__restrict__ a,
                                                                   long long total,
                                                                   const uint32_t *__restrict__ offs) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  const long long base = (long long)blockIdx.x * kScanChunk + 4ll * threadIdx.x;
  uint32_t v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = base + k < total ? a[base + k] : 0u;
  const uint32_t own = v[0] + v[1] + v[2] + v[3];
  const uint32_t incl = wave_incl_scan(own);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t off = offs[blockIdx.x] + incl - own;
  for (int i = 0; i < w; ++i) off += wsum[i];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < total) a[base + k] = off;
    off += v[k];
  }
}

__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, long long n, int shift,
    const uint32_t *__restrict__ hist, int nblocks) {
  __shared__ uint32_t s_off[256];                  // global slot of the tile's digit run
  __shared__ uint32_t s_run[256];                  // tile-local start of each digit run
  __shared__ uint32_t s_cnt[kThreads / 64][256];   // a round's per-wave digit counts
  __shared__ uint32_t s_key[kTile], s_val[kTile];  // the tile in (digit, rank) order
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const unsigned long long lt = (1ull << lane) - 1ull;
  s_off[tid] = hist[(long long)tid * nblocks + blockIdx.x];
  s_run[tid] = 0;                                  // running count of digit tid
  const long long base = (long long)blockIdx.x * kTile;
  const int tn = n - base < kTile ? (int)(n - base) : kTile;
  uint32_t key[kItems], val[kItems], rank[kItems];
  // ranks: stable order (round, wave, lane) among the tile's entries of a digit
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) s_cnt[w][tid] = 0;
    const int li = r * kThreads + tid;
    const bool valid = li < tn;
    key[r] = valid ? kin[base + li] : 0u;
    val[r] = valid ? vin[base + li] : 0u;
    const uint32_t d = (key[r] >> shift) & 255u;
    const unsigned long long same = digit_peers(d, valid);
    const int wr = __popcll(same & lt);
    __syncthreads();
    if (valid && wr == 0) s_cnt[wid][d] = (uint32_t)__popcll(same);
    __syncthreads();
    uint32_t rk = s_run[d] + (uint32_t)wr;
    for (int w = 0; w < wid; ++w) rk += s_cnt[w][d];
    rank[r] = rk;
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) add += s_cnt[w][tid];
    s_run[tid] += add;                             // digit tid's count so far
  }
  __syncthreads();
  // tile-local run starts: exclusive scan of the 256 digit counts
  {
    const uint32_t c = s_run[tid];
    uint32_t incl = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t o = __shfl_up(incl, d, 64);
      if (lane >= d) incl += o;
    }
    __shared__ uint32_t s_wsum[kThreads / 64];
    if (lane == 63) s_wsum[wid] = incl;
    __syncthreads();
    uint32_t off = incl - c;
    for (int w = 0; w < wid; ++w) off += s_wsum[w];
    __syncthreads();
    s_run[tid] = off;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    if (r * kThreads + tid < tn) {
      const uint32_t p = s_run[(key[r] >> shift) & 255u] + rank[r];
      s_key[p] = key[r];
      s_val[p] = val[r];
    }
  }
  __syncthreads();
  // slot i of the staged tile: digit d, the (i - run start)-th of the tile's
  // entries of d, so its final slot is s_off[d] + i - s_run[d]
#pragma unroll
  for (int r = 0; r < kItems; ++r) {
    const int i = r * kThreads + tid;
    if (i < tn) {
      const uint32_t k = s_key[i], d = (k >> shift) & 255u;
      const uint32_t pos = s_off[d] + (uint32_t)i - s_run[d];
      kout[pos] = k;
      vout[pos] = s_val[i];
    }
  }
}

__global__ void copy_u32_kernel(const uint32_t *__restrict__ a, const uint32_t *__restrict__ b,
                                uint32_t *__restrict__ ao, uint32_t *__restrict__ bo,
                                long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    ao[i] = a[i];
    bo[i] = b[i];
  }
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t radix_sort_bytes(long long n) {
  long long nb = (n + kTile - 1) / kTile;
  if (nb < 1) nb = 1;
  const long long nchunks = (nb * 256 + kScanChunk - 1) / kScanChunk;
  return 2 * align256((size_t)n * 4) + align256((size_t)nb * 256 * 4) +
         align256((size_t)nchunks * 4);
}

pdg_status radix_sort(uint32_t *keys, uint32_t *vals, long long n, int bits, void *scratch,
                      hipStream_t st) {
  if (n <= 1) return PDG_OK;
  if (n > (1ll << 31)) {
    set_error("radix_sort: %lld entries exceed 2^31", n);
    return PDG_EINVAL;
  }
  int passes = (bits + 7) / 8;
  if (passes < 1) passes = 1;
  if (passes > 4) passes = 4;
  int nb = (int)((n + kTile - 1) / kTile);
  char *s = (char *)scratch;
  uint32_t *kalt = (uint32_t *)s;
  uint32_t *valt = (uint32_t *)(s + align256((size_t)n * 4));
  uint32_t *hist = (uint32_t *)(s + 2 * align256((size_t)n * 4));
  const long long htotal = (long long)nb * 256;
  const int nchunks = (int)((htotal + kScanChunk - 1) / kScanChunk);
  uint32_t *sums = (uint32_t *)(s + 2 * align256((size_t)n * 4) + align256((size_t)htotal * 4));
  uint32_t *ks = keys, *vs = vals, *kd = kalt, *vd = valt;
  for (int p = 0; p < passes; ++p) {
    int shift = 8 * p;
    radix_hist_kernel<<<nb, kThreads, 0, st>>>(ks, n, shift, hist, nb);
    PDG_TRY(launched("radix_hist"));
    scan_sums_kernel<<<nchunks, kScanThreads, 0, st>>>(hist, htotal, sums);
    PDG_TRY(launched("radix_scan_sums"));
    scan_kernel<<<1, kScanThreads, 0, st>>>(sums, nchunks);
    PDG_TRY(launched("radix_scan_top"));
    scan_chunks_kernel<<<nchunks, kScanThreads, 0, st>>>(hist, htotal, sums);
    PDG_TRY(launched("radix_scan_chunks"));
    radix_scatter_kernel<<<nb, kThreads, 0, st>>>(ks, vs, kd, vd, n, shift, hist, nb);
    PDG_TRY(launched("radix_scatter"));
    uint32_t *t0 = ks, *t1 = vs;
    ks = kd;
    vs = vd;
    kd = t0;
    vd = t1;
  }
  if (ks != keys) {
    copy_u32_kernel<<<div_up(n, 256), 256, 0, st>>>(ks, vs, keys, vals, n);
    PDG_TRY(launched("radix_copy"));
  }
  return PDG_OK;
}

}  // namespace pdg
