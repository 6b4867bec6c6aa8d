// Nearest neighbours (paper Eq. 12) with a bf16 matrix-core screen and an
// exact float32 re-rank: the served form of the Chamfer search.
//
// Screen.  For query q and candidate c the matrix cores evaluate
//     S(q, c) = |c|^2 - 2 q.c           (|q|^2 is constant per query)
// as one K = 16 row of v_mfma_f32_32x32x16_bf16 with float32 accumulation.
// Each coordinate is split into two bf16 terms, x = x_hi + x_lo, and |c|^2
// into three, which fills 12 of the 16 K slots:
//     query row     [q_hi, q_hi, q_lo, 1, 1, 1, 0, 0, 0, 0]
//     candidate row [-2c_hi, -2c_lo, -2c_hi, n_hi, n_mid, n_lo, 0 x 4]
// (three coordinates per vector entry), so the only term dropped from q.c is
// q_lo.c_lo.  With a = |q| and b = max |c| over the candidate set,
//     |S + |q|^2 - |q - c|^2| <= eps(q) = 3e-5 a b + 2e-6 (a^2 + b^2) + 1e-6,
// which covers the bf16 split and dropped term (6.02 * 2^-18 a b), the float32
// accumulation of 16 terms (16 * 2^-24 (2.01 a b + b^2)), the float32
// rounding of |c|^2 and |q|^2, and the float32 threshold arithmetic.
//
// Re-rank.  Every lane keeps the exact best (d2, index) of its query under the
// library's contract (float32 difference form, no FMA, lowest index on ties).
// A candidate can be skipped only if its screened lower bound exceeds the
// current best, S + |q|^2 - eps > best (1 + 2^-20), which implies that its
// contract distance is strictly larger (the contract value is within
// 5 * 2^-24 relative of the true distance).  Every other candidate is
// evaluated exactly, so the result equals the exact search bit for bit.
// The scan may be warm-started from a previous assignment (any valid index
// is an upper bound; it changes the work, never the result).
//
// Layout.  Queries are the B operand (32 columns per MFMA), candidates the A
// operand (32 rows), so each lane holds 16 screened values of one query and
// reduces them lane-locally; lanes l and l+32 hold the two row halves of the
// same query and are merged at the end.  A workgroup (4 waves) owns 256
// queries (two 32-query blocks per wave, so one LDS read of a candidate
// fragment feeds two MFMAs) and streams the packed candidates through LDS in
// tiles of 256: the next tile is fetched into registers while the current one
// is screened, then written to the other LDS buffer.  The rare exact re-rank
// reads candidate coordinates from global memory (L2).
//
// Tile culling.  Both point sets are packed in Morton order (the permutation
// is computed once for a fixed set and reused for its smooth deformations), so
// a tile of 256 consecutive points is spatially compact, and the pack records
// each tile's bounding box.  A candidate tile is skipped for a query tile when
// the squared distance between the two boxes, times (1 - 2^-20), exceeds every
// query's current best: the box distance bounds every pair's true distance from
// below, the contract distance is within 5 * 2^-24 relative of the true one and
// the float32 box distance within 6 * 2^-24, so a skipped candidate is strictly
// farther than the best and can be neither the nearest nor a tie.  Tiles are
// listed by that test against the warm-start bests, visited starting from the
// candidate tile of the same Morton rank, and re-tested against the improving
// bests before each visit; each wave also skips a visited tile whose box
// distance to its own 64 queries exceeds their largest best.  Ties are broken on the original indices, which the
// packed coordinates carry, so the result is the exact search's bit for bit.
#include "common.h"

namespace pdg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

#ifndef PDG_SCREEN_QB
#define PDG_SCREEN_QB 2
#endif
#ifndef PDG_SCREEN_TILE
#define PDG_SCREEN_TILE 256
#endif
constexpr int kThreads = 256;
constexpr int kQB = PDG_SCREEN_QB;  // 32-query blocks per wave
constexpr int kQPerBlock = 4 * 32 * kQB;
constexpr int kCTile = PDG_SCREEN_TILE;   // candidates per LDS tile
constexpr int kPerThread = kCTile / kThreads;
constexpr int kTile = 256;          // points per box tile (query block and candidate tile)
static_assert(kQPerBlock == kTile && kCTile == kTile, "box tiles must match the screen tiles");
constexpr int kListMax = 1024;      // candidate tiles listed per pass of the cull
constexpr float kCullSlack = 1.0f - 1.0f / 1048576.0f;   // 1 - 2^-20
constexpr float kEpsAB = 3e-5f, kEpsSq = 2e-6f, kEpsAbs = 1e-6f;
constexpr float kRelSlack = 1.0f + 1.0f / 1048576.0f;   // 1 + 2^-20

__device__ __forceinline__ unsigned short bf16_rn(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);          // round to nearest even (finite inputs)
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ float d2_contract(float qx, float qy, float qz, float cx, float cy,
                                             float cz) {
#pragma clang fp contract(off)
  const float dx = qx - cx;
  const float dy = qy - cy;
  const float dz = qz - cz;
  return (dx * dx + dy * dy) + dz * dz;
}

// 30-bit Morton code of a point over [-1, 1]^3 (10 bits per axis, clamped).
__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__device__ __forceinline__ uint32_t morton_cell(float s) {
  const float u = (s + 1.0f) * 512.0f;
  return u <= 0.0f ? 0u : (u >= 1023.0f ? 1023u : (uint32_t)u);
}
__global__ __launch_bounds__(256) void morton_kernel(const float *__restrict__ x, long long ld, int n,
                                                     uint32_t *__restrict__ keys,
                                                     uint32_t *__restrict__ vals) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  keys[i] = (spread10(morton_cell(x[i])) << 2) | (spread10(morton_cell(x[ld + i])) << 1) |
            spread10(morton_cell(x[2 * ld + i]));
  vals[i] = (uint32_t)i;
}

// One thread per packed position i (original point perm[i]): the packed bf16
// row (32 B), the float32 coordinates with the original index, max |c| over
// the set (float bits of non-negative values order like unsigned integers, so
// an integer atomic max is exact and order independent; one per block), and,
// one block per 256-point tile, the tile's bounding box.
__global__ __launch_bounds__(256) void pack_kernel(const ScreenSet *__restrict__ sets, int nsets,
                                                   unsigned nb) {
  __shared__ float red[7][4];
  unsigned job, tb;                   // one set's workgroups on one XCD
  if (!job_block(blockIdx.x, (unsigned)nsets, nb, job, tb)) return;
  const ScreenSet S = sets[job];
  if ((long long)tb * 256 >= S.n) return;
  const PDG_GLOBAL float *sx = glb(S.x);
  const PDG_GLOBAL int *sperm = glb(S.perm);
  PDG_GLOBAL uint4 *spk = glb(S.pack);
  PDG_GLOBAL float4 *scoords = glb(S.coords);
  PDG_GLOBAL float4 *sboxes = glb(S.boxes);
  const int i = tb * 256 + threadIdx.x;
  float nrm = 0.f;
  float lo[3] = {__builtin_huge_valf(), __builtin_huge_valf(), __builtin_huge_valf()};
  float hi3[3] = {-__builtin_huge_valf(), -__builtin_huge_valf(), -__builtin_huge_valf()};
  if (i < S.n) {
    const long long n = S.n;
    const int o = S.perm ? sperm[i] : i;
    const float c[3] = {sx[o], sx[n + o], sx[2 * n + o]};
    unsigned short hi[3], lw[3];
    for (int k = 0; k < 3; ++k) {
      hi[k] = bf16_rn(c[k]);
      lw[k] = bf16_rn(c[k] - bf16_f(hi[k]));
      lo[k] = c[k];
      hi3[k] = c[k];
    }
    const float nn = (c[0] * c[0] + c[1] * c[1]) + c[2] * c[2];
    const unsigned short n0 = bf16_rn(nn);
    const unsigned short n1 = bf16_rn(nn - bf16_f(n0));
    const unsigned short n2 = bf16_rn((nn - bf16_f(n0)) - bf16_f(n1));
    unsigned short row[16];
    for (int k = 0; k < 3; ++k) {
      row[k] = bf16_rn(-2.0f * bf16_f(hi[k]));
      row[3 + k] = bf16_rn(-2.0f * bf16_f(lw[k]));
      row[6 + k] = row[k];
    }
    row[9] = n0;
    row[10] = n1;
    row[11] = n2;
    row[12] = row[13] = row[14] = row[15] = 0;
    uint4 w0, w1;
    w0.x = row[0] | ((unsigned)row[1] << 16);
    w0.y = row[2] | ((unsigned)row[3] << 16);
    w0.z = row[4] | ((unsigned)row[5] << 16);
    w0.w = row[6] | ((unsigned)row[7] << 16);
    w1.x = row[8] | ((unsigned)row[9] << 16);
    w1.y = row[10] | ((unsigned)row[11] << 16);
    w1.z = 0u;
    w1.w = 0u;
    spk[2 * i] = w0;
    spk[2 * i + 1] = w1;
    scoords[i] = make_float4(c[0], c[1], c[2], __int_as_float(o));
    nrm = sqrtf(nn);
  }
  for (int o = 32; o > 0; o >>= 1) {
    nrm = fmaxf(nrm, __shfl_xor(nrm, o, 64));
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], o, 64));
      hi3[k] = fmaxf(hi3[k], __shfl_xor(hi3[k], o, 64));
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[6][wv] = nrm;
    for (int k = 0; k < 3; ++k) {
      red[k][wv] = lo[k];
      red[3 + k][wv] = hi3[k];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float b[6];
    for (int k = 0; k < 3; ++k) {
      b[k] = fminf(fminf(red[k][0], red[k][1]), fminf(red[k][2], red[k][3]));
      b[3 + k] = fmaxf(fmaxf(red[3 + k][0], red[3 + k][1]), fmaxf(red[3 + k][2], red[3 + k][3]));
    }
    // one atomic per block; each set's maximum sits on a cache line of its own
    const float m = fmaxf(fmaxf(red[6][0], red[6][1]), fmaxf(red[6][2], red[6][3]));
    if (m > 0.f) atomicMax(glb(S.maxnorm), __float_as_uint(m));
    sboxes[2 * tb] = make_float4(b[0], b[1], b[2], 0.f);
    sboxes[2 * tb + 1] = make_float4(b[3], b[4], b[5], 0.f);
  }
}

// Squared distance between two axis-aligned boxes (0 when they overlap).
__device__ __forceinline__ float box_lb(const float4 &amin, const float4 &amax, const float4 &bmin,
                                        const float4 &bmax) {
#pragma clang fp contract(off)
  const float dx = fmaxf(fmaxf(amin.x - bmax.x, bmin.x - amax.x), 0.f);
  const float dy = fmaxf(fmaxf(amin.y - bmax.y, bmin.y - amax.y), 0.f);
  const float dz = fmaxf(fmaxf(amin.z - bmax.z, bmin.z - amax.z), 0.f);
  return (dx * dx + dy * dy) + dz * dz;
}

struct QState {
  float x, y, z, qn, eps, best, thr;
  int idx;
};

__device__ __forceinline__ void set_thr(QState &s) { s.thr = s.best * kRelSlack - s.qn + s.eps; }

// rows held by this lane for output register r of a 32x32 MFMA
__device__ __forceinline__ int out_row(int r, int lane) {
  return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

__device__ __forceinline__ void consider(QState &s, const f32x16 &v, int lane, int cbase, int nc,
                                         const PDG_GLOBAL float4 *__restrict__ cc) {
  // (the chain starts from +inf, a canonical value, so that no product needs
  // a canonicalising instruction before the three-operand minima)
  float m = __builtin_huge_valf();
#pragma unroll
  for (int r = 0; r < 16; r += 2) m = fminf(fminf(m, v[r]), v[r + 1]);
  if (!(m <= s.thr)) return;
  // rare path: rows whose screened value passes the current threshold (the
  // threshold only tightens below, so re-ranking all of them is safe)
  unsigned mask = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) mask |= (v[r] <= s.thr ? 1u : 0u) << r;
  while (mask) {
    const int r = __builtin_ctz(mask);
    mask &= mask - 1;
    const int c = cbase + out_row(r, lane);
    if (c >= nc) continue;             // padded rows never count
    const float4 p = cc[c];
    const float d = d2_contract(s.x, s.y, s.z, p.x, p.y, p.z);
    const int o = __float_as_int(p.w);
    if (d < s.best || (d == s.best && o < s.idx)) {
      s.best = d;
      s.idx = o;
      set_thr(s);
    }
  }
}

// this thread's share of a tile: packed rows of candidates c0 + tid + k*256
struct TileRegs {
  uint4 w[kPerThread][2];
};

__device__ __forceinline__ void fetch_tile(const PDG_GLOBAL uint4 *pack, int nc, int c0,
                                           TileRegs &t) {
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    // every lane loads (rows past the end re-read the last row), so the
    // number of loads in flight is the same on every path
    const int c = c0 + k * kThreads + (int)threadIdx.x;
    const long long cl = c < nc ? c : nc - 1;
    t.w[k][0] = pack[2 * cl];
    t.w[k][1] = pack[2 * cl + 1];
    if (c >= nc) {
      t.w[k][0] = make_uint4(0u, 0u, 0u, 0u);
      t.w[k][1] = make_uint4(0x7F800000u, 0u, 0u, 0u);   // n_hi = +inf: S = +inf
    }
  }
}

__device__ __forceinline__ void store_tile(const TileRegs &t, uint4 *spack) {
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int i = k * kThreads + (int)threadIdx.x;
    spack[2 * i] = t.w[k][0];
    spack[2 * i + 1] = t.w[k][1];
  }
}

template <int D>
__device__ __forceinline__ float row_shr(float x) {   // lane l - D of its row of 16, else 0
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x110 + D, 0xf, 0xf, true));
}

// Largest current best of this wave's valid queries (lanes without a query
// report 0); the block maximum bounds every query's best from above.
__device__ __forceinline__ float wave_best_max(const QState *st, const bool *ok) {
  float m = 0.f;
#pragma unroll
  for (int h = 0; h < kQB; ++h) m = ok[h] ? fmaxf(m, st[h].best) : m;
  // row maxima by DPP shifts (bests are >= 0, so the zeros shifted in are
  // harmless; all lanes are active here), then the four row ends read out
  m = fmaxf(m, row_shr<1>(m));
  m = fmaxf(m, row_shr<2>(m));
  m = fmaxf(m, row_shr<4>(m));
  m = fmaxf(m, row_shr<8>(m));
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 15));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 31));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 47));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 63));
  return fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
}

// Workgroups are dealt to the 8 XCDs round robin; remap the linear block id so
// that each XCD takes one contiguous run of (job, query tile) pairs: Morton-
// adjacent query tiles visit mostly the same candidate tiles, which then stay
// in that XCD's L2.
constexpr int kXcds = 8;

// The grid is 1-D with a multiple of 8 blocks, so lin -> tile is a bijection;
// tile = job * qt + query tile, tiles >= nblk do nothing.
__global__ __launch_bounds__(kThreads, 5) void nn_screen_kernel(const ScreenJob *__restrict__ jobs,
                                                             int warm, unsigned qt, unsigned nblk) {
  const unsigned lin = blockIdx.x;
  const unsigned per = gridDim.x / kXcds;
  const unsigned tile = (lin % kXcds) * per + lin / kXcds;
  if (tile >= nblk) return;
  const unsigned bx = tile % qt, by = tile / qt;
  const ScreenJob J = jobs[by];
  const int q0 = bx * kQPerBlock;
  if (q0 >= J.nq) return;
  const PDG_GLOBAL float4 *jq = glb(J.q), *jcc = glb(J.cc);
  const PDG_GLOBAL float4 *jqboxes = glb(J.qboxes), *jcboxes = glb(J.cboxes);
  const PDG_GLOBAL float *jc = glb(J.c);
  const PDG_GLOBAL uint4 *jpack = glb(J.pack);
  PDG_GLOBAL int *jnn = glb(J.nn);
  __shared__ uint4 spack[2][kCTile * 2];
  __shared__ int tlist[kListMax];
  __shared__ float tlb[kListMax];
  __shared__ float wmax[2][4];
  __shared__ int s_count;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int half = lane >> 5;
  const long long nc = J.nc;
  const float cmax = __uint_as_float(*glb(J.maxnorm));
  QState st[kQB];
  bool ok[kQB];
  int qorig[kQB];
  bf16x8 bq[kQB];
#pragma unroll
  for (int h = 0; h < kQB; ++h) {
    const int q = q0 + wv * 32 * kQB + h * 32 + (lane & 31);   // packed position
    QState &s = st[h];
    ok[h] = q < J.nq;
    float4 qc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ok[h]) qc = jq[q];
    qorig[h] = __float_as_int(qc.w);
    s.x = qc.x;
    s.y = qc.y;
    s.z = qc.z;
    s.qn = (s.x * s.x + s.y * s.y) + s.z * s.z;
    const float a = sqrtf(s.qn);
    s.eps = kEpsAB * a * cmax + kEpsSq * (s.qn + cmax * cmax) + kEpsAbs;
    s.best = __builtin_huge_valf();
    s.idx = 0x7fffffff;
    if (ok[h] && warm) {
      const int p = jnn[qorig[h]];
      if (p >= 0 && p < J.nc) {
        s.best = d2_contract(s.x, s.y, s.z, jc[p], jc[nc + p], jc[2 * nc + p]);
        s.idx = p;
      }
    }
    set_thr(s);
    // B operand: column (lane & 31), k-slots 8*half .. 8*half+7 of the query row
    const float qv[3] = {s.x, s.y, s.z};
    unsigned short hi[3], lo[3];
    for (int k = 0; k < 3; ++k) {
      hi[k] = bf16_rn(qv[k]);
      lo[k] = bf16_rn(qv[k] - bf16_f(hi[k]));
    }
    const unsigned short one = 0x3F80;
    unsigned short row[16] = {hi[0], hi[1], hi[2], hi[0], hi[1], hi[2], lo[0], lo[1],
                              lo[2], one, one, one, 0, 0, 0, 0};
    for (int e = 0; e < 8; ++e) {
      const unsigned short b = row[8 * half + e];
      bq[h][e] = *reinterpret_cast<const __bf16 *>(&b);
    }
  }
  const float4 qmin = jqboxes[2 * bx], qmax = jqboxes[2 * bx + 1];
  // this wave's 64 queries: their box (wave-uniform)
  float4 wmin = make_float4(__builtin_huge_valf(), __builtin_huge_valf(), __builtin_huge_valf(), 0.f);
  float4 wmaxc = make_float4(-__builtin_huge_valf(), -__builtin_huge_valf(), -__builtin_huge_valf(), 0.f);
#pragma unroll
  for (int h = 0; h < kQB; ++h)
    if (ok[h]) {
      wmin = make_float4(fminf(wmin.x, st[h].x), fminf(wmin.y, st[h].y), fminf(wmin.z, st[h].z), 0.f);
      wmaxc = make_float4(fmaxf(wmaxc.x, st[h].x), fmaxf(wmaxc.y, st[h].y), fmaxf(wmaxc.z, st[h].z), 0.f);
    }
  for (int o = 32; o > 0; o >>= 1) {
    wmin.x = fminf(wmin.x, __shfl_xor(wmin.x, o, 64));
    wmin.y = fminf(wmin.y, __shfl_xor(wmin.y, o, 64));
    wmin.z = fminf(wmin.z, __shfl_xor(wmin.z, o, 64));
    wmaxc.x = fmaxf(wmaxc.x, __shfl_xor(wmaxc.x, o, 64));
    wmaxc.y = fmaxf(wmaxc.y, __shfl_xor(wmaxc.y, o, 64));
    wmaxc.z = fmaxf(wmaxc.z, __shfl_xor(wmaxc.z, o, 64));
  }
  // wave-uniform: keep it in scalar registers
  wmin = make_float4(__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wmin.x))),
                     __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wmin.y))),
                     __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wmin.z))), 0.f);
  wmaxc = make_float4(__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wmaxc.x))),
                      __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wmaxc.y))),
                      __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wmaxc.z))), 0.f);
  const bool wany = wmin.x <= wmaxc.x;       // the wave has at least one query
  const int ntiles = (J.nc + kTile - 1) / kTile;
  const int qtiles = (J.nq + kTile - 1) / kTile;
  const int start = (int)((long long)bx * ntiles / qtiles);
  {
    const float m = wave_best_max(st, ok);
    if (lane == 0) wmax[0][wv] = m;
  }
  __syncthreads();
  float bmax = fmaxf(fmaxf(wmax[0][0], wmax[0][1]), fmaxf(wmax[0][2], wmax[0][3]));
  int it = 1;                   // parity of the wmax buffer written next
  unsigned issued = 0;          // matrix-core products this wave issued (wave-uniform)
  TileRegs regs;
  for (int base = 0; base < ntiles; base += kListMax) {
    const int span = ntiles - base < kListMax ? ntiles - base : kListMax;
    if (wv == 0) {              // list the tiles that pass the box test, in visiting order
      int count = 0;
      for (int k0 = 0; k0 < span; k0 += 64) {
        const int k = k0 + lane;
        bool pass = false;
        float lb = 0.f;
        int tile = 0;
        if (k < span) {
          tile = (start + base + k) % ntiles;
          lb = box_lb(qmin, qmax, jcboxes[2 * tile], jcboxes[2 * tile + 1]);
          pass = !(lb * kCullSlack > bmax);
        }
        const unsigned long long m = __ballot(pass);
        const int pos = count + __popcll(m & ((1ull << lane) - 1ull));
        if (pass) {
          tlist[pos] = tile;
          tlb[pos] = lb;
        }
        count += __popcll(m);
      }
      if (lane == 0) s_count = count;
    }
    __syncthreads();
    const int count = s_count;
    int i = 0;
    while (i < count && tlb[i] * kCullSlack > bmax) ++i;
    float4 tmin = make_float4(0.f, 0.f, 0.f, 0.f), tmax = tmin;   // box of tile tlist[i]
    if (i < count) {
      fetch_tile(jpack, J.nc, tlist[i] * kTile, regs);
      tmin = jcboxes[2 * tlist[i]];
      tmax = jcboxes[2 * tlist[i] + 1];
      store_tile(regs, spack[0]);
    }
    int buf = 0;
    while (i < count) {
      const float wbest = wave_best_max(st, ok);
      if (lane == 0) wmax[it & 1][wv] = wbest;
      __syncthreads();          // tile tlist[i] is in spack[buf]; the other buffer is free
      bmax = fmaxf(fmaxf(wmax[it & 1][0], wmax[it & 1][1]), fmaxf(wmax[it & 1][2], wmax[it & 1][3]));
      ++it;
      int nxt = i + 1;
      while (nxt < count && tlb[nxt] * kCullSlack > bmax) ++nxt;
      const bool more = nxt < count;
      // the next tile and its box, in flight while this tile is screened
      // (issued on every path; without a next tile this one is read again)
      const int ft = tlist[more ? nxt : i];
      fetch_tile(jpack, J.nc, ft * kTile, regs);
      const float4 nmin = jcboxes[2 * ft], nmax = jcboxes[2 * ft + 1];
      const int c0 = tlist[i] * kTile;
      const int left = (J.nc - c0 + 31) / 32;
      // the wave skips a tile that cannot beat any of its own queries' bests
      const bool wskip = !wany || box_lb(wmin, wmaxc, tmin, tmax) * kCullSlack > wbest;
      const int nsub = wskip ? 0 : (left < kCTile / 32 ? left : kCTile / 32);
      // the next sub-tile's operand is read from LDS before this one's products
      uint4 nraw = spack[buf][2 * (lane & 31) + half];
      for (int sub = 0; sub < nsub; ++sub) {
        const uint4 raw = nraw;
        const int ns = sub + 1 < nsub ? sub + 1 : sub;
        nraw = spack[buf][2 * (ns * 32 + (lane & 31)) + half];
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&raw);
        const f32x16 z = {};
#pragma unroll
        for (int h = 0; h < kQB; ++h) {   // one result live at a time (register budget)
          const f32x16 v = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bq[h], z, 0, 0, 0);
          consider(st[h], v, lane, c0 + sub * 32, J.nc, jcc);
        }
      }
      if (more) store_tile(regs, spack[buf ^ 1]);
      buf ^= 1;
      i = nxt;
      tmin = nmin;
      tmax = nmax;
      issued += (unsigned)(nsub * kQB);
    }
    __syncthreads();            // the list is rebuilt next
  }
#pragma unroll
  for (int h = 0; h < kQB; ++h) {
    QState &s = st[h];
    const float ob = __shfl_xor(s.best, 32, 64);
    const int oi = __shfl_xor(s.idx, 32, 64);
    if (ob < s.best || (ob == s.best && oi < s.idx)) {
      s.best = ob;
      s.idx = oi;
    }
    if (half == 0 && ok[h]) jnn[qorig[h]] = s.idx;
  }
  // one integer atomic per wave: the 32 x 32 x 16 products it issued (tiles
  // a wave skipped by its own box test count nothing)
  if (J.tiles && lane == 0 && issued) atomicAdd(glb(J.tiles), (unsigned long long)issued);
}

}  // namespace

pdg_status launch_morton(const float *x, long long ld, int n, uint32_t *keys, uint32_t *vals,
                         hipStream_t st) {
  if (n <= 0) return PDG_OK;
  morton_kernel<<<div_up(n, 256), 256, 0, st>>>(x, ld, n, keys, vals);
  return launched("morton");
}

pdg_status launch_screen_pack(const ScreenSet *sets, int nsets, int max_n, hipStream_t st) {
  if (nsets <= 0 || max_n <= 0) return PDG_OK;
  const unsigned nb = div_up(max_n, 256);
  pack_kernel<<<(unsigned)job_grid(nsets, nb), 256, 0, st>>>(sets, nsets, nb);
  return launched("screen_pack");
}

pdg_status launch_nn_screen(const ScreenJob *jobs, int njobs, int max_nq, int warm,
                            hipStream_t st) {
  if (njobs <= 0 || max_nq <= 0) return PDG_OK;
  const unsigned qt = div_up(max_nq, kQPerBlock);
  const unsigned long long nblk = (unsigned long long)qt * njobs;
  const unsigned long long padded = (nblk + kXcds - 1) / kXcds * kXcds;
  if (padded >= (1ull << 31)) {
    set_error("nn screen: %llu workgroups exceed the launch limit", padded);
    return PDG_EINVAL;
  }
  nn_screen_kernel<<<(unsigned)padded, kThreads, 0, st>>>(jobs, warm, qt, (unsigned)nblk);
  return launched("nn_screen");
}

}  // namespace pdg
