// Nearest neighbours (paper Eq. 12) with a bf16 matrix-core screen and an
// exact float32 re-rank: the served form of the Chamfer search.
//
// Screen.  Candidates come in Morton-ordered tiles of 256; every tile has a
// frame, its box centre C (float32), and is packed relative to it,
// delta = fl(c - C).  A query q entering the tile is moved into the same frame,
// x = fl(q - C), and the matrix cores evaluate
//     S(x, delta) = |delta|^2 - 2 x.delta      (|x|^2 is constant per query)
// as one K = 16 row of v_mfma_f32_32x32x16_bf16 with float32 accumulation.
// Each coordinate is split into two bf16 terms, x = x_hi + x_lo, and
// |delta|^2 into three, which fills 12 of the 16 K slots:
//     query row     [x_hi, x_hi, x_lo, 1, 1, 1, 0, 0, 0, 0]
//     candidate row [-2d_hi, -2d_lo, -2d_hi, n_hi, n_mid, n_lo, 0 x 4]
// (three coordinates per vector entry), so the only term dropped from x.delta
// is x_lo.d_lo.  With a = |x| and b >= |delta| over the tile (its radius),
//     |S + |x|^2 - |q - c|^2| <= 3e-5 a b + 2e-6 (a^2 + b^2),
// which covers the bf16 split and dropped term (6.02 * 2^-18 a b), the float32
// accumulation of 16 terms (16 * 2^-24 (2.01 a b + 1.01 b^2)), the float32
// rounding of |delta|^2 and |x|^2 (3.01 * 2^-24 each) and of the two frame
// shifts (4 * 2^-24 (a + b)^2), with 15% to spare.  Every term scales with the
// local sizes a and b, not with the distance from the origin: near the query,
// where the nearest neighbour is, the window is a small fraction of the
// neighbour distance, so the exact re-rank rarely runs for a row that is not
// the nearest one.  The float32 arithmetic of the threshold itself adds at
// most 3 * 2^-24 (best + |x|^2), covered by 4 * 2^-24 |x|^2 in the bound and
// by 2^-22 best in the slack below.
//
// Re-rank.  Every lane keeps the exact best (d2, index) of its query under the
// library's contract (float32 difference form, no FMA, lowest index on ties).
// A candidate can be skipped only if its screened lower bound exceeds the
// current best, S + |x|^2 - eps > best (1 + 2^-20), which implies that its
// contract distance is strictly larger (the contract value is within
// 5 * 2^-24 relative of the true distance).  Every other candidate is
// evaluated exactly, from the tile's float32 coordinates staged in LDS beside
// its packed rows, so the result equals the exact search bit for bit.
// The scan may be warm-started from a previous assignment (any valid index
// is an upper bound; it changes the work, never the result).
//
// Layout.  Queries are the B operand (32 columns per MFMA), candidates the A
// operand (32 rows), so each lane holds 16 screened values of one query and
// reduces them lane-locally; lanes l and l+32 hold the two row halves of the
// same query and are merged at the end.  A workgroup is one wave and owns 64
// Morton-consecutive queries (two 32-query blocks: one A operand feeds two
// MFMAs, issued before either result is reduced), so waves finish
// independently and a wave whose queries need many candidate tiles delays no
// other.  A visited tile's eight A operands go from L2 straight into
// registers, all issued at the start of the tile and consumed in order; the
// rare exact re-rank reads the candidate's float32 coordinates from L2.  The
// wave rebuilds its B operands and thresholds in the frame of every tile it
// screens.
//
// Tile culling.  Both point sets are packed in Morton order (the permutation
// is computed once for a fixed set and reused for its smooth deformations), so
// a tile of 256 consecutive points is spatially compact, and the pack records
// each tile's bounding box.  A candidate tile is skipped for a wave when the
// squared distance between its box and the box of the wave's 64 queries, times
// (1 - 2^-20), exceeds every one of their current bests: the box distance bounds every pair's true distance from
// below, the contract distance is within 5 * 2^-24 relative of the true one and
// the float32 box distance within 6 * 2^-24, so a skipped candidate is strictly
// farther than the best and can be neither the nearest nor a tie.  Tiles are
// listed by that test against the warm-start bests, visited starting from the
// candidate tile of the same Morton rank, and re-tested against the improving
// bests before each visit.  Ties are broken on the original indices, which
// the packed coordinates carry, so the result is the exact search's bit for
// bit.  (The pack also records the boxes of each tile's eight 32-point
// sub-tiles, for the exact culled search below.  Testing them here as well,
// per 32-query block, leaves about a quarter of a visited tile's products,
// but the screen's time is set by its per-tile latency, not by its products:
// the listing of the masks made it 15% slower, so the screen computes whole
// tiles.)
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
#ifndef PDG_SCREEN_WAVES
#define PDG_SCREEN_WAVES 1
#endif
#ifndef PDG_SCREEN_STAGE
#define PDG_SCREEN_STAGE 1
#endif
constexpr int kWaves = PDG_SCREEN_WAVES;   // independent waves per workgroup
constexpr int kThreads = 64 * kWaves;
constexpr bool kStage = PDG_SCREEN_STAGE;  // tile coordinates staged in LDS for the re-rank
constexpr int kQB = PDG_SCREEN_QB;  // 32-query blocks per wave
static_assert(kQB * 8 <= 32, "one flag bit per (step, query block) of a tile");
constexpr int kQPerWave = 32 * kQB;
constexpr int kQPerBlock = kWaves * kQPerWave;
constexpr int kCTile = PDG_SCREEN_TILE;   // candidates per LDS tile
constexpr int kTile = 256;          // points per box tile (query block and candidate tile)
static_assert(kCTile == kTile, "candidate boxes must match the screened tiles");
constexpr int kListMax = 256;       // candidate tiles listed per pass of a wave's cull
// float4 per tile: min corner, max corner, (centre, radius), then the min and
// max corners of its eight 32-point sub-tiles
constexpr int kSubBoxes = kTile / 32;
constexpr int kBoxStride = 3 + 2 * kSubBoxes;
static_assert(kBoxStride == 19, "the box layout is declared in common.h (screen_box_count)");
constexpr float kCullSlack = 1.0f - 1.0f / 1048576.0f;   // 1 - 2^-20
// screen error bound in a tile's frame (a = |q - C|, b = tile radius)
constexpr float kEpsAB = 3e-5f, kEpsSq = 2e-6f;
constexpr float kEpsQn = 4.0f / 16777216.0f;             // 4 * 2^-24, threshold arithmetic
constexpr float kEpsAbs = 1e-30f;                        // keeps the bound above underflow
constexpr float kThrSlack = 1.0f + 1.0f / 1048576.0f + 1.0f / 4194304.0f;   // 1 + 2^-20 + 2^-22
constexpr float kRadSlack = 1.0f + 1.0f / 1048576.0f;    // 1 + 2^-20

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

// One workgroup per 256-point tile, one thread per packed position i (original
// point perm[i]).  The tile's bounding box and its centre C (midpoint of the
// box in float32) come first; then every point is packed relative to C:
// delta = fl(c - C), its bf16 row (32 B) and |delta|^2 split in three, the
// float32 coordinates with the original index, and the tile's radius
// r = max |delta| (rounded up) beside C.
__global__ __launch_bounds__(256) void pack_kernel(const ScreenSet *__restrict__ sets, int nsets,
                                                   unsigned nb) {
#pragma clang fp contract(off)
  __shared__ float red[6][4];
  __shared__ float rads[4];
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
  if (i < S.n && S.inv) glb(S.inv)[S.perm ? sperm[i] : i] = i;   // the inverse order
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool in = i < S.n;
  float c[3] = {0.f, 0.f, 0.f};
  int o = 0;
  float lo[3] = {__builtin_huge_valf(), __builtin_huge_valf(), __builtin_huge_valf()};
  float hi3[3] = {-__builtin_huge_valf(), -__builtin_huge_valf(), -__builtin_huge_valf()};
  if (in) {
    const long long n = S.n;
    o = S.perm ? sperm[i] : i;
    c[0] = sx[o];
    c[1] = sx[n + o];
    c[2] = sx[2 * n + o];
    for (int k = 0; k < 3; ++k) lo[k] = hi3[k] = c[k];
  }
  // the 32-point sub-tile boxes (each half wave), then the wave's
  for (int d = 16; d > 0; d >>= 1)
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(lo[k], __shfl_xor(lo[k], d, 64));
      hi3[k] = fmaxf(hi3[k], __shfl_xor(hi3[k], d, 64));
    }
  if ((lane & 31) == 0) {
    const int sb = (int)(threadIdx.x >> 5);   // sub-tile of the tile
    sboxes[kBoxStride * tb + 3 + 2 * sb] = make_float4(lo[0], lo[1], lo[2], 0.f);
    sboxes[kBoxStride * tb + 4 + 2 * sb] = make_float4(hi3[0], hi3[1], hi3[2], 0.f);
  }
  for (int k = 0; k < 3; ++k) {
    lo[k] = fminf(lo[k], __shfl_xor(lo[k], 32, 64));
    hi3[k] = fmaxf(hi3[k], __shfl_xor(hi3[k], 32, 64));
  }
  if (lane == 0)
    for (int k = 0; k < 3; ++k) {
      red[k][wv] = lo[k];
      red[3 + k][wv] = hi3[k];
    }
  __syncthreads();
  float b[6], ctr[3];
  for (int k = 0; k < 3; ++k) {
    b[k] = fminf(fminf(red[k][0], red[k][1]), fminf(red[k][2], red[k][3]));
    b[3 + k] = fmaxf(fmaxf(red[3 + k][0], red[3 + k][1]), fmaxf(red[3 + k][2], red[3 + k][3]));
    ctr[k] = 0.5f * (b[k] + b[3 + k]);
  }
  float rad = 0.f;
  if (in && !S.pack) {   // coordinates only (the exact culled search)
    scoords[i] = make_float4(c[0], c[1], c[2], __int_as_float(o));
    const float d0 = c[0] - ctr[0], d1 = c[1] - ctr[1], d2 = c[2] - ctr[2];
    rad = sqrtf((d0 * d0 + d1 * d1) + d2 * d2);
  } else if (in) {
    float dl[3];
    unsigned short hi[3], lw[3];
    for (int k = 0; k < 3; ++k) {
      dl[k] = c[k] - ctr[k];
      hi[k] = bf16_rn(dl[k]);
      lw[k] = bf16_rn(dl[k] - bf16_f(hi[k]));
    }
    const float nn = (dl[0] * dl[0] + dl[1] * dl[1]) + dl[2] * dl[2];
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
    rad = sqrtf(nn);
  }
  for (int d = 32; d > 0; d >>= 1) rad = fmaxf(rad, __shfl_xor(rad, d, 64));
  if (lane == 0) rads[wv] = rad;
  __syncthreads();
  if (threadIdx.x == 0) {
    // |delta| <= sqrt(fl(|delta|^2)) (1 + 2^-20): the float32 norm and square
    // root are within 2.5 * 2^-24 of it
    const float r = fmaxf(fmaxf(rads[0], rads[1]), fmaxf(rads[2], rads[3])) * kRadSlack;
    sboxes[kBoxStride * tb] = make_float4(b[0], b[1], b[2], 0.f);
    sboxes[kBoxStride * tb + 1] = make_float4(b[3], b[4], b[5], 0.f);
    sboxes[kBoxStride * tb + 2] = make_float4(ctr[0], ctr[1], ctr[2], r);
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
  float x, y, z;      // the query (global coordinates)
  float best;         // contract d2 of the current best candidate
  int idx;            // its original index
  int pos;            // its packed position (-1: not known)
  float qn, eps;      // |q - C|^2 and the screen's error bound in the current tile's frame
  float thr;          // screened values above it are neither a better neighbour nor a tie
};

// best (1 + 2^-20 + 2^-22): the 2^-20 separates the contract distance from
// the true one, the 2^-22 covers the float32 threshold arithmetic's rounding
// of best.
__device__ __forceinline__ void set_thr(QState &s) { s.thr = s.best * kThrSlack - s.qn + s.eps; }

// The query in the frame of a candidate tile with centre C and radius rb:
// x = fl(q - C) split into bf16 hi/lo terms as this lane's half of the B
// operand (half 0: slots 0..7 = x_hi, x_hi, x_lo.x, x_lo.y; half 1: slots
// 8..15 = x_lo.z, 1, 1, 1, 0 x 4), and the error bound of the screen in
// that frame.
__device__ __forceinline__ void enter_tile(QState &s, const float4 &cen, int half, bf16x8 &bq) {
#pragma clang fp contract(off)
  const float lx = s.x - cen.x, ly = s.y - cen.y, lz = s.z - cen.z;
  const __bf16 hx = (__bf16)lx, hy = (__bf16)ly, hz = (__bf16)lz;
  const __bf16 ox = (__bf16)(lx - (float)hx), oy = (__bf16)(ly - (float)hy),
               oz = (__bf16)(lz - (float)hz);
  const __bf16 one = (__bf16)1.0f, zero = (__bf16)0.0f;
  if (half == 0) {
    bq[0] = hx; bq[1] = hy; bq[2] = hz; bq[3] = hx;
    bq[4] = hy; bq[5] = hz; bq[6] = ox; bq[7] = oy;
  } else {
    bq[0] = oz; bq[1] = one; bq[2] = one; bq[3] = one;
    bq[4] = zero; bq[5] = zero; bq[6] = zero; bq[7] = zero;
  }
  s.qn = (lx * lx + ly * ly) + lz * lz;
  // hardware square root (within 1 ulp): the constants keep 15% above the
  // derived bound
  const float a = __builtin_amdgcn_sqrtf(s.qn), rb = cen.w;
  s.eps = kEpsAB * a * rb + kEpsSq * (s.qn + rb * rb) + kEpsQn * s.qn + kEpsAbs;
  set_thr(s);
}

// Coordinates staged for the re-rank: each lane's 16 bytes go from global
// memory straight into LDS at base + 16 * lane (no registers, no wait at the
// issue); stage_wait() waits for every outstanding vector memory load,
// these included, before LDS is read.
__device__ __forceinline__ void stage_lds(const PDG_GLOBAL float4 *src, float4 *lds_base) {
  __builtin_amdgcn_global_load_lds((const PDG_GLOBAL void *)src,
                                   (__attribute__((address_space(3))) void *)lds_base, 16, 0, 0);
}
__device__ __forceinline__ void stage_wait() {
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0); expcnt and lgkmcnt not waited for
}

// rows held by this lane for output register r of a 32x32 MFMA
__device__ __forceinline__ int out_row(int r, int lane) {
  return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// Lane-local minimum of 16 screened values: two chains of three-operand
// minima from +inf (a canonical value, so no product needs a canonicalising
// instruction), joined at the end.
__device__ __forceinline__ float min16(const f32x16 &v) {
  float a = __builtin_huge_valf(), b = __builtin_huge_valf();
#pragma unroll
  for (int r = 0; r < 8; r += 2) {
    a = fminf(fminf(a, v[r]), v[r + 1]);
    b = fminf(fminf(b, v[r + 8]), v[r + 9]);
  }
  return fminf(a, b);
}

// Exact re-rank of every row of this lane whose screened value passes its
// threshold.  The lane first notes those rows against the threshold it has on
// entry (thresholds only tighten, so the rows a tighter one would skip are
// extra work, never a different result: each is strictly farther than the
// best at that point), leaving out the row of its current best itself (its
// distance equals the best and its index is the best's, so it changes
// nothing); then every lane evaluates one of its rows per round, lowest
// first, so that a round issues all lanes' coordinate loads together and a
// product costs as many rounds as its busiest lane has rows.
template <typename CoordPtr>
__device__ __forceinline__ void rerank(QState &s, const f32x16 &v, int lane, int r0, int nleft,
                                       CoordPtr tc, int c0) {
  unsigned pm = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) pm |= (v[r] <= s.thr ? 1u : 0u) << r;
  // the current best's row, when this product holds it on this lane's half
  const int rel = s.pos - (c0 + r0);
  if (rel >= 0 && rel < 32 && ((rel >> 2) & 1) == (lane >> 5))
    pm &= ~(1u << (((rel >> 3) << 2) | (rel & 3)));
  while (__ballot(pm != 0u)) {
    if (pm != 0u) {
      const int r = __builtin_ctz(pm);
      pm &= pm - 1u;
      const int row = r0 + out_row(r, lane);   // position in the tile
      if (row < nleft) {                       // padded rows never count
        const float4 p = tc[row];
        const float d = d2_contract(s.x, s.y, s.z, p.x, p.y, p.z);
        const int o = __float_as_int(p.w);
        if (d < s.best || (d == s.best && o < s.idx)) {
          s.best = d;
          s.idx = o;
          s.pos = c0 + row;
          set_thr(s);
        }
      }
    }
  }
}

// Largest current best of this wave's valid queries (lanes without a query
// report 0): an upper bound of every best the wave still improves.
template <int D>
__device__ __forceinline__ float row_shr(float x) {   // lane l - D of its row of 16, else 0
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x110 + D, 0xf, 0xf, true));
}
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

// Every wave works alone on its 64 queries: it lists the candidate tiles whose
// box can hold a better neighbour than its queries' current bests, and
// screens them one after another, re-testing each against the improved bests
// before the visit.  A visited tile's packed rows go straight from L2 into
// registers (the A operands of its eight 32-candidate steps, issued together
// at the start of the tile) and its coordinates into the wave's own LDS slice
// (for the re-rank); no workgroup barrier is taken.
//
// The grid is 1-D with a multiple of 8 blocks, so lin -> tile is a bijection;
// tile = job * qt + query tile, tiles >= nblk do nothing.
// Four waves per SIMD (the second bound counts waves per execution unit):
// at most 128 VGPRs.
__global__ __launch_bounds__(kThreads, 4) void nn_screen_kernel(
    const ScreenJob *__restrict__ jobs, int warm, unsigned qt, unsigned nblk) {
  const unsigned lin = blockIdx.x;
  const unsigned per = gridDim.x / kXcds;
  const unsigned tile = (lin % kXcds) * per + lin / kXcds;
  if (tile >= nblk) return;
  const unsigned bx = tile % qt, by = tile / qt;
  const ScreenJob J = jobs[by];
  const int q0 = bx * kQPerBlock;
  if (q0 >= J.nq) return;
  const PDG_GLOBAL float4 *jq = glb(J.q), *jcc = glb(J.cc);
  const PDG_GLOBAL float4 *jcboxes = glb(J.cboxes);
  const PDG_GLOBAL float *jc = glb(J.c);
  const PDG_GLOBAL uint4 *jpack = glb(J.pack);
  PDG_GLOBAL int *jnn = glb(J.nn);
  __shared__ float4 tcs[kWaves][kStage ? kTile : 1];   // each wave's visited tile's coordinates
  __shared__ int wls[kWaves][kListMax];
  __shared__ float wlbs[kWaves][kListMax];
  __shared__ float4 wcs[kWaves][kListMax];   // the listed tiles' (centre, radius)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  float4 *tc = tcs[wv];
  int *wl = wls[wv];
  float *wlb = wlbs[wv];
  float4 *wc = wcs[wv];
  const int half = lane >> 5;
  const long long nc = J.nc;
  QState st[kQB];
  bool ok[kQB];
  int qorig[kQB];
  bf16x8 bq[kQB];
#pragma unroll
  for (int h = 0; h < kQB; ++h) {
    const int q = q0 + wv * kQPerWave + h * 32 + (lane & 31);   // packed position
    QState &s = st[h];
    ok[h] = q < J.nq;
    float4 qc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ok[h]) qc = jq[q];
    qorig[h] = __float_as_int(qc.w);
    s.x = qc.x;
    s.y = qc.y;
    s.z = qc.z;
    // a lane without a query starts at best = -inf, so its threshold never
    // passes and it flags no product
    s.best = ok[h] ? __builtin_huge_valf() : -__builtin_huge_valf();
    s.idx = 0x7fffffff;
    s.pos = -1;
    if (ok[h] && warm) {
      const int p = jnn[qorig[h]];
      if (p >= 0 && p < J.nc) {
        s.best = d2_contract(s.x, s.y, s.z, jc[p], jc[nc + p], jc[2 * nc + p]);
        s.idx = p;
        if (J.cinv) s.pos = glb(J.cinv)[p];
      }
    }
    s.qn = 0.f;
    s.eps = 0.f;
    set_thr(s);
  }
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
  unsigned issued = 0;          // matrix-core products this wave issued (wave-uniform)
  if (wmin.x <= wmaxc.x) {      // the wave has at least one query
    const int ntiles = (J.nc + kTile - 1) / kTile;
    const int qtiles = (J.nq + kQPerWave - 1) / kQPerWave;
    const int start = (int)((long long)(bx * kWaves + wv) * ntiles / qtiles);   // same Morton rank
    float wbest = wave_best_max(st, ok);
    for (int base = 0; base < ntiles; base += kListMax) {
      const int span = ntiles - base < kListMax ? ntiles - base : kListMax;
      // list the tiles that pass the box test, in visiting order
      int count = 0;
      for (int k0 = 0; k0 < span; k0 += 64) {
        const int k = k0 + lane;
        bool pass = false;
        float lb = 0.f;
        int t = 0;
        if (k < span) {
          t = (start + base + k) % ntiles;
          lb = box_lb(wmin, wmaxc, jcboxes[kBoxStride * t], jcboxes[kBoxStride * t + 1]);
          pass = !(lb * kCullSlack > wbest);
        }
        const unsigned long long m = __ballot(pass);
        const int pos = count + __popcll(m & ((1ull << lane) - 1ull));
        if (pass) {
          wl[pos] = t;
          wlb[pos] = lb;
          wc[pos] = jcboxes[kBoxStride * t + 2];
        }
        count += __popcll(m);
      }
      __builtin_amdgcn_wave_barrier();   // the list is written before it is read
      for (int i = 0; i < count; ++i) {
        // list entries are wave-uniform: keep them (and all tile addressing) scalar
        const float lbi = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wlb[i])));
        if (lbi * kCullSlack > wbest) continue;   // the improved bests rule it out
        const int ti = __builtin_amdgcn_readfirstlane(wl[i]);
        const int c0 = ti * kTile;
        const int nleft = J.nc - c0;
        const bool full = nleft >= kTile;   // wave-uniform
        const int nsub = full ? kCTile / 32 : (nleft + 31) / 32;
        // the tile's A operands (candidate c0 + 32 s + (lane & 31), this lane's
        // half row) and coordinates; full tiles address them from one scalar
        // base with immediate offsets
        uint4 fr[kCTile / 32];
        const float4 cl = wc[i];   // wave-uniform
        const float4 cen = make_float4(
            __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(cl.x))),
            __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(cl.y))),
            __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(cl.z))),
            __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(cl.w))));
        const PDG_GLOBAL uint4 *tp = jpack + 2 * (long long)c0 + 2 * (lane & 31) + half;
        const PDG_GLOBAL float4 *tq = jcc + c0 + lane;
        __builtin_amdgcn_wave_barrier();   // the previous tile's re-rank reads are done
        if (full) {
#pragma unroll
          for (int sidx = 0; sidx < kCTile / 32; ++sidx) fr[sidx] = tp[64 * sidx];
          if (kStage) {   // straight from memory into LDS, 16 B per lane
#pragma unroll
            for (int k = 0; k < kTile / 64; ++k) stage_lds(tq + 64 * k, tc + 64 * k);
          }
        } else {
#pragma unroll
          for (int sidx = 0; sidx < kCTile / 32; ++sidx) {
            const int c = c0 + sidx * 32 + (lane & 31);
            const long long cl = c < J.nc ? c : J.nc - 1;
            fr[sidx] = jpack[2 * cl + half];
            if (c >= J.nc)   // padded rows: n_hi = +inf, so S = +inf
              fr[sidx] = half ? make_uint4(0x7F800000u, 0u, 0u, 0u) : make_uint4(0u, 0u, 0u, 0u);
          }
          if (kStage) {
#pragma unroll
            for (int k = 0; k < kTile / 64; ++k) {
              const int c = c0 + k * 64 + lane;
              stage_lds(jcc + (c < J.nc ? c : J.nc - 1), tc + 64 * k);
            }
          }
        }
        const PDG_GLOBAL float4 *tg = jcc + c0;   // the re-rank's coordinates without staging
#pragma unroll
        for (int h = 0; h < kQB; ++h) enter_tile(st[h], cen, half, bq[h]);
        // The screen proper has no branch: the wave only notes which
        // (step, query block) products hold a row inside some lane's
        // threshold (a ballot, kept in scalar registers), and those are
        // recomputed and re-ranked after the tile.  Thresholds only tighten, so a product not noted
        // cannot hold a better neighbour or a tie later, and a noted one is
        // re-ranked against the tighter threshold.
        const f32x16 z = {};
        unsigned flags = 0;   // bit kQB * step + block (wave-uniform)
        constexpr int kProducts = kQB * kCTile / 32;
        if (full) {
          // software-pipelined: product i + 1 is issued before product i is
          // reduced, so the matrix core and the vector ALU overlap
          f32x16 v = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              *reinterpret_cast<const bf16x8 *>(&fr[0]), bq[0], z, 0, 0, 0);
#pragma unroll
          for (int i = 0; i < kProducts; ++i) {
            f32x16 vn = z;
            if (i + 1 < kProducts)
              vn = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  *reinterpret_cast<const bf16x8 *>(&fr[(i + 1) / kQB]), bq[(i + 1) % kQB], z, 0,
                  0, 0);
            flags |= (__ballot(min16(v) <= st[i % kQB].thr) != 0ull ? 1u : 0u) << i;
            v = vn;
          }
        } else {
#pragma unroll
          for (int sidx = 0; sidx < kCTile / 32; ++sidx) {
            if (sidx < nsub) {
              const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&fr[sidx]);
#pragma unroll
              for (int h = 0; h < kQB; ++h) {
                const f32x16 v = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bq[h], z, 0, 0, 0);
                flags |= (__ballot(min16(v) <= st[h].thr) != 0ull ? 1u : 0u) << (kQB * sidx + h);
              }
            }
          }
        }
        if (flags != 0u) {   // rare: rows inside the error window
          if (kStage) {
            stage_wait();   // the tile's coordinates have reached LDS
            __builtin_amdgcn_wave_barrier();
          }
#pragma unroll
          for (int sidx = 0; sidx < kCTile / 32; ++sidx) {
            const unsigned fs = (flags >> (kQB * sidx)) & ((1u << kQB) - 1u);
            if (sidx < nsub && fs != 0u) {
              const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&fr[sidx]);
#pragma unroll
              for (int h = 0; h < kQB; ++h) {
                if ((fs >> h) & 1u) {
                  ++issued;   // the recomputed product is issued work too
                  const f32x16 v = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bq[h], z, 0, 0, 0);
                  if (kStage)
                    rerank(st[h], v, lane, sidx * 32, nleft, tc, c0);
                  else
                    rerank(st[h], v, lane, sidx * 32, nleft, tg, c0);
                }
              }
            }
          }
        }
        issued += (unsigned)(nsub * kQB);
        wbest = wave_best_max(st, ok);
      }
      __builtin_amdgcn_wave_barrier();   // the list is rebuilt next
    }
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
  // a wave's own box test rules out count nothing)
  if (J.tiles && lane == 0 && issued) atomicAdd(glb(J.tiles), (unsigned long long)issued);
}

// Exact float32 search with the same tile and sub-tile culls and no matrix
// cores (the reference against which the bf16 screen's gain is measured): one
// wave of 64 queries per workgroup, one query per lane; the wave lists and
// walks its candidate tiles as the screen does, keeps the 32-candidate
// sub-tiles whose boxes pass its test, and every lane evaluates the contract
// distance to each of their candidates, read once for the wave through the
// scalar cache.  The counter adds one per 1,024 candidate-query pairs
// evaluated (32 candidates x 32 queries, the unit of the screen's).
__global__ __launch_bounds__(64) void nn_cull_kernel(const ScreenJob *__restrict__ jobs,
                                                         int warm, unsigned qt, unsigned nblk) {
  const unsigned lin = blockIdx.x;
  const unsigned per = gridDim.x / kXcds;
  const unsigned tile = (lin % kXcds) * per + lin / kXcds;
  if (tile >= nblk) return;
  const unsigned bx = tile % qt, by = tile / qt;
  const ScreenJob J = jobs[by];
  const int q0 = bx * 64;
  if (q0 >= J.nq) return;
  const PDG_GLOBAL float4 *jq = glb(J.q);
  const PDG_GLOBAL float4 *jcboxes = glb(J.cboxes);
  const PDG_GLOBAL float *jc = glb(J.c);
  PDG_GLOBAL int *jnn = glb(J.nn);
  __shared__ int wl[kListMax];
  __shared__ float wlb[kListMax];
  const int lane = threadIdx.x;
  const long long nc = J.nc;
  const int q = q0 + lane;
  const bool ok = q < J.nq;
  float4 qc = make_float4(0.f, 0.f, 0.f, 0.f);
  if (ok) qc = jq[q];
  const int qorig = __float_as_int(qc.w);
  float best = __builtin_huge_valf();
  int idx = 0x7fffffff;
  if (ok && warm) {
    const int p = jnn[qorig];
    if (p >= 0 && p < J.nc) {
      best = d2_contract(qc.x, qc.y, qc.z, jc[p], jc[nc + p], jc[2 * nc + p]);
      idx = p;
    }
  }
  float4 wmin = make_float4(ok ? qc.x : __builtin_huge_valf(), ok ? qc.y : __builtin_huge_valf(),
                            ok ? qc.z : __builtin_huge_valf(), 0.f);
  float4 wmaxc = make_float4(ok ? qc.x : -__builtin_huge_valf(), ok ? qc.y : -__builtin_huge_valf(),
                             ok ? qc.z : -__builtin_huge_valf(), 0.f);
  for (int o = 32; o > 0; o >>= 1) {
    wmin.x = fminf(wmin.x, __shfl_xor(wmin.x, o, 64));
    wmin.y = fminf(wmin.y, __shfl_xor(wmin.y, o, 64));
    wmin.z = fminf(wmin.z, __shfl_xor(wmin.z, o, 64));
    wmaxc.x = fmaxf(wmaxc.x, __shfl_xor(wmaxc.x, o, 64));
    wmaxc.y = fmaxf(wmaxc.y, __shfl_xor(wmaxc.y, o, 64));
    wmaxc.z = fmaxf(wmaxc.z, __shfl_xor(wmaxc.z, o, 64));
  }
  auto wave_best = [&]() {
    float m = ok ? best : 0.f;
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(m)));
  };
  unsigned pairs = 0;           // 1,024-pair units evaluated (wave-uniform)
  const int ntiles = (J.nc + kTile - 1) / kTile;
  const int qtiles = (J.nq + 63) / 64;
  const int start = (int)((long long)bx * ntiles / qtiles);
  float wbest = wave_best();
  for (int base = 0; base < ntiles; base += kListMax) {
    const int span = ntiles - base < kListMax ? ntiles - base : kListMax;
    int count = 0;
    for (int k0 = 0; k0 < span; k0 += 64) {
      const int k = k0 + lane;
      bool pass = false;
      float lb = 0.f;
      int t = 0;
      if (k < span) {
        t = (start + base + k) % ntiles;
        lb = box_lb(wmin, wmaxc, jcboxes[kBoxStride * t], jcboxes[kBoxStride * t + 1]);
        pass = !(lb * kCullSlack > wbest);
      }
      const unsigned long long m = __ballot(pass);
      const int pos = count + __popcll(m & ((1ull << lane) - 1ull));
      if (pass) {
        wl[pos] = t;
        wlb[pos] = lb;
      }
      count += __popcll(m);
    }
    __builtin_amdgcn_wave_barrier();
    for (int i = 0; i < count; ++i) {
      const float lbi = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(wlb[i])));
      if (lbi * kCullSlack > wbest) continue;
      const int ti = __builtin_amdgcn_readfirstlane(wl[i]);
      const int c0 = ti * kTile;
      const int nleft = J.nc - c0 < kTile ? J.nc - c0 : kTile;
      // the 32-candidate sub-tiles whose boxes pass the wave's test (lane s
      // tests sub-tile s)
      unsigned sm;
      {
        const int sb = lane & (kSubBoxes - 1);
        const float lbs = box_lb(wmin, wmaxc, jcboxes[kBoxStride * ti + 3 + 2 * sb],
                                 jcboxes[kBoxStride * ti + 4 + 2 * sb]);
        sm = (unsigned)__ballot(!(lbs * kCullSlack > wbest) && 32 * sb < nleft) &
             ((1u << kSubBoxes) - 1u);
      }
      // the candidate is the same for every lane: read it through the scalar
      // cache (the coordinates are read-only in this kernel)
      const PDG_CONST float4 *cp = (const PDG_CONST float4 *)(J.cc + c0);
      // (distance bits, index) as one 64-bit key: distances are >= 0, so the
      // unsigned order of the key is the lowest-index-on-ties order
      unsigned long long key = ((unsigned long long)__float_as_uint(best) << 32) | (unsigned)idx;
      auto visit = [&](const float4 &p) {
        const float d = d2_contract(qc.x, qc.y, qc.z, p.x, p.y, p.z);
        const unsigned long long k =
            ((unsigned long long)__float_as_uint(d) << 32) | (unsigned)__float_as_int(p.w);
        key = k < key ? k : key;
      };
      for (unsigned m = sm; m; m &= m - 1) {
        const int j0 = 32 * __builtin_ctz(m);
        const int j1 = nleft - j0 < 32 ? nleft : j0 + 32;
        int j = j0;
        for (; j + 8 <= j1; j += 8) {
          float4 p[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) p[k] = cp[j + k];
#pragma unroll
          for (int k = 0; k < 8; ++k) visit(p[k]);
        }
        for (; j < j1; ++j) visit(cp[j]);
      }
      best = __uint_as_float((unsigned)(key >> 32));
      idx = (int)(unsigned)key;
      pairs += 2u * (unsigned)__popc(sm);
      wbest = wave_best();
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (ok) jnn[qorig] = idx;
  if (J.tiles && lane == 0 && pairs) atomicAdd(glb(J.tiles), (unsigned long long)pairs);
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

pdg_status launch_nn_cull(const ScreenJob *jobs, int njobs, int max_nq, int warm,
                          hipStream_t st) {
  if (njobs <= 0 || max_nq <= 0) return PDG_OK;
  const unsigned qt = div_up(max_nq, 64);
  const unsigned long long nblk = (unsigned long long)qt * njobs;
  const unsigned long long padded = (nblk + kXcds - 1) / kXcds * kXcds;
  if (padded >= (1ull << 31)) {
    set_error("nn cull: %llu workgroups exceed the launch limit", padded);
    return PDG_EINVAL;
  }
  nn_cull_kernel<<<(unsigned)padded, 64, 0, st>>>(jobs, warm, qt, (unsigned)nblk);
  return launched("nn_cull");
}

}  // namespace pdg
