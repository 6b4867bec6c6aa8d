// Exact grid Sobolev preconditioner (paper Sec. 3.2, Eq. 3) by separable
// DCT-II diagonalisation: g <- (I + lam L)^-2 g per (stack, level, channel).
//
// The orthonormal DCT-II basis C[k][x] = s_k cos(pi k (2x+1) / (2R))
// diagonalises the Laplacian of a path with free ends (eigenvalues
// mu_k = 2 - 2 cos(pi k / R)); the box Laplacian is the Kronecker sum of three
// path Laplacians, so
//     (I + lam L)^-2 = (C x C x C)^T diag((1 + lam (mu_i + mu_j + mu_k))^-2) (C x C x C).
// The step applies C along x, y and z, scales, and applies C^T along z, y, x:
// six in-place passes, each a dense contraction of every grid line with the
// R x R basis, run on the matrix cores as v_mfma_f32_32x32x2_f32 (float32 in,
// float32 accumulate).  The scale is fused into the first inverse pass.
//
// For R <= 128 three fused passes do this (x and y on a z-plane held in LDS;
// forward z, scale and inverse z on 32 z-pencils held in LDS; inverse y and x
// on a plane), i.e. 3 HBM round trips instead of 6.  Larger R use six axis
// passes: a wave owns 32 grid lines and all R outputs of each (R/32 output
// blocks of 32 x 32), reads every input of its lines once, accumulates, then
// writes its lines, so a pass is in place and touches each value once (8 B per
// value and pass).  Lines along y and z are taken 32-contiguous in x (coalesced
// loads and stores); along x the operands are swapped so that the stores stay
// contiguous.  The basis (and its transpose) is read through the caches.
#include "common.h"

namespace pdg {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;   // 4 waves, 32 lines each

struct PassArgs {
  float *g;
  long long stack;             // floats per stack
  long long off;               // float offset of the level
  long long lines;             // batch * 3 * R^2
  const float *mt;             // [in][out] operand matrix (transposed), R x R
  const float *mu;             // [R] Laplacian eigenvalues (scaling pass only)
  int R;
  int axis;                    // 0 x, 1 y, 2 z
  int scale;                   // multiply inputs by (1 + lam (mu_x + mu_y + mu_z))^-2
  float lam;
};

// NB: output blocks of 32 (R <= 32 NB); LDSM: stage the R x R operand in LDS.
// Inputs are fetched kChunk K-steps at a time (independent loads in flight)
// before the matching MFMAs.
constexpr int kChunk = 16;

template <int NB, bool LDSM>
__global__ __launch_bounds__(kThreads) void dct_pass_kernel(PassArgs a) {
  extern __shared__ float smt[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int j = lane & 31, h = lane >> 5;
  const int R = a.R;
  if (LDSM) {
    for (int i = threadIdx.x; i < R * R; i += kThreads) smt[i] = a.mt[i];
    __syncthreads();
  }
  const float *mt = LDSM ? smt : a.mt;
  const long long R2 = (long long)R * R, R3 = R2 * R;
  const long long line = ((long long)blockIdx.x * 4 + wv) * 32 + j;
  const bool valid = line < a.lines;
  long long base = 0, E = 1;
  int lx = 0, ly = 0;
  if (valid) {
    const long long sys = line / R2;
    const long long loc = line - sys * R2;
    base = (sys / 3) * a.stack + a.off + (sys % 3) * R3;
    const int u = (int)(loc / R), v = (int)(loc - (long long)u * R);
    if (a.axis == 0) {             // line (z = u, y = v), elements along x
      base += loc * R;
      E = 1;
    } else if (a.axis == 1) {      // line (z = u, x = v), elements along y
      base += (long long)u * R2 + v;
      E = R;
    } else {                       // line (y = u, x = v), elements along z
      base += (long long)u * R + v;
      E = R2;
      ly = u;
      lx = v;
    }
  }
  float sfix = 0.f;
  if (a.scale && valid) sfix = a.mu[lx] + a.mu[ly];
  f32x16 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = (f32x16){};
  for (int k0 = 0; k0 < R; k0 += 2 * kChunk) {
    float in[kChunk];
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const int xin = k0 + 2 * c + h;
      in[c] = (valid && xin < R) ? a.g[base + xin * E] : 0.f;
    }
    if (a.scale) {
#pragma unroll
      for (int c = 0; c < kChunk; ++c) {
        const int xin = k0 + 2 * c + h;
        if (xin < R) {
          const float d = 1.0f + a.lam * (sfix + a.mu[xin]);
          in[c] = in[c] / (d * d);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const int xin = k0 + 2 * c + h;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int ko = b * 32 + j;
        const float m = (xin < R && ko < R) ? mt[xin * R + ko] : 0.f;
        if (a.axis == 0)
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(in[c], m, acc[b], 0, 0, 0);
        else
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(m, in[c], acc[b], 0, 0, 0);
      }
    }
  }
  // D[i][jj]: lane holds rows i = 8 (r/4) + 4 h + (r%4), column jj = lane & 31
  if (a.axis == 0) {
    // rows are lines of this wave, columns are output elements
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = 8 * (r >> 2) + 4 * h + (r & 3);
        const long long ln = ((long long)blockIdx.x * 4 + wv) * 32 + i;
        const int ko = b * 32 + j;
        if (ln < a.lines && ko < R) {
          const long long sys = ln / R2;
          const long long loc = ln - sys * R2;
          a.g[(sys / 3) * a.stack + a.off + (sys % 3) * R3 + loc * R + ko] = acc[b][r];
        }
      }
  } else {
    // rows are output elements, columns are this lane's line
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ko = b * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (valid && ko < R) a.g[base + (long long)ko * E] = acc[b][r];
      }
  }
}

// ---------------------------------------------------------------------------
// Fused passes for R <= 128.  A block of 8 waves keeps the basis C in LDS
// (pitch R + 1, so that reading it along either index hits distinct banks)
// and loops over its share of the work:
//   plane kernel   one z-plane (R x R, pitch R + 1) in LDS gets two transforms,
//                  along x then along y;
//   pencil kernel  64 z-pencils (R x 64) in LDS get the forward z transform,
//                  the spectral scale and the inverse z transform.
// Outputs are 32 x 32 tiles (v_mfma_f32_32x32x2_f32); wave w owns tiles
// w and w + 8 of the (row band, column tile) grid.  Operands of 8 MFMA steps
// are read from LDS before their matrix-core operations.
struct FusedArgs {
  const float *src;            // input of the pass
  float *dst;                  // output of the pass (may equal src)
  long long stack, off, planes;   // planes = batch * 3 * R
  const float *c;              // C[k][x], R x R row-major
  const float *mu;
  int R;
  float lam;
};

// Adam epilogue of the last inverse pass of one level.
struct AdamEpi {
  float *th, *m, *v;
  float lr, b1, b2, eps;
  const int *step_dev;
  int step_host;
};

constexpr int kFusedMaxR = 128;
constexpr int kBig = 512;              // threads of a fused block (8 waves)
constexpr int kCh = 8;

// acc[p] = sum_k A(k) B_p(k) over k < K (a multiple of 16) for NP tiles that
// share their rows (one row band): this lane's operands are A(k) = a[k * sak]
// and B_p(k) = b[p][k * sbk] (lanes 32..63 take the odd k of each MFMA step).
template <int NP>
__device__ __forceinline__ void band_gemm(int K, const float *a, int sak, const float *const *b,
                                          int sbk, f32x16 (&acc)[NP]) {
  const int h = (threadIdx.x >> 5) & 1;
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = (f32x16){};
#pragma unroll 1
  for (int k0 = 0; k0 < K; k0 += 2 * kCh) {
    float av[kCh], bv[NP][kCh];
#pragma unroll
    for (int c = 0; c < kCh; ++c) {
      const int k = k0 + 2 * c + h;
      av[c] = a[k * sak];
#pragma unroll
      for (int p = 0; p < NP; ++p) bv[p][c] = b[p][k * sbk];
    }
#pragma unroll
    for (int c = 0; c < kCh; ++c)
#pragma unroll
      for (int p = 0; p < NP; ++p)
        acc[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[c], bv[p][c], acc[p], 0, 0, 0);
  }
}

// row of the output held by register r of this lane (column = lane & 31)
__device__ __forceinline__ int trow(int r) {
  const int lane = threadIdx.x & 63;
  return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// C into LDS as sc[k * P + x] for k, x < RP (zero outside R x R)
__device__ __forceinline__ void load_basis(float *sc, const float *c, int R, int RP, int P) {
  for (int i = threadIdx.x; i < RP * RP; i += kBig) {
    const int k = i / RP, x = i % RP;
    sc[k * P + x] = (k < R && x < R) ? c[k * R + x] : 0.f;
  }
}

// sp[(i / w) * pitch + i % w] = in[(i / w) * ld + i % w] for i < n: kLoadU loads in
// flight per thread before their LDS stores
constexpr int kLoadU = 8;
__device__ __forceinline__ void load_rows(float *sp, int pitch, const float *in, long long ld, int w,
                                          int n) {
  for (int i0 = threadIdx.x; i0 < n; i0 += kLoadU * kBig) {
    float v[kLoadU];
#pragma unroll
    for (int u = 0; u < kLoadU; ++u) {
      const int i = i0 + u * kBig;
      v[u] = i < n ? in[(i / w) * ld + i % w] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kLoadU; ++u) {
      const int i = i0 + u * kBig;
      if (i < n) sp[(i / w) * pitch + i % w] = v[u];
    }
  }
}

// Work split of an NT x NC grid of 32 x 32 output tiles over the 8 waves:
// with NT * NC == 16 wave w owns the two tiles (w / 2, 2 (w % 2) + {0, 1})
// of one row band; otherwise tiles w and w + 8, one at a time.
template <int NT, int NC>
struct Split {
  static constexpr bool kPair = NT * NC == 16 && NC % 2 == 0;
  static constexpr int NP = kPair ? 2 : 1;
  static constexpr int kRounds = kPair ? 1 : (NT * NC + 7) / 8;
  // tile of round `rnd` for this wave: (band, first column tile), or false
  __device__ static bool tile(int rnd, int &band, int &ct) {
    const int w = threadIdx.x >> 6;
    if (kPair) {
      constexpr int half = kPair ? NC / 2 : 1;
      band = w / half;
      ct = 2 * (w % half);
      return true;
    }
    const int t = w + 8 * rnd;
    band = t / NC;
    ct = t % NC;
    return t < NT * NC;
  }
};

// Two transforms of z-planes held in LDS (padded to RP = 32 NT with zeros):
// along x, t[y][k] = sum_x in[y][x] M(x, k), then along y,
// out[k'][k] = sum_y M(y, k') t[y][k]; M(in, out) = C[out][in] forward,
// C[in][out] inverse.  The first transform's tiles are written over the plane
// after a barrier; the second's go straight to HBM while the next plane is in
// flight into registers.
template <int NT, bool FULL>
__global__ __launch_bounds__(kBig) void dct_plane_kernel(FusedArgs a, int inverse) {
  using S = Split<NT, NT>;
  constexpr int RP = 32 * NT, P = RP + 1, NP = S::NP;
  extern __shared__ float lds[];
  const int R = FULL ? RP : a.R;     // FULL: R == 32 NT (no partial tiles)
  float *sc = lds;                 // basis, RP x P
  float *sp = lds + RP * P;        // plane, RP x P
  const long long R2 = (long long)R * R, R3 = R2 * R;
  load_basis(sc, a.c, R, RP, P);
  for (int i = threadIdx.x; i < RP * P; i += kBig) sp[i] = 0.f;   // padding stays zero
  const int col = threadIdx.x & 31;
  const int sbx = inverse ? P : 1, say = inverse ? P : 1;
  auto plane_base = [&](long long plane) {
    const long long sys = plane / R, z = plane % R;
    return (sys / 3) * a.stack + a.off + (sys % 3) * R3 + z * R2;
  };
  __syncthreads();
  long long plane = blockIdx.x;
  if (plane < a.planes) load_rows(sp, P, a.src + plane_base(plane), R, R, R * R);
  __syncthreads();
  for (; plane < a.planes; plane += gridDim.x) {
    const long long base = plane_base(plane);
    f32x16 acc[S::kRounds][NP];
#pragma unroll
    for (int rnd = 0; rnd < S::kRounds; ++rnd) {
      int band, ct;
      if (S::tile(rnd, band, ct)) {
        const int i = 32 * band + col;
        const float *bx[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const int j = 32 * (ct + p) + col;
          bx[p] = inverse ? sc + j : sc + j * P;      // B(x = k, k = j) = M(x, j)
        }
        band_gemm<NP>(RP, sp + i * P, 1, bx, sbx, acc[rnd]);   // A(y = i, x = k)
      }
    }
    __syncthreads();
#pragma unroll
    for (int rnd = 0; rnd < S::kRounds; ++rnd) {
      int band, ct;
      if (S::tile(rnd, band, ct)) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const int k = 32 * (ct + p) + col;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int y = 32 * band + trow(r);
            if (FULL || (y < R && k < R)) sp[y * P + k] = acc[rnd][p][r];
          }
        }
      }
    }
    __syncthreads();
    // the next plane is fetched into registers while the second transform runs
    constexpr int kPre = RP * RP / kBig;
    const long long next = plane + gridDim.x;
    float pre[kPre];
    if (next < a.planes) {
      const float *in = a.src + plane_base(next);
#pragma unroll
      for (int e = 0; e < kPre; ++e) {
        const int i = threadIdx.x + e * kBig;
        pre[e] = (FULL || i < R * R) ? in[i] : 0.f;
      }
    }
    float *out = a.dst + base;
#pragma unroll
    for (int rnd = 0; rnd < S::kRounds; ++rnd) {
      int band, ct;
      if (S::tile(rnd, band, ct)) {
        const int i = 32 * band + col;
        const float *by[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) by[p] = sp + 32 * (ct + p) + col;   // B(y = k, k = j)
        f32x16 o[NP];
        band_gemm<NP>(RP, inverse ? sc + i : sc + i * P, say, by, P, o);   // A(k' = i, y = k)
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const int k = 32 * (ct + p) + col;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int kk = 32 * band + trow(r);
            if (FULL || (kk < R && k < R)) out[kk * R + k] = o[p][r];
          }
        }
      }
    }
    __syncthreads();
    if (next < a.planes) {
#pragma unroll
      for (int e = 0; e < kPre; ++e) {
        const int i = threadIdx.x + e * kBig;
        if (FULL || i < R * R) sp[(i / R) * P + i % R] = pre[e];
      }
    }
    __syncthreads();
  }
}

// Forward z, scale by (1 + lam (mu_x + mu_y + mu_z))^-2, inverse z for groups
// of 64 consecutive (y, x) pencils of one system, in place on dst.
constexpr int kPencils = 64;
constexpr int kPP = kPencils + 1;      // LDS pitch of a pencil row

template <int NT, bool FULL>
__global__ __launch_bounds__(kBig) void dct_pencil_kernel(FusedArgs a) {
  using S = Split<NT, kPencils / 32>;
  constexpr int RP = 32 * NT, P = RP + 1, NP = S::NP;
  extern __shared__ float lds[];
  const int R = FULL ? RP : a.R;     // FULL: R == 32 NT (R^2 is a multiple of 64)
  float *sc = lds;                 // basis, RP x P
  float *sq = lds + RP * P;        // pencils, RP x kPP (rows >= R stay zero)
  const long long R2 = (long long)R * R, R3 = R2 * R;
  const long long groups = (R2 + kPencils - 1) / kPencils;   // per system
  const long long total = a.planes / R * groups;
  load_basis(sc, a.c, R, RP, P);
  for (int i = threadIdx.x; i < RP * kPP; i += kBig) sq[i] = 0.f;
  const int col = threadIdx.x & 31;
  const int r2 = (int)R2;
  auto group_ptr = [&](long long g, int &nl) {
    const long long sys = g / groups;
    const long long line0 = (g % groups) * kPencils;   // first (y, x) line = y * R + x
    nl = R2 - line0 < kPencils ? (int)(R2 - line0) : kPencils;
    return a.dst + (sys / 3) * a.stack + a.off + (sys % 3) * R3 + line0;
  };
  constexpr int kPre = RP * kPencils / kBig;
  float pre[kPre];
  auto fetch = [&](long long g) {
    int nl;
    const float *in = group_ptr(g, nl);
#pragma unroll
    for (int e = 0; e < kPre; ++e) {
      const int i = threadIdx.x + e * kBig, z = i / kPencils, j = i % kPencils;
      pre[e] = (FULL || (z < R && j < nl)) ? in[z * r2 + j] : 0.f;
    }
  };
  if (blockIdx.x < total) fetch(blockIdx.x);
  for (long long g = blockIdx.x; g < total; g += gridDim.x) {
    const long long line0 = (g % groups) * kPencils;
    int nl;
    float *d0 = group_ptr(g, nl);
    __syncthreads();               // the previous group's reads of sq are done
#pragma unroll
    for (int e = 0; e < kPre; ++e) {
      const int i = threadIdx.x + e * kBig, z = i / kPencils, j = i % kPencils;
      if (FULL || z < R) sq[z * kPP + j] = pre[e];
    }
    __syncthreads();
    if (g + gridDim.x < total) fetch(g + gridDim.x);   // in flight during this group
    f32x16 acc[S::kRounds][NP];
#pragma unroll
    for (int rnd = 0; rnd < S::kRounds; ++rnd) {
      int band, ct;
      if (S::tile(rnd, band, ct)) {
        const float *bp[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) bp[p] = sq + 32 * (ct + p) + col;   // B(z = k, j)
        band_gemm<NP>(RP, sc + (32 * band + col) * P, 1, bp, kPP, acc[rnd]);   // C[kz][z]
      }
    }
    __syncthreads();
#pragma unroll
    for (int rnd = 0; rnd < S::kRounds; ++rnd) {
      int band, ct;
      if (S::tile(rnd, band, ct)) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const int j = 32 * (ct + p) + col;
          const int ln = (int)line0 + j;
          float sxy = 0.f;
          if (FULL || j < nl) sxy = a.mu[ln / R] + a.mu[ln % R];
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int kz = 32 * band + trow(r);
            if (FULL || kz < R) {
              const float d = 1.0f + a.lam * (sxy + a.mu[kz]);
              sq[kz * kPP + j] = (FULL || j < nl) ? acc[rnd][p][r] / (d * d) : 0.f;
            }
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int rnd = 0; rnd < S::kRounds; ++rnd) {
      int band, ct;
      if (S::tile(rnd, band, ct)) {
        const float *bp[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) bp[p] = sq + 32 * (ct + p) + col;
        f32x16 o[NP];
        band_gemm<NP>(RP, sc + 32 * band + col, P, bp, kPP, o);   // A(z = i, kz = k) = C[kz][z]
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const int j = 32 * (ct + p) + col;
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int z = 32 * band + trow(r);
            if (FULL || (z < R && j < nl)) d0[z * r2 + j] = o[p][r];
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Even/odd form for R = 64 and 128.  C[k][R-1-x] = (-1)^k C[k][x], so a
// forward transform needs only the left half of C on folded inputs,
//   out[2p] = sum_{x<R/2} C[2p][x] (in[x] + in[R-1-x]),
//   out[2p+1] = sum_{x<R/2} C[2p+1][x] (in[x] - in[R-1-x]),
// and an inverse one two half products combined,
//   E[x] = sum_p C[2p][x] s[2p], O[x] = sum_p C[2p+1][x] s[2p+1],
//   out[x] = E[x] + O[x], out[R-1-x] = E[x] - O[x]   (x < R/2):
// half the matrix-core work of the dense form.  Between the passes the spectra
// are kept in the order [even frequencies | odd frequencies] along each axis
// (index p stands for frequency 2p below R/2 and 2(p - R/2) + 1 above), which
// the scale and the inverse passes read consistently.  LDS holds the two half
// bases Ce[p][x] = C[2p][x], Co[p][x] = C[2p+1][x] (x < R/2, pitch R/2 + 1).
constexpr int kPencilsEO = 128;
constexpr int kPQ = kPencilsEO + 1;

__device__ __forceinline__ void load_basis_eo(float *sh, const float *c, int R, int RH, int PH) {
  for (int i = threadIdx.x; i < R * RH; i += kBig) {
    const int k = i / RH, x = i % RH;
    sh[(k & 1) * RH * PH + (k >> 1) * PH + x] = c[k * R + x];
  }
}

__device__ __forceinline__ float mu_perm(const float *mu, int p, int RH) {
  return mu[p < RH ? 2 * p : 2 * (p - RH) + 1];
}

// acc[p] = sum_k A(k) B_p(k) over k < K (a multiple of 16) with
//   A(k) = a0[k sa] (+ sga a1[-k sa] with FA),  B_p(k) = b0[p][k sb] (+ sgb b1[p][-k sb] with FB);
// the NP tiles share A.
template <int NP, bool FA, bool FB>
__device__ __forceinline__ void fold_gemm(int K, const float *a0, const float *a1, int sa, float sga,
                                          const float *const *b0, const float *const *b1, int sb,
                                          float sgb, f32x16 (&acc)[NP]) {
  const int h = (threadIdx.x >> 5) & 1;
#pragma unroll
  for (int p = 0; p < NP; ++p) acc[p] = (f32x16){};
#pragma unroll 1
  for (int k0 = 0; k0 < K; k0 += 2 * kCh) {
    float av[kCh], bv[NP][kCh];
#pragma unroll
    for (int c = 0; c < kCh; ++c) {
      const int k = k0 + 2 * c + h;
      av[c] = FA ? a0[k * sa] + sga * a1[-k * sa] : a0[k * sa];
#pragma unroll
      for (int p = 0; p < NP; ++p) bv[p][c] = FB ? b0[p][k * sb] + sgb * b1[p][-k * sb] : b0[p][k * sb];
    }
#pragma unroll
    for (int c = 0; c < kCh; ++c)
#pragma unroll
      for (int p = 0; p < NP; ++p)
        acc[p] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[c], bv[p][c], acc[p], 0, 0, 0);
  }
}

// e = sum_k ae[k sa] be[k sb], o = sum_k ao[k sa] bo[k sb] over k < K.
__device__ __forceinline__ void eo_gemm(int K, const float *ae, const float *ao, int sa,
                                        const float *be, const float *bo, int sb, f32x16 &e,
                                        f32x16 &o) {
  const int h = (threadIdx.x >> 5) & 1;
  e = (f32x16){};
  o = (f32x16){};
#pragma unroll 1
  for (int k0 = 0; k0 < K; k0 += 2 * kCh) {
    float a[2][kCh], b[2][kCh];
#pragma unroll
    for (int c = 0; c < kCh; ++c) {
      const int k = k0 + 2 * c + h;
      a[0][c] = ae[k * sa];
      b[0][c] = be[k * sb];
      a[1][c] = ao[k * sa];
      b[1][c] = bo[k * sb];
    }
#pragma unroll
    for (int c = 0; c < kCh; ++c) {
      e = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][c], b[0][c], e, 0, 0, 0);
      o = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1][c], b[1][c], o, 0, 0, 0);
    }
  }
}

// Forward x and y transforms of z-planes: natural (y, x) in, spectra (q, p) out.
template <int NT>
__global__ __launch_bounds__(kBig) void dct_plane_eo_fwd_kernel(FusedArgs a) {
  constexpr int R = 32 * NT, RH = R / 2, P = R + 1, PH = RH + 1, NH = NT / 2;
  constexpr int NP = NT == 4 ? 2 : 1;          // tiles per wave (one row band)
  extern __shared__ float lds[];
  float *sh = lds;                             // Ce, Co
  float *sp = lds + 2 * RH * PH;               // plane, R x P
  constexpr long long R2 = (long long)R * R, R3 = R2 * R;
  load_basis_eo(sh, a.c, R, RH, PH);
  const int w = threadIdx.x >> 6, col = threadIdx.x & 31;
  const bool act = NT == 4 || w < 4;
  const int band = w >> 1, ct0 = NT == 4 ? 2 * (w & 1) : (w & 1);
  auto plane_base = [&](long long plane) {
    const long long sys = plane / R, z = plane % R;
    return (sys / 3) * a.stack + a.off + (sys % 3) * R3 + z * R2;
  };
  long long plane = blockIdx.x;
  if (plane < a.planes) load_rows(sp, P, a.src + plane_base(plane), R, R, R * R);
  __syncthreads();
  for (; plane < a.planes; plane += gridDim.x) {
    const long long base = plane_base(plane);
    f32x16 acc[NP];
    if (act) {
      // along x: t[y][p] = sum_{x<RH} (in[y][x] +- in[y][R-1-x]) C[k(p)][x]
      const float sg = ct0 < NH ? 1.f : -1.f;
      const float *a0 = sp + (32 * band + col) * P;
      const float *b0[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int pc = 32 * (ct0 + p) + col;
        b0[p] = sh + (pc < RH ? 0 : RH * PH) + (pc % RH) * PH;     // C[k(pc)][x] along x
      }
      fold_gemm<NP, true, false>(RH, a0, a0 + R - 1, 1, sg, b0, b0, 1, 0.f, acc);
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int pc = 32 * (ct0 + p) + col;
#pragma unroll
        for (int r = 0; r < 16; ++r) sp[(32 * band + trow(r)) * P + pc] = acc[p][r];
      }
    }
    __syncthreads();
    constexpr int kPre = R * R / kBig;
    const long long next = plane + gridDim.x;
    float pre[kPre];
    if (next < a.planes) {
      const float *in = a.src + plane_base(next);
#pragma unroll
      for (int e = 0; e < kPre; ++e) pre[e] = in[threadIdx.x + e * kBig];
    }
    if (act) {
      // along y: out[q][p] = sum_{y<RH} C[k(q)][y] (t[y][p] +- t[R-1-y][p])
      const float sg = band < NH ? 1.f : -1.f;
      const int qr = 32 * band + col;
      const float *a0 = sh + (qr < RH ? 0 : RH * PH) + (qr % RH) * PH;   // C[k(q)][y] along y
      const float *b0[NP], *b1[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int pc = 32 * (ct0 + p) + col;
        b0[p] = sp + pc;
        b1[p] = sp + (R - 1) * P + pc;
      }
      fold_gemm<NP, false, true>(RH, a0, a0, 1, 0.f, b0, b1, P, sg, acc);
      float *out = a.dst + base;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int pc = 32 * (ct0 + p) + col;
#pragma unroll
        for (int r = 0; r < 16; ++r) out[(32 * band + trow(r)) * R + pc] = acc[p][r];
      }
    }
    __syncthreads();
    if (next < a.planes) {
      float *pb = sp + (threadIdx.x / R) * P + threadIdx.x % R;   // kBig is a multiple of R
#pragma unroll
      for (int e = 0; e < kPre; ++e) pb[e * (kBig / R) * P] = pre[e];
    }
    __syncthreads();
  }
}

// Inverse y and x transforms: spectra (q, p) in, natural (y, x) out.  With
// ADAM the outputs are not stored: they drive an Adam step of the
// parameters at the same positions instead: each thread loads its float4 groups of
// parameters and first moments when the plane starts and of second moments
// before the y product, so that the loads overlap the products, and the y
// products reach the linear epilogue through LDS.
template <int NT, bool ADAM>
__global__ __launch_bounds__(kBig) void dct_plane_eo_inv_kernel(FusedArgs a, AdamEpi ad) {
  constexpr int R = 32 * NT, RH = R / 2, P = R + 1, PH = RH + 1, NH = NT / 2;
  constexpr int kV = R * R / (4 * kBig);        // float4 groups per thread and plane
  extern __shared__ float lds[];
  float *sh = lds;
  float *sp = lds + 2 * RH * PH;
  constexpr long long R2 = (long long)R * R, R3 = R2 * R;
  float bc1 = 1.f, bc2 = 1.f;
  if constexpr (ADAM) {
    __shared__ float sbc[2];
    adam_bias(ad.b1, ad.b2, ad.step_dev, ad.step_host, sbc);
    bc1 = sbc[0];
    bc2 = sbc[1];
  }
  load_basis_eo(sh, a.c, R, RH, PH);
  const int w = threadIdx.x >> 6, col = threadIdx.x & 31;
  const bool act = w < NT * NH;                // NT * NH = NH * NT items per phase
  auto plane_base = [&](long long plane) {
    const long long sys = plane / R, z = plane % R;
    return (sys / 3) * a.stack + a.off + (sys % 3) * R3 + z * R2;
  };
  long long plane = blockIdx.x;
  if (plane < a.planes) load_rows(sp, P, a.src + plane_base(plane), R, R, R * R);
  __syncthreads();
  for (; plane < a.planes; plane += gridDim.x) {
    const long long base = plane_base(plane);
    float4 th[ADAM ? kV : 1], mo[ADAM ? kV : 1], vo[ADAM ? kV : 1];
    if constexpr (ADAM) {
#pragma unroll
      for (int k = 0; k < kV; ++k) {
        const unsigned i = 4u * (threadIdx.x + k * kBig);
        th[k] = *reinterpret_cast<const float4 *>(ad.th + base + i);
        mo[k] = *reinterpret_cast<const float4 *>(ad.m + base + i);
      }
    }
    f32x16 e, o;
    // along x (item: spectral row band qb, spatial column tile xt < NH):
    // t[q][x] = E + O, t[q][R-1-x] = E - O
    const int qb = w / NH, xt = w % NH;
    if (act) {
      const float *arow = sp + (32 * qb + col) * P;
      eo_gemm(RH, arow, arow + RH, 1, sh + 32 * xt + col, sh + RH * PH + 32 * xt + col, PH, e, o);
    }
    __syncthreads();
    if (act) {
      const int x = 32 * xt + col;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int q = 32 * qb + trow(r);
        sp[q * P + x] = e[r] + o[r];
        sp[q * P + R - 1 - x] = e[r] - o[r];
      }
    }
    __syncthreads();
    constexpr int kPre = R * R / kBig;
    const long long next = plane + gridDim.x;
    float pre[kPre];
    auto prefetch = [&]() {
      if (next < a.planes) {
        const float *in = a.src + plane_base(next);
#pragma unroll
        for (int k = 0; k < kPre; ++k) pre[k] = in[threadIdx.x + k * kBig];
      }
    };
    if constexpr (!ADAM) prefetch();           // (with ADAM after the y product: registers)
    if constexpr (ADAM) {                      // second moments: one product ahead
#pragma unroll
      for (int k = 0; k < kV; ++k)
        vo[k] = *reinterpret_cast<const float4 *>(ad.v + base + 4u * (threadIdx.x + k * kBig));
    }
    // along y (item: spatial row band yb < NH, column tile xc):
    // out[y][x] = E + O, out[R-1-y][x] = E - O
    const int yb = w / NT, xc = w % NT;
    if (act) {
      const int y = 32 * yb + col;
      eo_gemm(RH, sh + y, sh + RH * PH + y, PH, sp + 32 * xc + col, sp + RH * P + 32 * xc + col, P,
              e, o);
    }
    if constexpr (ADAM) {
      prefetch();
      __syncthreads();                         // every product has read sp
      if (act) {
        // rows 32 yb + trow(r) and R - 1 - (32 yb + trow(r)), trow(r) =
        // 4 (lane / 32) + c_r with c_r = 8 (r / 4) + r % 4 in 0..27: two lane
        // bases and compile-time offsets
        const int h4 = 4 * ((threadIdx.x & 63) >> 5);
        float *top = sp + (32 * yb + h4) * P + 32 * xc + col;
        float *bot = sp + (R - 1 - 32 * yb - h4 - 27) * P + 32 * xc + col;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int cr = 8 * (r >> 2) + (r & 3);
          top[cr * P] = e[r] + o[r];
          bot[(27 - cr) * P] = e[r] - o[r];
        }
      }
      __syncthreads();
      // thread's group k starts at row (4 t) / R + k (4 kBig / R), column (4 t) % R
      const float *gb = sp + (4 * threadIdx.x / R) * P + (4 * threadIdx.x) % R;
#pragma unroll
      for (int k = 0; k < kV; ++k) {
        const unsigned i = 4u * (threadIdx.x + k * kBig);
        const float *gr = gb + k * (4 * kBig / R) * P;
        const float4 gv = make_float4(gr[0], gr[1], gr[2], gr[3]);
        th[k].x = adam_one(ad.b1, ad.b2, ad.eps, ad.lr, bc1, bc2, gv.x, mo[k].x, vo[k].x, th[k].x);
        th[k].y = adam_one(ad.b1, ad.b2, ad.eps, ad.lr, bc1, bc2, gv.y, mo[k].y, vo[k].y, th[k].y);
        th[k].z = adam_one(ad.b1, ad.b2, ad.eps, ad.lr, bc1, bc2, gv.z, mo[k].z, vo[k].z, th[k].z);
        th[k].w = adam_one(ad.b1, ad.b2, ad.eps, ad.lr, bc1, bc2, gv.w, mo[k].w, vo[k].w, th[k].w);
        *reinterpret_cast<float4 *>(ad.th + base + i) = th[k];
        *reinterpret_cast<float4 *>(ad.m + base + i) = mo[k];
        *reinterpret_cast<float4 *>(ad.v + base + i) = vo[k];
      }
    } else if (act) {
      const int x = 32 * xc + col;
      float *out = a.dst + base;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int yy = 32 * yb + trow(r);
        out[yy * R + x] = e[r] + o[r];
        out[(R - 1 - yy) * R + x] = e[r] - o[r];
      }
    }
    __syncthreads();
    if (next < a.planes) {
      float *pb = sp + (threadIdx.x / R) * P + threadIdx.x % R;   // kBig is a multiple of R
#pragma unroll
      for (int k = 0; k < kPre; ++k) pb[k * (kBig / R) * P] = pre[k];
    }
    __syncthreads();
  }
}

// Forward z, spectral scale, inverse z for groups of 128 (qy, qx) lines of
// one system, in place on dst (spectral order in y and x, natural z).
template <int NT>
__global__ __launch_bounds__(kBig) void dct_pencil_eo_kernel(FusedArgs a) {
  constexpr int R = 32 * NT, RH = R / 2, PH = RH + 1, NH = NT / 2, JT = kPencilsEO / 32;
  constexpr int NP = NT == 4 ? 2 : 1;
  extern __shared__ float lds[];
  float *sh = lds;
  float *sq = lds + 2 * RH * PH;               // R x kPQ
  constexpr long long R2 = (long long)R * R, R3 = R2 * R;
  constexpr long long groups = R2 / kPencilsEO;   // per system
  const long long total = a.planes / R * groups;
  load_basis_eo(sh, a.c, R, RH, PH);
  const int w = threadIdx.x >> 6, col = threadIdx.x & 31;
  // forward tiles: row band fb, column tiles fc0 .. fc0 + NP - 1
  const int fb = NT == 4 ? (w >> 1) : (w >> 2), fc0 = NT == 4 ? 2 * (w & 1) : (w & 3);
  // inverse items: spatial row band ib < NH, column tile ic
  const int ib = w / JT, ic = w % JT;
  const bool iact = w < NH * JT;
  auto group_ptr = [&](long long g) {
    const long long sys = g / groups;
    return a.dst + (sys / 3) * a.stack + a.off + (sys % 3) * R3 + (g % groups) * kPencilsEO;
  };
  constexpr int kPre = R * kPencilsEO / kBig;
  float pre[kPre];
  auto fetch = [&](long long g) {
    const float *in = group_ptr(g);
#pragma unroll
    for (int e = 0; e < kPre; ++e) {
      const int i = threadIdx.x + e * kBig;
      pre[e] = in[(i / kPencilsEO) * R2 + i % kPencilsEO];
    }
  };
  if (blockIdx.x < total) fetch(blockIdx.x);
  for (long long g = blockIdx.x; g < total; g += gridDim.x) {
    const long long line0 = (g % groups) * kPencilsEO;
    float *d0 = group_ptr(g);
    __syncthreads();               // the previous group's reads of sq are done
#pragma unroll
    for (int e = 0; e < kPre; ++e) {
      const int i = threadIdx.x + e * kBig;
      sq[(i / kPencilsEO) * kPQ + i % kPencilsEO] = pre[e];
    }
    __syncthreads();
    if (g + gridDim.x < total) fetch(g + gridDim.x);   // in flight during this group
    // forward z: F[qz][j] = sum_{z<RH} C[k(qz)][z] (s[z][j] +- s[R-1-z][j])
    f32x16 acc[NP];
    {
      const float sg = fb < NH ? 1.f : -1.f;
      const int qr = 32 * fb + col;
      const float *a0 = sh + (qr < RH ? 0 : RH * PH) + (qr % RH) * PH;
      const float *b0[NP], *b1[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const int j = 32 * (fc0 + p) + col;
        b0[p] = sq + j;
        b1[p] = sq + (R - 1) * kPQ + j;
      }
      fold_gemm<NP, false, true>(RH, a0, a0, 1, 0.f, b0, b1, kPQ, sg, acc);
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int j = 32 * (fc0 + p) + col;
      const int ln = (int)line0 + j;                 // qy * R + qx
      const float sxy = mu_perm(a.mu, ln / R, RH) + mu_perm(a.mu, ln % R, RH);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int qz = 32 * fb + trow(r);
        const float d = 1.0f + a.lam * (sxy + mu_perm(a.mu, qz, RH));
        sq[qz * kPQ + j] = acc[p][r] / (d * d);
      }
    }
    __syncthreads();
    // inverse z: out[z] = E + O, out[R-1-z] = E - O
    if (iact) {
      f32x16 e, o;
      const int z = 32 * ib + col, j = 32 * ic + col;
      eo_gemm(RH, sh + z, sh + RH * PH + z, PH, sq + j, sq + RH * kPQ + j, kPQ, e, o);
      const int r2 = (int)R2;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int zz = 32 * ib + trow(r);
        d0[zz * r2 + j] = e[r] + o[r];
        d0[(R - 1 - zz) * r2 + j] = e[r] - o[r];
      }
    }
  }
}

template <int NT>
pdg_status eo_level(const FusedArgs &f0, const AdamEpi *ad, hipStream_t st) {
  constexpr int R = 32 * NT, RH = R / 2;
  const size_t plane = (size_t)(2 * RH * (RH + 1) + R * (R + 1)) * sizeof(float);
  const size_t pencil = (size_t)(2 * RH * (RH + 1) + R * kPQ) * sizeof(float);
  static bool attrs = false;
  if (!attrs) {
    PDG_TRY_HIP(hipFuncSetAttribute((const void *)dct_plane_eo_fwd_kernel<NT>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)plane));
    PDG_TRY_HIP(hipFuncSetAttribute((const void *)dct_plane_eo_inv_kernel<NT, false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)plane));
    PDG_TRY_HIP(hipFuncSetAttribute((const void *)dct_plane_eo_inv_kernel<NT, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)plane));
    PDG_TRY_HIP(hipFuncSetAttribute((const void *)dct_pencil_eo_kernel<NT>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)pencil));
    attrs = true;
  }
  FusedArgs f = f0;
  const long long groups = f.planes / R * ((long long)R * R / kPencilsEO);
  const unsigned gp = (unsigned)(f.planes < 2048 ? f.planes : 2048);
  const unsigned gg = (unsigned)(groups < 2048 ? groups : 2048);
  dct_plane_eo_fwd_kernel<NT><<<gp, kBig, plane, st>>>(f);
  PDG_TRY(launched("dct_plane_eo_fwd"));
  f.src = f.dst;
  dct_pencil_eo_kernel<NT><<<gg, kBig, pencil, st>>>(f);
  PDG_TRY(launched("dct_pencil_eo"));
  if (ad) {
    dct_plane_eo_inv_kernel<NT, true><<<gp, kBig, plane, st>>>(f, *ad);
  } else {
    AdamEpi none;
    memset(&none, 0, sizeof none);
    dct_plane_eo_inv_kernel<NT, false><<<gp, kBig, plane, st>>>(f, none);
  }
  return launched("dct_plane_eo_inv");
}

int padded(int R) { return 32 * ((R + 31) / 32); }
size_t plane_lds(int R) { return (size_t)2 * padded(R) * (padded(R) + 1) * sizeof(float); }
size_t pencil_lds(int R) { return (size_t)(padded(R) * (padded(R) + 1) + padded(R) * kPP) * sizeof(float); }

template <int NT, bool FULL>
pdg_status fused_level(const FusedArgs &f0, hipStream_t st) {
  static bool attrs = false;
  if (!attrs) {
    PDG_TRY_HIP(hipFuncSetAttribute((const void *)dct_plane_kernel<NT, FULL>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)plane_lds(32 * NT)));
    PDG_TRY_HIP(hipFuncSetAttribute((const void *)dct_pencil_kernel<NT, FULL>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)pencil_lds(32 * NT)));
    attrs = true;
  }
  FusedArgs f = f0;
  const int R = f.R;
  const long long groups = f.planes / R * (((long long)R * R + kPencils - 1) / kPencils);
  const unsigned gp = (unsigned)(f.planes < 2048 ? f.planes : 2048);
  const unsigned gg = (unsigned)(groups < 2048 ? groups : 2048);
  dct_plane_kernel<NT, FULL><<<gp, kBig, plane_lds(R), st>>>(f, 0);
  PDG_TRY(launched("dct_plane"));
  f.src = f.dst;
  dct_pencil_kernel<NT, FULL><<<gg, kBig, pencil_lds(R), st>>>(f);
  PDG_TRY(launched("dct_pencil"));
  dct_plane_kernel<NT, FULL><<<gp, kBig, plane_lds(R), st>>>(f, 1);
  return launched("dct_plane");
}

template <int NT>
pdg_status fused_level(const FusedArgs &f, hipStream_t st) {
  return f.R == 32 * NT ? fused_level<NT, true>(f, st) : fused_level<NT, false>(f, st);
}

// basis C[k][x] (row-major), its transpose, and mu_k, in float64 then rounded
__global__ void dct_basis_kernel(int R, float *c, float *ct, float *mu) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < R * R) {
    const int k = idx / R, x = idx % R;
    const double s = k == 0 ? sqrt(1.0 / R) : sqrt(2.0 / R);
    const float v = (float)(s * cos(M_PI * (double)k * (2.0 * x + 1.0) / (2.0 * R)));
    c[k * R + x] = v;
    ct[x * R + k] = v;
  }
  if (idx < R) mu[idx] = (float)(2.0 - 2.0 * cos(M_PI * (double)idx / (double)R));
}

template <int NB>
pdg_status launch_pass(const PassArgs &a, hipStream_t st) {
  const long long blocks = (a.lines + 127) / 128;
  if (a.R <= 128) {
    const size_t shmem = (size_t)a.R * a.R * sizeof(float);
    dct_pass_kernel<NB, true><<<(unsigned)blocks, kThreads, shmem, st>>>(a);
  } else {
    dct_pass_kernel<NB, false><<<(unsigned)blocks, kThreads, 0, st>>>(a);
  }
  return launched("dct_pass");
}

pdg_status pass(const PassArgs &a, hipStream_t st) {
  switch ((a.R + 31) / 32) {
    case 1: return launch_pass<1>(a, st);
    case 2: return launch_pass<2>(a, st);
    case 3: return launch_pass<3>(a, st);
    case 4: return launch_pass<4>(a, st);
    case 5: return launch_pass<5>(a, st);
    case 6: return launch_pass<6>(a, st);
    case 7: return launch_pass<7>(a, st);
    case 8: return launch_pass<8>(a, st);
    default:
      set_error("DCT preconditioner supports R <= 256 (got %d)", a.R);
      return PDG_EUNSUPPORTED;
  }
}


}  // namespace

size_t dct_bytes(const GridDev &g) {
  size_t b = 0;
  for (int l = 0; l < g.levels; ++l) {
    const size_t R = g.res[l];
    b += 2 * a256(R * R * 4) + a256(R * 4);
  }
  return b;
}

pdg_status dct_basis(const GridDev &g, void *ws, hipStream_t st) {
  char *w = (char *)ws;
  for (int l = 0; l < g.levels; ++l) {
    const int R = g.res[l];
    float *c = (float *)w;
    w += a256((size_t)R * R * 4);
    float *ct = (float *)w;
    w += a256((size_t)R * R * 4);
    float *mu = (float *)w;
    w += a256((size_t)R * 4);
    dct_basis_kernel<<<div_up((long long)R * R, 256), 256, 0, st>>>(R, c, ct, mu);
    PDG_TRY(launched("dct_basis"));
  }
  return PDG_OK;
}

pdg_status run_dct(const GridDev &g, int batch, const float *lam, const float *src, float *data,
                   const void *ws, hipStream_t st, const AdamFuse *adam, unsigned *fused) {
  if (fused) *fused = 0u;
  // Out of place only when every level runs the fused passes (whose first
  // pass reads src); otherwise copy once and work in place.
  bool fused_all = true;
  for (int l = 0; l < g.levels; ++l)
    fused_all = fused_all && g.res[l] > 1 && g.res[l] <= kFusedMaxR && lam[l] != 0.0f;
  if (src != data && !fused_all) {
    PDG_TRY(launch_copy(data, src, (long long)batch * g.size, st));
    src = data;
  }
  const char *w = (const char *)ws;
  for (int l = 0; l < g.levels; ++l) {
    const int R = g.res[l];
    const float *c = (const float *)w;
    w += a256((size_t)R * R * 4);
    const float *ct = (const float *)w;
    w += a256((size_t)R * R * 4);
    const float *mu = (const float *)w;
    w += a256((size_t)R * 4);
    if (R == 1 || lam[l] == 0.0f) continue;   // identity: L = 0 on one cell, or lam = 0
    if (R <= kFusedMaxR) {
      FusedArgs f;
      f.src = src;
      f.dst = data;
      f.stack = g.size;
      f.off = g.off[l];
      f.planes = (long long)batch * 3 * R;
      f.c = c;
      f.mu = mu;
      f.R = R;
      f.lam = lam[l];
      if (R == 128 || R == 64) {
        AdamEpi ad;
        if (adam) {
          ad.th = adam->th;
          ad.m = adam->m;
          ad.v = adam->v;
          ad.lr = adam->lv.lr[l];
          ad.b1 = adam->b1;
          ad.b2 = adam->b2;
          ad.eps = adam->eps;
          ad.step_dev = adam->step_dev;
          ad.step_host = adam->step_host;
          if (fused) *fused |= 1u << l;
        }
        if (R == 128)
          PDG_TRY(eo_level<4>(f, adam ? &ad : nullptr, st));
        else
          PDG_TRY(eo_level<2>(f, adam ? &ad : nullptr, st));
        continue;
      }
      switch ((R + 31) / 32) {
        case 1: PDG_TRY(fused_level<1>(f, st)); break;
        case 2: PDG_TRY(fused_level<2>(f, st)); break;
        case 3: PDG_TRY(fused_level<3>(f, st)); break;
        default: PDG_TRY(fused_level<4>(f, st)); break;
      }
      continue;
    }
    PassArgs a;
    a.g = data;
    a.stack = g.size;
    a.off = g.off[l];
    a.lines = (long long)batch * 3 * R * R;
    a.mu = mu;
    a.R = R;
    a.lam = lam[l];
    a.scale = 0;
    // forward: out[k] = sum_x C[k][x] in[x]; operand stored [in][out] = C^T
    a.mt = ct;
    for (int axis = 0; axis < 3; ++axis) {
      a.axis = axis;
      PDG_TRY(pass(a, st));
    }
    // inverse: out[x] = sum_k C[k][x] in[k]; operand [in][out] = C; scale first
    a.mt = c;
    for (int axis = 2; axis >= 0; --axis) {
      a.axis = axis;
      a.scale = axis == 2;
      PDG_TRY(pass(a, st));
    }
  }
  return PDG_OK;
}

}  // namespace pdg
