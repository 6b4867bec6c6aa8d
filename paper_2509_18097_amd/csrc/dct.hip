// Exact grid Sobolev preconditioner (paper Sec. 3.2, Eq. 3) by separable
// DCT-II diagonalisation: g <- (I + lam L)^-2 g per (stack, level, channel).
//
// The orthonormal DCT-II basis C[k][x] = s_k cos(pi k (2x+1) / (2R))
// diagonalises the Laplacian of a path with free ends (eigenvalues
// mu_k = 2 - 2 cos(pi k / R)); the box Laplacian is the Kronecker sum of three
// path Laplacians, so
//     (I + lam L)^-2 = (C x C x C)^T diag((1 + lam (mu_i + mu_j + mu_k))^-2) (C x C x C).
// The step applies C along x, y and z, scales, and applies C^T along z, y, x.
// Three forms:
//   R = 16, 32, 64, 128 (the step's levels): three passes over
//     HBM (x and y on a z-plane held in LDS; forward z, scale and inverse z on
//     128 z-pencils held in LDS; inverse y and x on a plane), each line
//     transformed by fast factorised transforms on one thread's registers, so
//     that the passes are bound by memory (the "Fast form" section);
//   other R <= 128: the same three passes as dense contractions of every line
//     with the R x R basis on the matrix cores (v_mfma_f32_32x32x2_f32, float32
//     in and accumulate);
//   R > 128: six axis passes on the matrix cores: a wave owns 32 grid lines and
//     all R outputs of each (R/32 output blocks of 32 x 32), reads every input
//     of its lines once, accumulates, then writes its lines, so a pass is in
//     place and touches each value once (8 B per value and pass).  Lines along
//     y and z are taken 32-contiguous in x (coalesced loads and stores); along
//     x the operands are swapped so that the stores stay contiguous.  The basis
//     (and its transpose) is read through the caches; the scale is fused into
//     the first inverse pass.
#include "common.h"
#include "fastdct_gen.h"

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

// Several levels of one generic pass in one launch: level i owns workgroups
// [first[i], first[i + 1]) and strides over its planes or pencil groups with
// that many workgroups (the levels are independent systems).
struct FusedBatch {
  int n;
  int first[PDG_MAX_LEVELS + 1];
  FusedArgs lv[PDG_MAX_LEVELS];
};
// this workgroup's level, its index among the level's workgroups and their count
__device__ __forceinline__ const FusedArgs &batch_level(const FusedBatch &b, long long &blk,
                                                        long long &nblk) {
  int i = 0;
  while (i + 1 < b.n && (int)blockIdx.x >= b.first[i + 1]) ++i;
  blk = (long long)blockIdx.x - b.first[i];
  nblk = b.first[i + 1] - b.first[i];
  return b.lv[i];
}

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
__global__ __launch_bounds__(kBig) void dct_plane_kernel(FusedBatch fb, int inverse) {
  long long blk, nblk;
  const FusedArgs &a = batch_level(fb, blk, nblk);
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
  long long plane = blk;
  if (plane < a.planes) load_rows(sp, P, a.src + plane_base(plane), R, R, R * R);
  __syncthreads();
  for (; plane < a.planes; plane += nblk) {
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
    const long long next = plane + nblk;
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
__global__ __launch_bounds__(kBig) void dct_pencil_kernel(FusedBatch fb) {
  long long blk, nblk;
  const FusedArgs &a = batch_level(fb, blk, nblk);
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
  if (blk < total) fetch(blk);
  for (long long g = blk; g < total; g += nblk) {
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
    if (g + nblk < total) fetch(g + nblk);   // in flight during this group
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
// Fast form for R = 16, 32, 64 and 128.  The even/odd split of a line of R
// values (its folded sums give the even frequencies by a DCT-II of length R/2,
// its folded differences the odd ones by a DCT-IV of length R/2) is taken one
// level further: each half is a fast transform of length R/2 on one thread's
// registers (fastdct_gen.h: split-radix DFTs between twiddle steps, about ten
// operations per value against R/2 multiply-adds of the dense product), so the
// passes are bound by memory, not arithmetic.  The transforms are unnormalised
// (cos(pi k (2x+1) / 2R) without s_k); the squared normalisations s_k^2 of the
// three axes join the spectral scale in the pencil pass:
//   C^T D C = Cu^T (S^2 D) Cu,  C = S Cu,  S = diag(s_k).
// The two threads of a line sit in different waves, so each wave runs one of
// the two transforms.  Spectra between the passes keep the order
// [even frequencies | odd frequencies] along each axis: position p < R/2 holds
// frequency 2p, position p >= R/2 frequency 2 (p - R/2) + 1.
//
//   plane fwd   256 / 2R z-planes in LDS (pitch R + 1; one for R = 128):
//               transforms along x (rows, in LDS), then along y (columns,
//               straight to HBM);
//   pencil      128 consecutive (qy, qx) pencils of one system in LDS: forward
//               z, scale by s^2 / (1 + lam mu)^2, inverse z (DCT-III of the
//               even half, DCT-IV of the odd half), combined through LDS;
//   plane inv   inverse along x, then along y, combined through LDS into the
//               natural plane, stored (or, with Adam, driving an Adam step of
//               the parameters at the same positions, float4 at a time).
constexpr int kFT = 256;            // threads of a fast-transform block (4 waves)
constexpr int kFP = 128;            // pencils per block
constexpr int kFQ = kFP + 1;

template <int H>
__device__ __forceinline__ void fdct2(float (&v)[H]) {
  if constexpr (H == 64) fdct::dct2_64(v);
  else if constexpr (H == 32) fdct::dct2_32(v);
  else if constexpr (H == 16) fdct::dct2_16(v);
  else fdct::dct2_8(v);
}
template <int H>
__device__ __forceinline__ void fdct3(float (&v)[H]) {
  if constexpr (H == 64) fdct::dct3_64(v);
  else if constexpr (H == 32) fdct::dct3_32(v);
  else if constexpr (H == 16) fdct::dct3_16(v);
  else fdct::dct3_8(v);
}
template <int H>
__device__ __forceinline__ void fdct4(float (&v)[H]) {
  if constexpr (H == 64) fdct::dct4_64(v);
  else if constexpr (H == 32) fdct::dct4_32(v);
  else if constexpr (H == 16) fdct::dct4_16(v);
  else fdct::dct4_8(v);
}

// This thread's half (0: even frequencies, 1: odd; uniform per wave) and its
// line among the block's 128 (plane kernels: plane pl of the block, line ln).
struct FastLane {
  int h, gl;
};
__device__ __forceinline__ FastLane fast_lane() {
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  return {w & 1, (w >> 1) * 64 + (int)(threadIdx.x & 63)};
}

// Block's planes (kFT / 2R of them) from HBM into LDS (pitch R + 1).
// Streams read or written once per pass go past the caches (non-temporal
// loads and stores)
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 nt_load4(const float *p) {
  const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void nt_store4(float *p, float4 x) {
  const nt_f4 v = {x.x, x.y, x.z, x.w};
  __builtin_nontemporal_store(v, reinterpret_cast<nt_f4 *>(p));
}

template <int R>
__device__ __forceinline__ void fast_load_planes(float *sp, const float *src, long long stack,
                                                 long long off, long long plane0) {
  constexpr int PPB = kFT / (2 * R), P = R + 1, G = PPB * R * R / (4 * kFT);
  constexpr long long R2 = (long long)R * R, R3 = R2 * R;
  float4 t[G];
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const int idx = 4 * ((int)threadIdx.x + k * kFT);
    const long long plane = plane0 + idx / (R * R);
    const long long sys = plane / R, z = plane % R;
    const int o = idx % (R * R);
    t[k] = nt_load4(src + (sys / 3) * stack + off + (sys % 3) * R3 + z * R2 + o);
  }
#pragma unroll
  for (int k = 0; k < G; ++k) {
    const int idx = 4 * ((int)threadIdx.x + k * kFT);
    const int pl = idx / (R * R), o = idx % (R * R);
    float *d = sp + pl * R * P + (o / R) * P + o % R;
    d[0] = t[k].x;
    d[1] = t[k].y;
    d[2] = t[k].z;
    d[3] = t[k].w;
  }
}

template <int R>
__global__ __launch_bounds__(kFT) void fdct_plane_fwd_kernel(FusedArgs a) {
  constexpr int H = R / 2, P = R + 1, PPB = kFT / (2 * R);
  constexpr long long R2 = (long long)R * R, R3 = R2 * R;
  extern __shared__ float lds[];
  const long long plane0 = (long long)blockIdx.x * PPB;
  fast_load_planes<R>(lds, a.src, a.stack, a.off, plane0);
  __syncthreads();
  const FastLane fl = fast_lane();
  const int pl = fl.gl / R, ln = fl.gl % R;
  float *sp = lds + pl * R * P;
  float v[H];
  {   // along x: row ln
    const float *row = sp + ln * P;
    if (fl.h == 0) {
#pragma unroll
      for (int n = 0; n < H; ++n) v[n] = row[n] + row[R - 1 - n];
      fdct2<H>(v);
    } else {
#pragma unroll
      for (int n = 0; n < H; ++n) v[n] = row[n] - row[R - 1 - n];
      fdct4<H>(v);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < H; ++k) sp[ln * P + fl.h * H + k] = v[k];
  __syncthreads();
  {   // along y: column ln
    const float *col = sp + ln;
    if (fl.h == 0) {
#pragma unroll
      for (int n = 0; n < H; ++n) v[n] = col[n * P] + col[(R - 1 - n) * P];
      fdct2<H>(v);
    } else {
#pragma unroll
      for (int n = 0; n < H; ++n) v[n] = col[n * P] - col[(R - 1 - n) * P];
      fdct4<H>(v);
    }
    const long long plane = plane0 + pl, sys = plane / R, z = plane % R;
    float *out = a.dst + (sys / 3) * a.stack + a.off + (sys % 3) * R3 + z * R2 + ln;
#pragma unroll
    for (int k = 0; k < H; ++k) __builtin_nontemporal_store(v[k], &out[(fl.h * H + k) * R]);
  }
}

template <int R>
__global__ __launch_bounds__(kFT) void fdct_pencil_kernel(FusedArgs a) {
  constexpr int H = R / 2, G = R * kFP / (4 * kFT);
  constexpr long long R2 = (long long)R * R, R3 = R2 * R;
  constexpr int groups = R * R / kFP;   // pencil groups per system
  extern __shared__ float sq[];
  float *smu = sq + R * kFQ;            // mu_f of the z frequencies
  if (threadIdx.x < R) smu[threadIdx.x] = a.mu[threadIdx.x];
  const long long sys = blockIdx.x / groups;
  const int j0 = (blockIdx.x % groups) * kFP;
  float *base = a.dst + (sys / 3) * a.stack + a.off + (sys % 3) * R3 + j0;
  {
    float4 t[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int idx = 4 * ((int)threadIdx.x + k * kFT);
      t[k] = nt_load4(base + (idx / kFP) * R2 + idx % kFP);
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int idx = 4 * ((int)threadIdx.x + k * kFT);
      float *d = sq + (idx / kFP) * kFQ + idx % kFP;
      d[0] = t[k].x;
      d[1] = t[k].y;
      d[2] = t[k].z;
      d[3] = t[k].w;
    }
  }
  __syncthreads();
  const FastLane fl = fast_lane();
  const int j = fl.gl;
  const float *col = sq + j;
  float v[H];
  if (fl.h == 0) {
#pragma unroll
    for (int n = 0; n < H; ++n) v[n] = col[n * kFQ] + col[(R - 1 - n) * kFQ];
    fdct2<H>(v);
  } else {
#pragma unroll
    for (int n = 0; n < H; ++n) v[n] = col[n * kFQ] - col[(R - 1 - n) * kFQ];
    fdct4<H>(v);
  }
  {   // (S^2 D) at (qy, qx, qz): frequency 2p of position p < H, 2 (p - H) + 1 above
    const int ln = j0 + j, qy = ln / R, qx = ln % R;
    const int fy = qy < H ? 2 * qy : 2 * (qy - H) + 1, fx = qx < H ? 2 * qx : 2 * (qx - H) + 1;
    const float s0 = 1.0f / R, s1 = 2.0f / R;
    const float sxy = (fy ? s1 : s0) * (fx ? s1 : s0);
    const float mxy = a.mu[fy] + a.mu[fx];
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const int fz = 2 * k + fl.h;
      const float d = 1.0f + a.lam * (mxy + smu[fz]);
      v[k] *= sxy * (fz ? s1 : s0) / (d * d);
    }
  }
  if (fl.h == 0) fdct3<H>(v); else fdct4<H>(v);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < H; ++k) sq[(fl.h * H + k) * kFQ + j] = v[k];
  __syncthreads();
  // out[z] = E[z] + O[z], out[R-1-z] = E[z] - O[z]  (z < H)
  const float sg = fl.h ? -1.f : 1.f;
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const float r = col[k * kFQ] + sg * col[(H + k) * kFQ];
    __builtin_nontemporal_store(r, &base[(fl.h ? R - 1 - k : k) * R2 + j]);
  }
}

template <int R, bool ADAM>
__global__ __launch_bounds__(kFT) void fdct_plane_inv_kernel(FusedArgs a, AdamEpi ad) {
  constexpr int H = R / 2, P = R + 1, PPB = kFT / (2 * R), G = PPB * R * R / (4 * kFT);
  constexpr long long R2 = (long long)R * R, R3 = R2 * R;
  extern __shared__ float lds[];
  float bc1 = 1.f, bc2 = 1.f;
  if constexpr (ADAM) {
    __shared__ float sbc[2];
    adam_bias(ad.b1, ad.b2, ad.step_dev, ad.step_host, sbc);
    bc1 = sbc[0];
    bc2 = sbc[1];
  }
  const long long plane0 = (long long)blockIdx.x * PPB;
  fast_load_planes<R>(lds, a.src, a.stack, a.off, plane0);
  __syncthreads();
  const FastLane fl = fast_lane();
  const int pl = fl.gl / R, ln = fl.gl % R;
  float *sp = lds + pl * R * P;
  float v[H];
  {   // along x, spectral row ln: E (even half) or O (odd half) in place
    float *row = sp + ln * P + fl.h * H;
#pragma unroll
    for (int k = 0; k < H; ++k) v[k] = row[k];
    if (fl.h == 0) fdct3<H>(v); else fdct4<H>(v);
#pragma unroll
    for (int k = 0; k < H; ++k) row[k] = v[k];
  }
  __syncthreads();
  {   // along y, natural column ln: t[q][x] = E_q[x] + O_q[x], t[q][R-1-x] = E_q[x] - O_q[x]
    const int xx = ln < H ? ln : R - 1 - ln;
    const float sg = ln < H ? 1.f : -1.f;
    const float *col = sp + fl.h * H * P + xx;
#pragma unroll
    for (int k = 0; k < H; ++k) v[k] = col[k * P] + sg * col[k * P + H];
    if (fl.h == 0) fdct3<H>(v); else fdct4<H>(v);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < H; ++k) sp[(fl.h * H + k) * P + ln] = v[k];
  __syncthreads();
  // natural (y, x): E_y[y] + O_y[y] for y < H, E_y[R-1-y] - O_y[R-1-y] above;
  // float4 group k of this thread starts at 4 (threadIdx.x + k kFT)
  auto grad4 = [&](int k, long long &at) {
    const int idx = 4 * ((int)threadIdx.x + k * kFT);
    const int p = idx / (R * R), o = idx % (R * R), y = o / R, x = o % R;
    const int yy = y < H ? y : R - 1 - y;
    const float sg = y < H ? 1.f : -1.f;
    const float *e = lds + p * R * P + yy * P + x, *od = e + H * P;
    const long long plane = plane0 + p, sys = plane / R, z = plane % R;
    at = (sys / 3) * a.stack + a.off + (sys % 3) * R3 + z * R2 + o;
    return make_float4(e[0] + sg * od[0], e[1] + sg * od[1], e[2] + sg * od[2], e[3] + sg * od[3]);
  };
  if constexpr (ADAM) {
    // batches of groups: every parameter and moment load of a batch in flight
    // before its first use (the arrays do not overlap)
    float *__restrict__ pth = ad.th;
    float *__restrict__ pm = ad.m;
    float *__restrict__ pv = ad.v;
    constexpr int GB = G < 8 ? G : 8;
#pragma unroll
    for (int k0 = 0; k0 < G; k0 += GB) {
      float4 th[GB], mo[GB], vo[GB];
#pragma unroll
      for (int k = 0; k < GB; ++k) {
        const int idx = 4 * ((int)threadIdx.x + (k0 + k) * kFT);
        const int p = idx / (R * R), o = idx % (R * R);
        const long long plane = plane0 + p, sys = plane / R, z = plane % R;
        const long long at = (sys / 3) * a.stack + a.off + (sys % 3) * R3 + z * R2 + o;
        th[k] = nt_load4(pth + at);
        mo[k] = nt_load4(pm + at);
        vo[k] = nt_load4(pv + at);
      }
#pragma unroll
      for (int k = 0; k < GB; ++k) {
        long long at;
        const float4 g = grad4(k0 + k, at);
        th[k].x = adam_one(ad.b1, ad.b2, ad.eps, ad.lr, bc1, bc2, g.x, mo[k].x, vo[k].x, th[k].x);
        th[k].y = adam_one(ad.b1, ad.b2, ad.eps, ad.lr, bc1, bc2, g.y, mo[k].y, vo[k].y, th[k].y);
        th[k].z = adam_one(ad.b1, ad.b2, ad.eps, ad.lr, bc1, bc2, g.z, mo[k].z, vo[k].z, th[k].z);
        th[k].w = adam_one(ad.b1, ad.b2, ad.eps, ad.lr, bc1, bc2, g.w, mo[k].w, vo[k].w, th[k].w);
        nt_store4(pth + at, th[k]);
        nt_store4(pm + at, mo[k]);
        nt_store4(pv + at, vo[k]);
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < G; ++k) {
      long long at;
      const float4 g = grad4(k, at);
      *reinterpret_cast<float4 *>(a.dst + at) = g;
    }
  }
}

template <int R>
pdg_status fast_level(const FusedArgs &f0, const AdamEpi *ad, hipStream_t st) {
  constexpr int PPB = kFT / (2 * R);
  const size_t plane = (size_t)PPB * R * (R + 1) * sizeof(float);
  const size_t pencil = (size_t)(R * kFQ + R) * sizeof(float);
  static PerDevice attrs;
  int dev = 0;
  PDG_TRY_HIP(hipGetDevice(&dev));
  if (!attrs.done(dev)) {
    PDG_TRY_HIP(hipFuncSetAttribute((const void *)fdct_plane_fwd_kernel<R>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)plane));
    PDG_TRY_HIP(hipFuncSetAttribute((const void *)fdct_plane_inv_kernel<R, false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)plane));
    PDG_TRY_HIP(hipFuncSetAttribute((const void *)fdct_plane_inv_kernel<R, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)plane));
    PDG_TRY_HIP(hipFuncSetAttribute((const void *)fdct_pencil_kernel<R>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)pencil));
    attrs.mark(dev);
  }
  FusedArgs f = f0;
  if (f.planes % R != 0 || f.planes % PPB != 0) {   // planes = batch * 3 * R
    set_error("fast DCT: %lld planes is not a whole number of systems and blocks", f.planes);
    return PDG_EINVAL;
  }
  const long long pblocks = f.planes / PPB;
  const long long gblocks = f.planes / R * ((long long)R * R / kFP);
  if (pblocks > 0x7fffffffLL || gblocks > 0x7fffffffLL) {
    set_error("fast DCT: batch too large (%lld planes)", f.planes);
    return PDG_EINVAL;
  }
  if (pblocks == 0) return PDG_OK;
  fdct_plane_fwd_kernel<R><<<(unsigned)pblocks, kFT, plane, st>>>(f);
  PDG_TRY(launched("fdct_plane_fwd"));
  f.src = f.dst;
  fdct_pencil_kernel<R><<<(unsigned)gblocks, kFT, pencil, st>>>(f);
  PDG_TRY(launched("fdct_pencil"));
  if (ad) {
    fdct_plane_inv_kernel<R, true><<<(unsigned)pblocks, kFT, plane, st>>>(f, *ad);
  } else {
    AdamEpi none;
    memset(&none, 0, sizeof none);
    fdct_plane_inv_kernel<R, false><<<(unsigned)pblocks, kFT, plane, st>>>(f, none);
  }
  return launched("fdct_plane_inv");
}

int padded(int R) { return 32 * ((R + 31) / 32); }
size_t plane_lds(int R) { return (size_t)2 * padded(R) * (padded(R) + 1) * sizeof(float); }
size_t pencil_lds(int R) { return (size_t)(padded(R) * (padded(R) + 1) + padded(R) * kPP) * sizeof(float); }

template <int NT, bool FULL>
pdg_status fused_levels(const FusedArgs *f0, int n, hipStream_t st) {
  static PerDevice attrs;
  int dev = 0;
  PDG_TRY_HIP(hipGetDevice(&dev));
  if (!attrs.done(dev)) {
    PDG_TRY_HIP(hipFuncSetAttribute((const void *)dct_plane_kernel<NT, FULL>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)plane_lds(32 * NT)));
    PDG_TRY_HIP(hipFuncSetAttribute((const void *)dct_pencil_kernel<NT, FULL>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)pencil_lds(32 * NT)));
    attrs.mark(dev);
  }
  // the levels' three passes, each one launch for all of them (the levels of
  // one call share NT, so one LDS size serves them)
  FusedBatch fwd, pen, inv;   // plane forward, pencil, plane inverse
  fwd.n = pen.n = inv.n = n;
  fwd.first[0] = pen.first[0] = inv.first[0] = 0;
  for (int i = 0; i < n; ++i) {
    const FusedArgs &f = f0[i];
    const int R = f.R;
    const long long groups = f.planes / R * (((long long)R * R + kPencils - 1) / kPencils);
    const int gp = (int)(f.planes < 2048 ? f.planes : 2048);
    const int gg = (int)(groups < 2048 ? groups : 2048);
    fwd.lv[i] = pen.lv[i] = inv.lv[i] = f;
    pen.lv[i].src = inv.lv[i].src = f.dst;   // the later passes work on dst
    fwd.first[i + 1] = inv.first[i + 1] = fwd.first[i] + gp;
    pen.first[i + 1] = pen.first[i] + gg;
  }
  const int RP = 32 * NT;
  dct_plane_kernel<NT, FULL><<<(unsigned)fwd.first[n], kBig, plane_lds(RP), st>>>(fwd, 0);
  PDG_TRY(launched("dct_plane"));
  dct_pencil_kernel<NT, FULL><<<(unsigned)pen.first[n], kBig, pencil_lds(RP), st>>>(pen);
  PDG_TRY(launched("dct_pencil"));
  dct_plane_kernel<NT, FULL><<<(unsigned)inv.first[n], kBig, plane_lds(RP), st>>>(inv, 1);
  return launched("dct_plane");
}

template <int NT>
pdg_status fused_level(const FusedArgs &f, hipStream_t st) {
  return f.R == 32 * NT ? fused_levels<NT, true>(&f, 1, st) : fused_levels<NT, false>(&f, 1, st);
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
  FusedArgs small[PDG_MAX_LEVELS];   // the generic fused levels with R < 32
  int nsmall = 0;
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
      // fast form: its float4 accesses need 16-byte aligned buffers and level
      // and transition offsets that are multiples of 4 floats (else the
      // generic fused passes below, and Adam in its own stage)
      auto al16 = [](const void *q) { return ((uintptr_t)q & 15u) == 0; };
      const bool al = g.size % 4 == 0 && g.off[l] % 4 == 0 && al16(src) && al16(data) &&
                      (!adam || (al16(adam->th) && al16(adam->m) && al16(adam->v)));
      if ((R == 128 || R == 64 || R == 32 || R == 16) && al) {
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
        switch (R) {
          case 128: PDG_TRY(fast_level<128>(f, adam ? &ad : nullptr, st)); break;
          case 64: PDG_TRY(fast_level<64>(f, adam ? &ad : nullptr, st)); break;
          case 32: PDG_TRY(fast_level<32>(f, adam ? &ad : nullptr, st)); break;
          default: PDG_TRY(fast_level<16>(f, adam ? &ad : nullptr, st)); break;
        }
        continue;
      }
      if (R < 32) {   // every such level's passes go in one launch each, below
        small[nsmall++] = f;
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
  if (nsmall > 0) PDG_TRY((fused_levels<1, false>(small, nsmall, st)));
  return PDG_OK;
}

}  // namespace pdg
