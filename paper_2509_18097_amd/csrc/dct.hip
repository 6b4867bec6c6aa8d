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
// Fused passes for R <= 128: a z-plane (R x R, rows padded by one float so that
// column reads hit distinct LDS banks) or 32 z-pencils live in LDS and receive
// two transforms per HBM round trip.  Every wave owns one row of 32 x 32 output
// tiles; operands come from LDS (data) and the cached basis (coefficients).
struct FusedArgs {
  const float *src;            // input of the pass
  float *dst;                  // output of the pass (may equal src)
  long long stack, off, planes;   // planes = batch * 3 * R (z-planes or pencil groups)
  const float *cf;             // [in][out] = C^T  (forward coefficients)
  const float *ci;             // [in][out] = C    (inverse coefficients)
  const float *mu;
  int R;
  float lam;
};

constexpr int kFusedMaxR = 128;

// acc[t][i][j] = sum_k A(i0 + i, k) B(k, 32 t + j), k < R, for the NT tiles of
// one 32-row band; A and B are functors that return 0 outside the valid range.
// K is consumed kCh MFMA steps at a time: all operands of a chunk are loaded
// (independent loads in flight) before its NT x kCh matrix-core operations.
constexpr int kCh = 8;

template <int NT, class FA, class FB>
__device__ __forceinline__ void band_gemm(int R, int i0, const FA &a, const FB &b, f32x16 (&acc)[NT]) {
  const int lane = threadIdx.x & 63, jj = lane & 31, h = lane >> 5;
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = (f32x16){};
  for (int k0 = 0; k0 < R; k0 += 2 * kCh) {
    float av[kCh], bv[kCh][NT];
#pragma unroll
    for (int c = 0; c < kCh; ++c) {
      const int k = k0 + 2 * c + h;
      av[c] = a(i0 + jj, k);
#pragma unroll
      for (int t = 0; t < NT; ++t) bv[c][t] = b(k, 32 * t + jj);
    }
#pragma unroll
    for (int c = 0; c < kCh; ++c)
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[c], bv[c][t], acc[t], 0, 0, 0);
  }
}

// row of the output held by register r of this lane (column = lane & 31)
__device__ __forceinline__ int trow(int r) {
  const int lane = threadIdx.x & 63;
  return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

// Two transforms of one z-plane held in LDS: along x (t[y][k] = sum_x in[y][x] M[x][k])
// then along y (out[k'][k] = sum_y M[y][k'] t[y][k]), M = [in][out] coefficients
// (forward: C^T, inverse: C).  NT = ceil(R / 32) <= 4; wave w owns output band w
// (rows 32 w .. 32 w + 31, all NT column tiles) in both phases.
template <int NT>
__global__ __launch_bounds__(kThreads) void dct_plane_kernel(FusedArgs a, int inverse) {
  __shared__ float sp[kFusedMaxR * (kFusedMaxR + 1)];
  const int R = a.R, P = R + 1;
  const long long plane = blockIdx.x;
  if (plane >= a.planes) return;
  const long long sys = plane / R, z = plane % R;
  const long long R2 = (long long)R * R, R3 = R2 * R;
  const long long base = (sys / 3) * a.stack + a.off + (sys % 3) * R3 + z * R2;
  const float *m = inverse ? a.ci : a.cf;
  for (int i = threadIdx.x; i < R * R; i += kThreads) sp[(i / R) * P + i % R] = a.src[base + i];
  __syncthreads();
  const int ti = threadIdx.x >> 6, col = threadIdx.x & 31;
  f32x16 acc[NT];
  auto ax = [&](int y, int x) { return (y < R && x < R) ? sp[y * P + x] : 0.f; };
  auto bx = [&](int x, int k) { return (x < R && k < R) ? m[x * R + k] : 0.f; };
  if (ti < NT) band_gemm<NT>(R, ti * 32, ax, bx, acc);
  __syncthreads();
  if (ti < NT) {
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int y = ti * 32 + trow(r), k = tj * 32 + col;
        if (y < R && k < R) sp[y * P + k] = acc[tj][r];
      }
  }
  __syncthreads();
  auto ay = [&](int kk, int y) { return (kk < R && y < R) ? m[y * R + kk] : 0.f; };
  auto by = [&](int y, int k) { return (y < R && k < R) ? sp[y * P + k] : 0.f; };
  if (ti < NT) {
    band_gemm<NT>(R, ti * 32, ay, by, acc);
#pragma unroll
    for (int tj = 0; tj < NT; ++tj)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int kk = ti * 32 + trow(r), k = tj * 32 + col;
        if (kk < R && k < R) a.dst[base + (long long)kk * R + k] = acc[tj][r];
      }
  }
}

// Forward z, scale by (1 + lam (mu_x + mu_y + mu_z))^-2, inverse z for 32
// consecutive (y, x) pencils of one system, in place on dst.  Wave w owns the
// 32 output rows (z frequencies, then z) of band w.
__global__ __launch_bounds__(kThreads) void dct_pencil_kernel(FusedArgs a) {
  __shared__ float sp[kFusedMaxR * 32];
  const int R = a.R;
  const long long R2 = (long long)R * R, R3 = R2 * R;
  const long long groups = (R2 + 31) / 32;         // pencil groups per system
  const long long g = blockIdx.x;
  if (g >= a.planes / R * groups) return;
  const long long sys = g / groups;
  const long long line0 = (g % groups) * 32;       // first (y, x) line = y * R + x
  const long long base = (sys / 3) * a.stack + a.off + (sys % 3) * R3;
  for (int i = threadIdx.x; i < R * 32; i += kThreads) {
    const int z = i / 32, j = i % 32;
    const long long ln = line0 + j;
    sp[z * 32 + j] = ln < R2 ? a.dst[base + z * R2 + ln] : 0.f;
  }
  __syncthreads();
  const int T = (R + 31) / 32, ti = threadIdx.x >> 6, j = threadIdx.x & 31;
  const long long ln = line0 + j;
  auto af = [&](int kz, int z) { return (kz < R && z < R) ? a.cf[z * R + kz] : 0.f; };
  auto bp = [&](int z, int c) { return z < R ? sp[z * 32 + c] : 0.f; };
  f32x16 acc[1];
  if (ti < T) band_gemm<1>(R, ti * 32, af, bp, acc);
  __syncthreads();
  if (ti < T) {
    float sxy = 0.f;
    if (ln < R2) sxy = a.mu[ln / R] + a.mu[ln % R];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int kz = ti * 32 + trow(r);
      if (kz < R) {
        const float d = 1.0f + a.lam * (sxy + a.mu[kz]);
        sp[kz * 32 + j] = ln < R2 ? acc[0][r] / (d * d) : 0.f;
      }
    }
  }
  __syncthreads();
  auto ai = [&](int z, int kz) { return (z < R && kz < R) ? a.ci[kz * R + z] : 0.f; };
  if (ti < T) {
    band_gemm<1>(R, ti * 32, ai, bp, acc);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int z = ti * 32 + trow(r);
      if (z < R && ln < R2) a.dst[base + z * R2 + ln] = acc[0][r];
    }
  }
}

pdg_status launch_plane(const FusedArgs &f, int inverse, hipStream_t st) {
  const unsigned blocks = (unsigned)f.planes;
  switch ((f.R + 31) / 32) {
    case 1: dct_plane_kernel<1><<<blocks, kThreads, 0, st>>>(f, inverse); break;
    case 2: dct_plane_kernel<2><<<blocks, kThreads, 0, st>>>(f, inverse); break;
    case 3: dct_plane_kernel<3><<<blocks, kThreads, 0, st>>>(f, inverse); break;
    case 4: dct_plane_kernel<4><<<blocks, kThreads, 0, st>>>(f, inverse); break;
    default:
      set_error("fused DCT passes need R <= %d (got %d)", kFusedMaxR, f.R);
      return PDG_EUNSUPPORTED;
  }
  return launched("dct_plane");
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

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

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
                   const void *ws, hipStream_t st) {
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
      f.cf = ct;
      f.ci = c;
      f.mu = mu;
      f.R = R;
      f.lam = lam[l];
      const long long groups = (long long)batch * 3 * (((long long)R * R + 31) / 32);
      PDG_TRY(launch_plane(f, 0, st));
      f.src = data;
      dct_pencil_kernel<<<(unsigned)groups, kThreads, 0, st>>>(f);
      PDG_TRY(launched("dct_pencil"));
      PDG_TRY(launch_plane(f, 1, st));
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
