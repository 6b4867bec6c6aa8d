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
// A wave owns 32 grid lines and all R outputs of each (R/32 output blocks of
// 32 x 32): it reads every input of its lines once, accumulates, then writes
// its lines, so a pass is in place and touches each value once (8 B per value
// and pass).  Lines along y and z are taken 32-contiguous in x (coalesced
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

pdg_status run_dct(const GridDev &g, int batch, const float *lam, float *data, const void *ws,
                   hipStream_t st) {
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
