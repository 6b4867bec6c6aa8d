// Multi-resolution trilinear warp (paper Sec. 3.1, Eq. 1; translation form
// of Eq. 7-8), its position adjoint and the deterministic grid scatter.
//
// Data layout: samples SoA [3][ld]; a grid stack packs levels one after the
// other, each level 3 dense channels of R^3 floats with x fastest.
#include "common.h"

namespace pdg {
namespace {

// Gather one level's interpolated value (3 channels) at s.
__device__ __forceinline__ void level_value(const float *__restrict__ L, int R, float sx, float sy,
                                            float sz, float &v0, float &v1, float &v2) {
  if (R == 1) {
    v0 = L[0];
    v1 = L[1];
    v2 = L[2];
    return;
  }
  int ix, iy, iz;
  float fx, fy, fz;
  bool in;
  stencil1(R, sx, ix, fx, in);
  stencil1(R, sy, iy, fy, in);
  stencil1(R, sz, iz, fz, in);
  const long long R2 = (long long)R * R, R3 = R2 * R;
  const long long b = (iz * R2) + (long long)iy * R + ix;
  const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
  const float w[8] = {gx * gy * gz, fx * gy * gz, gx * fy * gz, fx * fy * gz,
                      gx * gy * fz, fx * gy * fz, gx * fy * fz, fx * fy * fz};
  const long long o[8] = {0, 1, R, R + 1, R2, R2 + 1, R2 + R, R2 + R + 1};
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a0 += w[k] * L[b + o[k]];
    a1 += w[k] * L[R3 + b + o[k]];
    a2 += w[k] * L[2 * R3 + b + o[k]];
  }
  v0 = a0;
  v1 = a1;
  v2 = a2;
}

__global__ __launch_bounds__(256) void warp_kernel(GridDev g, const float *__restrict__ grids,
                                                   long long gstride, const float *__restrict__ x,
                                                   long long xstride, long long ldx,
                                                   float *__restrict__ out, long long ostride,
                                                   long long ldo, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = blockIdx.y;
  const float *G = grids + b * gstride;
  const float *X = x + b * xstride;
  float *O = out + b * ostride;
  const float px = X[i], py = X[ldx + i], pz = X[2 * ldx + i];
  float d0 = 0.f, d1 = 0.f, d2 = 0.f;
  for (int l = 0; l < g.levels; ++l) {
    float v0, v1, v2;
    level_value(G + g.off[l], g.res[l], px, py, pz, v0, v1, v2);
    d0 += v0;
    d1 += v1;
    d2 += v2;
  }
  O[i] = px + g.scale * d0;
  O[ldo + i] = py + g.scale * d1;
  O[2 * ldo + i] = pz + g.scale * d2;
}

// lam_out = gdir + lam + (dD/dx)^T lam.
__global__ __launch_bounds__(256) void chain_adjoint_kernel(
    GridDev g, const float *__restrict__ G, const float *__restrict__ x, long long ldx,
    const float *__restrict__ lam, long long ldl, const float *__restrict__ gdir, long long ldd,
    float *__restrict__ lo, long long ldo, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float px = x[i], py = x[ldx + i], pz = x[2 * ldx + i];
  const float l0 = lam[i], l1 = lam[ldl + i], l2 = lam[2 * ldl + i];
  float j0 = 0.f, j1 = 0.f, j2 = 0.f;  // (dD/dx)^T lam, before level_scale
  for (int l = 0; l < g.levels; ++l) {
    const int R = g.res[l];
    if (R == 1) continue;
    const float *L = G + g.off[l];
    int ix, iy, iz;
    float fx, fy, fz;
    bool inx, iny, inz;
    stencil1(R, px, ix, fx, inx);
    stencil1(R, py, iy, fy, iny);
    stencil1(R, pz, iz, fz, inz);
    const long long R2 = (long long)R * R, R3 = R2 * R;
    const long long b = (iz * R2) + (long long)iy * R + ix;
    const long long o[8] = {0, 1, R, R + 1, R2, R2 + 1, R2 + R, R2 + R + 1};
    float s[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      s[k] = l0 * L[b + o[k]] + l1 * L[R3 + b + o[k]] + l2 * L[2 * R3 + b + o[k]];
    const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
    const float h = 0.5f * (float)R;
    // d/dfx of the trilinear form: (s[1]-s[0]) gy gz + (s[3]-s[2]) fy gz + ...
    float dx = (s[1] - s[0]) * gy * gz + (s[3] - s[2]) * fy * gz + (s[5] - s[4]) * gy * fz +
               (s[7] - s[6]) * fy * fz;
    float dy = (s[2] - s[0]) * gx * gz + (s[3] - s[1]) * fx * gz + (s[6] - s[4]) * gx * fz +
               (s[7] - s[5]) * fx * fz;
    float dz = (s[4] - s[0]) * gx * gy + (s[5] - s[1]) * fx * gy + (s[6] - s[2]) * gx * fy +
               (s[7] - s[3]) * fx * fy;
    if (inx) j0 += h * dx;
    if (iny) j1 += h * dy;
    if (inz) j2 += h * dz;
  }
  float r0 = l0 + g.scale * j0, r1 = l1 + g.scale * j1, r2 = l2 + g.scale * j2;
  if (gdir) {
    r0 += gdir[i];
    r1 += gdir[ldd + i];
    r2 += gdir[2 * ldd + i];
  }
  lo[i] = r0;
  lo[ldo + i] = r1;
  lo[2 * ldo + i] = r2;
}

// Key of a scatter entry: the parity class of its base cell (3 bits) above
// the global node id of the base cell.  Runs of one class have disjoint
// 2x2x2 corner sets, so a class can be scattered in one pass without
// conflicts; the classes run in a fixed order, which fixes the summation order
// at every node.
__global__ __launch_bounds__(256) void scatter_keys_kernel(GridDev g, const float *__restrict__ x,
                                                           long long xstride, long long ldx,
                                                           long long S, uint32_t *__restrict__ keys,
                                                           uint32_t *__restrict__ vals) {
  long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  const int seg = blockIdx.y;
  const float *X = x + seg * xstride;
  const float px = X[s], py = X[ldx + s], pz = X[2 * ldx + s];
  for (int l = 0; l < g.levels; ++l) {
    const int R = g.res[l];
    long long cell = 0;
    uint32_t cls = 0;
    if (R > 1) {
      int ix, iy, iz;
      float f;
      bool in;
      stencil1(R, px, ix, f, in);
      stencil1(R, py, iy, f, in);
      stencil1(R, pz, iz, f, in);
      cell = ((long long)iz * R + iy) * R + ix;
      cls = (uint32_t)((ix & 1) | ((iy & 1) << 1) | ((iz & 1) << 2));
    }
    long long e = ((long long)seg * g.levels + l) * S + s;
    keys[e] = (cls << kScatterClassShift) | (uint32_t)(seg * g.nodes + g.noff[l] + cell);
    vals[e] = (uint32_t)e;
  }
}

__global__ __launch_bounds__(256) void fill_kernel(float *__restrict__ p, long long n, float v) {
  long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i + 3 < n && (((uintptr_t)p) & 15) == 0) {
    *reinterpret_cast<float4 *>(p + i) = make_float4(v, v, v, v);
  } else {
    for (; i < n; ++i) p[i] = v;
  }
}

__global__ __launch_bounds__(256) void copy_kernel(float *__restrict__ d,
                                                   const float *__restrict__ s, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (long long)gridDim.x * blockDim.x) d[i] = s[i];
}

struct Blob {
  unsigned char b[2048];
};
__global__ void upload_kernel(Blob blob, unsigned char *__restrict__ dst, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = blob.b[i];
}

// One parity class: the first entry of every run of that class sums
// w_corner(s) * lam(s) over its samples for all 8 corners and adds
// level_scale times the sums to the 8 corner nodes.
__global__ __launch_bounds__(256) void scatter_pass_kernel(
    GridDev g, int cls, const uint32_t *__restrict__ keys, const uint32_t *__restrict__ vals,
    long long nent, long long S, const float *__restrict__ x, long long xstride, long long ldx,
    const float *__restrict__ lam, long long lstride, long long ldl, float *__restrict__ grad) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nent) return;
  const uint32_t key = keys[i];
  if ((int)(key >> kScatterClassShift) != cls) return;
  if (i > 0 && keys[i - 1] == key) return;  // only the first entry of a run works
  const uint32_t e0 = vals[i];
  const long long segl = (long long)e0 / S;
  const int seg = (int)(segl / g.levels);
  const int l = (int)(segl % g.levels);
  const int R = g.res[l];
  const float *X = x + seg * xstride;
  const float *Lm = lam + seg * lstride;
  float a[8][3];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k][0] = a[k][1] = a[k][2] = 0.f;
  for (long long j = i; j < nent && keys[j] == key; ++j) {
    const long long s = (long long)vals[j] % S;
    const float l0 = Lm[s], l1 = Lm[ldl + s], l2 = Lm[2 * ldl + s];
    if (R > 1) {
      int ii;
      float fx, fy, fz;
      bool in;
      stencil1(R, X[s], ii, fx, in);
      stencil1(R, X[ldx + s], ii, fy, in);
      stencil1(R, X[2 * ldx + s], ii, fz, in);
      const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
      const float w[8] = {gx * gy * gz, fx * gy * gz, gx * fy * gz, fx * fy * gz,
                          gx * gy * fz, fx * gy * fz, gx * fy * fz, fx * fy * fz};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        a[k][0] += w[k] * l0;
        a[k][1] += w[k] * l1;
        a[k][2] += w[k] * l2;
      }
    } else {
      a[0][0] += l0;
      a[0][1] += l1;
      a[0][2] += l2;
    }
  }
  const long long cell =
      (long long)(key & ((1u << kScatterClassShift) - 1u)) - (long long)seg * g.nodes - g.noff[l];
  const long long R2 = (long long)R * R, R3 = R2 * R;
  float *Gd = grad + (long long)seg * g.size + g.off[l];
  const int corners = R > 1 ? 8 : 1;
  for (int k = 0; k < corners; ++k) {
    const long long node = cell + (k & 1) + ((k >> 1) & 1) * R + ((k >> 2) & 1) * R2;
    Gd[node] += g.scale * a[k][0];
    Gd[R3 + node] += g.scale * a[k][1];
    Gd[2 * R3 + node] += g.scale * a[k][2];
  }
}

}  // namespace

pdg_status launch_warp(const GridDev &g, const float *grids, long long gstride, const float *x,
                       long long xstride, long long ldx, float *out, long long ostride,
                       long long ldo, long long n, int batch, hipStream_t st) {
  if (n <= 0 || batch <= 0) return PDG_OK;
  dim3 grid(div_up(n, 256), batch);
  warp_kernel<<<grid, 256, 0, st>>>(g, grids, gstride, x, xstride, ldx, out, ostride, ldo, n);
  return launched("warp");
}

pdg_status launch_chain_adjoint(const GridDev &g, const float *grids, const float *x, long long ldx,
                                const float *lam, long long ldl, const float *gdir, long long ldd,
                                float *lam_out, long long ldo, long long n, hipStream_t st) {
  if (n <= 0) return PDG_OK;
  chain_adjoint_kernel<<<div_up(n, 256), 256, 0, st>>>(g, grids, x, ldx, lam, ldl, gdir, ldd,
                                                       lam_out, ldo, n);
  return launched("chain_adjoint");
}

pdg_status launch_scatter_keys(const GridDev &g, const float *x, long long xstride, long long ldx,
                               long long S, int segs, uint32_t *keys, uint32_t *vals,
                               hipStream_t st) {
  if (S <= 0 || segs <= 0) return PDG_OK;
  dim3 grid(div_up(S, 256), segs);
  scatter_keys_kernel<<<grid, 256, 0, st>>>(g, x, xstride, ldx, S, keys, vals);
  return launched("scatter_keys");
}

pdg_status launch_fill(float *p, long long count, float value, hipStream_t st) {
  if (count <= 0) return PDG_OK;
  fill_kernel<<<div_up(div_up(count, 4), 256), 256, 0, st>>>(p, count, value);
  return launched("fill");
}

pdg_status launch_copy(float *dst, const float *src, long long count, hipStream_t st) {
  if (count <= 0) return PDG_OK;
  long long blocks = div_up(count, 256);
  if (blocks > 65536) blocks = 65536;
  copy_kernel<<<(unsigned)blocks, 256, 0, st>>>(dst, src, count);
  return launched("copy");
}

pdg_status upload_small(void *dst, const void *src, size_t bytes, hipStream_t st) {
  const unsigned char *s = (const unsigned char *)src;
  unsigned char *d = (unsigned char *)dst;
  while (bytes > 0) {
    const size_t n = bytes < sizeof(Blob) ? bytes : sizeof(Blob);
    Blob b;
    for (size_t i = 0; i < n; ++i) b.b[i] = s[i];
    upload_kernel<<<1, 256, 0, st>>>(b, d, (int)n);
    PDG_TRY(launched("upload"));
    s += n;
    d += n;
    bytes -= n;
  }
  return PDG_OK;
}

pdg_status launch_scatter_pass(const GridDev &g, int cls, const uint32_t *keys,
                               const uint32_t *vals, long long nent, long long S, const float *x,
                               long long xstride, long long ldx, const float *lam,
                               long long lstride, long long ldl, float *grad, hipStream_t st) {
  if (nent <= 0) return PDG_OK;
  scatter_pass_kernel<<<div_up(nent, 256), 256, 0, st>>>(g, cls, keys, vals, nent, S, x, xstride,
                                                         ldx, lam, lstride, ldl, grad);
  return launched("scatter_pass");
}

}  // namespace pdg
