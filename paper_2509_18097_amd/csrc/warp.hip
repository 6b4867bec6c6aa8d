// Multi-resolution trilinear warp (paper Sec. 3.1, Eq. 1; translation form
// of Eq. 7-8, and the six-channel cells of Sec. 3.3, Eq. 4-7), its position
// adjoint and the deterministic grid scatter.
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

// x + level_scale * sum_l D_l(x) (Eq. 1) at one point.
__device__ __forceinline__ void warp_point(const GridDev &g, const float *__restrict__ G, float px,
                                           float py, float pz, float &ox, float &oy, float &oz) {
  float d0 = 0.f, d1 = 0.f, d2 = 0.f;
  for (int l = 0; l < g.levels; ++l) {
    float v0, v1, v2;
    level_value(G + g.off[l], g.res[l], px, py, pz, v0, v1, v2);
    d0 += v0;
    d1 += v1;
    d2 += v2;
  }
  ox = px + g.scale * d0;
  oy = py + g.scale * d1;
  oz = pz + g.scale * d2;
}

// lam + level_scale * (dD/dx)^T lam at one point (the position adjoint of Eq. 1).
__device__ __forceinline__ void adjoint_point(const GridDev &g, const float *__restrict__ G, float px,
                                              float py, float pz, float l0, float l1, float l2,
                                              float &r0, float &r1, float &r2) {
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
  r0 = l0 + g.scale * j0;
  r1 = l1 + g.scale * j1;
  r2 = l2 + g.scale * j2;
}

// ---- six-channel cells (Sec. 3.3, Eq. 4-7): T = [z; t] per cell ---------

// One level's interpolated cell vector (6 channels, z then t) at s.
__device__ __forceinline__ void level_value6(const float *__restrict__ L, int R, float sx,
                                             float sy, float sz, float (&v)[6]) {
  if (R == 1) {
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = L[c];
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
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) a += w[k] * L[c * R3 + b + o[k]];
    v[c] = a;
  }
}

// sum_l trilerp(G_l, p) of the six channels; [z^; t^] is level_scale times it (Eq. 1).
__device__ __forceinline__ void cell_sum(const GridDev &g, const float *__restrict__ G, float px,
                                         float py, float pz, float (&acc)[6]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) acc[c] = 0.f;
  for (int l = 0; l < g.levels; ++l) {
    float v[6];
    level_value6(G + g.off[l], g.res[l], px, py, pz, v);
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += v[c];
  }
}

__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
  return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// out = R(z^) p + t^, R in the closed form of the Cayley map (Eq. 5):
// R p = p + 2 (z x p + z x (z x p)) / (1 + |z|^2).
__device__ __forceinline__ float3 warp6_point(const GridDev &g, const float *__restrict__ G,
                                              float3 p) {
  float T[6];
  cell_sum(g, G, p.x, p.y, p.z, T);
  const float3 z = make_float3(g.scale * T[0], g.scale * T[1], g.scale * T[2]);
  const float3 c1 = cross3(z, p), c2 = cross3(z, c1);
  const float k = 2.0f / (1.0f + dot3(z, z));
  // t^ added as level_scale * sum, as the translation warp does
  return make_float3((p.x + k * (c1.x + c2.x)) + g.scale * T[3],
                     (p.y + k * (c1.y + c2.y)) + g.scale * T[4],
                     (p.z + k * (c1.z + c2.z)) + g.scale * T[5]);
}

// Batch b = blockIdx.y reads grids G + b gs and samples x + b xs (SoA [3][n]).
__global__ __launch_bounds__(256) void warp6_kernel(GridDev g, const float *__restrict__ G,
                                                    long long gs, const float *__restrict__ x,
                                                    long long xs, float *__restrict__ out,
                                                    long long os, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  G += blockIdx.y * gs;
  x += blockIdx.y * xs;
  out += blockIdx.y * os;
  const float3 o = warp6_point(g, G, make_float3(x[i], x[n + i], x[2 * n + i]));
  out[i] = o.x;
  out[n + i] = o.y;
  out[2 * n + i] = o.z;
}

// sum_c lam_c d/dp trilerp(L_c, p) for one level (zero along clamped axes).
__device__ __forceinline__ void level_jt6(const float *__restrict__ L, int R, float px, float py,
                                          float pz, const float (&lam)[6], float &j0, float &j1,
                                          float &j2) {
  j0 = j1 = j2 = 0.f;
  if (R == 1) return;
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
  for (int k = 0; k < 8; ++k) {
    float a = 0.f;
#pragma unroll
    for (int c = 0; c < 6; ++c) a += lam[c] * L[c * R3 + b + o[k]];
    s[k] = a;
  }
  const float gx = 1.0f - fx, gy = 1.0f - fy, gz = 1.0f - fz;
  const float h = 0.5f * (float)R;
  const float dx = (s[1] - s[0]) * gy * gz + (s[3] - s[2]) * fy * gz + (s[5] - s[4]) * gy * fz +
                   (s[7] - s[6]) * fy * fz;
  const float dy = (s[2] - s[0]) * gx * gz + (s[3] - s[1]) * fx * gz + (s[6] - s[4]) * gx * fz +
                   (s[7] - s[5]) * fx * fz;
  const float dz = (s[4] - s[0]) * gx * gy + (s[5] - s[1]) * fx * gy + (s[6] - s[2]) * gx * fy +
                   (s[7] - s[3]) * fx * fy;
  if (inx) j0 = h * dx;
  if (iny) j1 = h * dy;
  if (inz) j2 = h * dz;
}

// Adjoint of warp6 for an upstream gradient q = dL/dout:
//   u  = dL/dz^ = (2/d) (p x q + (z x p) x q + p x (q x z)) - (4/d^2) (q . N) z,
//        N = z x p + z x (z x p), d = 1 + |z|^2   (the derivative of R p);
//   gx = R^T q + level_scale * sum_l sum_c [u; q]_c grad trilerp(G_l,c, p),
//        R^T q = q + (2/d) (z x (z x q) - z x q).
// u = d<q, R p>/dz^ and (when gx is set) gx = J^T q for one sample.
__device__ __forceinline__ void adjoint6_point(const GridDev &g, const float *__restrict__ G,
                                               float3 p, float3 q, float u[3], float3 *gx) {
  float T[6];
  cell_sum(g, G, p.x, p.y, p.z, T);
  const float3 z = make_float3(g.scale * T[0], g.scale * T[1], g.scale * T[2]);
  const float d = 1.0f + dot3(z, z);
  const float3 zp = cross3(z, p), zzp = cross3(z, zp);
  const float3 N = make_float3(zp.x + zzp.x, zp.y + zzp.y, zp.z + zzp.z);
  const float3 a1 = cross3(p, q), a2 = cross3(zp, q), a3 = cross3(p, cross3(q, z));
  const float ca = 2.0f / d, cz = 4.0f * dot3(q, N) / (d * d);
  u[0] = ca * (a1.x + a2.x + a3.x) - cz * z.x;
  u[1] = ca * (a1.y + a2.y + a3.y) - cz * z.y;
  u[2] = ca * (a1.z + a2.z + a3.z) - cz * z.z;
  if (gx) {
    const float3 zq = cross3(z, q), zzq = cross3(z, zq);
    const float lam[6] = {u[0], u[1], u[2], q.x, q.y, q.z};
    float j0 = 0.f, j1 = 0.f, j2 = 0.f;
    for (int l = 0; l < g.levels; ++l) {
      float a, b, c;
      level_jt6(G + g.off[l], g.res[l], p.x, p.y, p.z, lam, a, b, c);
      j0 += a;
      j1 += b;
      j2 += c;
    }
    *gx = make_float3((q.x + ca * (zzq.x - zq.x)) + g.scale * j0,
                      (q.y + ca * (zzq.y - zq.y)) + g.scale * j1,
                      (q.z + ca * (zzq.z - zq.z)) + g.scale * j2);
  }
}

// Batch b = blockIdx.y as warp6_kernel; gx (when set) = J^T gout + gx_add
// (gx_add nullable, laid out like gx).
__global__ __launch_bounds__(256) void adjoint6_kernel(GridDev g, const float *__restrict__ G,
                                                       long long gs, const float *__restrict__ x,
                                                       long long xs, const float *__restrict__ gout,
                                                       long long gos, float *__restrict__ uo,
                                                       long long us, float *__restrict__ gx,
                                                       const float *__restrict__ gx_add,
                                                       long long gxs, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long b = blockIdx.y;
  G += b * gs;
  x += b * xs;
  gout += b * gos;
  const float3 p = make_float3(x[i], x[n + i], x[2 * n + i]);
  const float3 q = make_float3(gout[i], gout[n + i], gout[2 * n + i]);
  float u[3];
  float3 r;
  adjoint6_point(g, G, p, q, u, gx ? &r : nullptr);
  if (uo) {
    uo += b * us;
    uo[i] = u[0];
    uo[n + i] = u[1];
    uo[2 * n + i] = u[2];
  }
  if (gx) {
    gx += b * gxs;
    if (gx_add) {
      gx_add += b * gxs;
      r.x += gx_add[i];
      r.y += gx_add[n + i];
      r.z += gx_add[2 * n + i];
    }
    gx[i] = r.x;
    gx[n + i] = r.y;
    gx[2 * n + i] = r.z;
  }
}

// The template chain on six-channel cells, one thread per vertex over all T
// transitions: xhat[t + 1] = R(z^_t) xhat[t] + t^_t (xhat[0] = X_0 is set).
__global__ __launch_bounds__(64) void chain_warp6_kernel(GridDev g, const float *__restrict__ params,
                                                         long long P, float *__restrict__ xhat,
                                                         long long V, int T) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  float3 p = make_float3(xhat[i], xhat[V + i], xhat[2 * V + i]);
  for (int t = 0; t < T; ++t) {
    p = warp6_point(g, params + (long long)t * P, p);
    float *o = xhat + (long long)(t + 1) * 3 * V;
    o[i] = p.x;
    o[V + i] = p.y;
    o[2 * V + i] = p.z;
  }
}

// Its reverse sweep: lam[T-1] = gd[T-1]; for t = T-1 .. 0 the rotation
// adjoint u[t] of transition t at xhat[t], and lam[t-1] = gd[t-1] + J_t^T lam[t].
__global__ __launch_bounds__(64) void chain_reverse6_kernel(GridDev g,
                                                            const float *__restrict__ params,
                                                            long long P,
                                                            const float *__restrict__ xhat,
                                                            const float *__restrict__ gd,
                                                            float *__restrict__ lam,
                                                            float *__restrict__ uo, long long V,
                                                            int T) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V) return;
  const long long s3 = 3 * V;
  const float *d = gd + (long long)(T - 1) * s3;
  float3 q = make_float3(d[i], d[V + i], d[2 * V + i]);
  float *l = lam + (long long)(T - 1) * s3;
  l[i] = q.x;
  l[V + i] = q.y;
  l[2 * V + i] = q.z;
  for (int t = T - 1; t >= 0; --t) {
    const float *x = xhat + (long long)t * s3;
    const float3 p = make_float3(x[i], x[V + i], x[2 * V + i]);
    float u[3];
    float3 r;
    adjoint6_point(g, params + (long long)t * P, p, q, u, t > 0 ? &r : nullptr);
    float *uu = uo + (long long)t * s3;
    uu[i] = u[0];
    uu[V + i] = u[1];
    uu[2 * V + i] = u[2];
    if (t > 0) {
      const float *dd = gd + (long long)(t - 1) * s3;
      q = make_float3(r.x + dd[i], r.y + dd[V + i], r.z + dd[2 * V + i]);
      float *ll = lam + (long long)(t - 1) * s3;
      ll[i] = q.x;
      ll[V + i] = q.y;
      ll[2 * V + i] = q.z;
    }
  }
}

// Thread i of batch b warps point order[b * order_stride + i] (or i): a
// spatial order keeps the grid cells of neighbouring threads close.
__global__ __launch_bounds__(256) void warp_kernel(GridDev g, const float *__restrict__ grids,
                                                   long long gstride, const float *__restrict__ x,
                                                   long long xstride, long long ldx,
                                                   float *__restrict__ out, long long ostride,
                                                   long long ldo, long long n,
                                                   const int *__restrict__ order,
                                                   long long order_stride, int batch,
                                                   unsigned nb) {
  unsigned job, blk;                  // one batch entry's workgroups on one XCD
  if (!job_block(blockIdx.x, (unsigned)batch, nb, job, blk)) return;
  const long long t = (long long)blk * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int b = (int)job;
  const long long i = order ? order[b * order_stride + t] : t;
  const float *X = x + b * xstride;
  float *O = out + b * ostride;
  warp_point(g, grids + b * gstride, X[i], X[ldx + i], X[2 * ldx + i], O[i], O[ldo + i],
             O[2 * ldo + i]);
}

// lam_out = gdir + lam + (dD/dx)^T lam.
__global__ __launch_bounds__(256) void chain_adjoint_kernel(
    GridDev g, const float *__restrict__ G, const float *__restrict__ x, long long ldx,
    const float *__restrict__ lam, long long ldl, const float *__restrict__ gdir, long long ldd,
    float *__restrict__ lo, long long ldo, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float r0, r1, r2;
  adjoint_point(g, G, x[i], x[ldx + i], x[2 * ldx + i], lam[i], lam[ldl + i], lam[2 * ldl + i],
                r0, r1, r2);
  if (gdir) {
    r0 += gdir[i];
    r1 += gdir[ldd + i];
    r2 += gdir[2 * ldd + i];
  }
  lo[i] = r0;
  lo[ldo + i] = r1;
  lo[2 * ldo + i] = r2;
}

// Per-level parts of warp_point and adjoint_point, so that the levels of one
// point can be gathered by different lanes.
__device__ __forceinline__ void level_jt(const float *__restrict__ L, int R, float px, float py,
                                         float pz, float l0, float l1, float l2, float &j0,
                                         float &j1, float &j2) {
  j0 = j1 = j2 = 0.f;
  if (R == 1) return;
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
  float dx = (s[1] - s[0]) * gy * gz + (s[3] - s[2]) * fy * gz + (s[5] - s[4]) * gy * fz +
             (s[7] - s[6]) * fy * fz;
  float dy = (s[2] - s[0]) * gx * gz + (s[3] - s[1]) * fx * gz + (s[6] - s[4]) * gx * fz +
             (s[7] - s[5]) * fx * fz;
  float dz = (s[4] - s[0]) * gx * gy + (s[5] - s[1]) * fx * gy + (s[6] - s[2]) * gx * fy +
             (s[7] - s[3]) * fx * fy;
  if (inx) j0 = h * dx;
  if (iny) j1 = h * dy;
  if (inz) j2 = h * dz;
}

// Template chains, one group of kChainLanes lanes per vertex (8, or 16 for
// more than eight levels; a divisor of the wave): lane l of the group gathers
// level l, lane 0 adds the levels in order (the same sums as warp_point /
// adjoint_point) and hands the new point to the group.
static_assert(PDG_MAX_LEVELS <= 16, "chain groups hold at most 16 levels");

// X_{t+1} = warp(G_t, X_t) for t = 0..T-1, X_0 copied to frame 0 (Eq. 8).
template <int kChainLanes>
__global__ __launch_bounds__(256) void chain_warp_kernel(GridDev g, const float *__restrict__ params,
                                                         long long P, const float *__restrict__ x0,
                                                         float *__restrict__ xhat, long long V, int T,
                                                         const int *__restrict__ order) {
  const long long item = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kChainLanes;
  const int l = threadIdx.x % kChainLanes;
  const int lead = (threadIdx.x & 63) - l;       // group leader lane in the wave
  const bool ok = item < V;
  const long long v = ok && order ? order[item] : item;   // vertex (spatial order)
  float px = 0.f, py = 0.f, pz = 0.f;
  if (ok) {
    px = x0[v];
    py = x0[V + v];
    pz = x0[2 * V + v];
    if (l == 0) {
      xhat[v] = px;
      xhat[V + v] = py;
      xhat[2 * V + v] = pz;
    }
  }
  for (int t = 0; t < T; ++t) {
    float v0 = 0.f, v1 = 0.f, v2 = 0.f;
    if (ok && l < g.levels)
      level_value(params + t * P + g.off[l], g.res[l], px, py, pz, v0, v1, v2);
    float d0 = 0.f, d1 = 0.f, d2 = 0.f;
    for (int k = 0; k < g.levels; ++k) {         // in level order, as warp_point
      d0 += __shfl(v0, lead + k, 64);
      d1 += __shfl(v1, lead + k, 64);
      d2 += __shfl(v2, lead + k, 64);
    }
    px = px + g.scale * d0;
    py = py + g.scale * d1;
    pz = pz + g.scale * d2;
    if (ok && l == 0) {
      float *o = xhat + (long long)(t + 1) * 3 * V;
      o[v] = px;
      o[V + v] = py;
      o[2 * V + v] = pz;
    }
  }
}

// Reverse sweep of the chain: lam_{T-1} = gd_{T-1} and, for k = T-1 .. 1,
// lam_{k-1} = gd_{k-1} + lam_k + (dD_k/dx)^T lam_k at X_k (grids k); lam_t is
// the total adjoint of X_{t+1} (frames 1..T).
template <int kChainLanes>
__global__ __launch_bounds__(256) void chain_reverse_kernel(GridDev g,
                                                            const float *__restrict__ params,
                                                            long long P,
                                                            const float *__restrict__ xhat,
                                                            const float *__restrict__ gd,
                                                            float *__restrict__ lam, long long V,
                                                            int T, const int *__restrict__ order) {
  const long long item = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / kChainLanes;
  const int l = threadIdx.x % kChainLanes;
  const int lead = (threadIdx.x & 63) - l;
  const bool ok = item < V;
  const long long v = ok && order ? order[item] : item;   // vertex (spatial order)
  const long long s3 = 3 * V;
  float l0 = 0.f, l1 = 0.f, l2 = 0.f;
  if (ok) {
    l0 = gd[(T - 1) * s3 + v];
    l1 = gd[(T - 1) * s3 + V + v];
    l2 = gd[(T - 1) * s3 + 2 * V + v];
    if (l == 0) {
      lam[(T - 1) * s3 + v] = l0;
      lam[(T - 1) * s3 + V + v] = l1;
      lam[(T - 1) * s3 + 2 * V + v] = l2;
    }
  }
  for (int k = T - 1; k >= 1; --k) {
    float j0 = 0.f, j1 = 0.f, j2 = 0.f;
    float d0 = 0.f, d1 = 0.f, d2 = 0.f;
    if (ok) {
      const float *x = xhat + k * s3;
      if (l < g.levels)
        level_jt(params + k * P + g.off[l], g.res[l], x[v], x[V + v], x[2 * V + v], l0, l1, l2,
                 j0, j1, j2);
      const float *d = gd + (k - 1) * s3;
      d0 = d[v];
      d1 = d[V + v];
      d2 = d[2 * V + v];
    }
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;
    for (int q = 0; q < g.levels; ++q) {         // in level order, as adjoint_point
      s0 += __shfl(j0, lead + q, 64);
      s1 += __shfl(j1, lead + q, 64);
      s2 += __shfl(j2, lead + q, 64);
    }
    float r0 = l0 + g.scale * s0, r1 = l1 + g.scale * s1, r2 = l2 + g.scale * s2;
    r0 += d0;
    r1 += d1;
    r2 += d2;
    if (ok && l == 0) {
      float *o = lam + (k - 1) * s3;
      o[v] = r0;
      o[V + v] = r1;
      o[2 * V + v] = r2;
    }
    l0 = r0;
    l1 = r1;
    l2 = r2;
  }
}

// Key of a scatter entry: the global node id of its base cell,
// seg*nodes + noff[l] + cell.  Sorted keys put the entries of one
// (segment, level, cell plane) next to each other and runs of equal keys
// gather the samples of one cell.
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
    if (R > 1) {
      int ix, iy, iz;
      float f;
      bool in;
      stencil1(R, px, ix, f, in);
      stencil1(R, py, iy, f, in);
      stencil1(R, pz, iz, f, in);
      cell = ((long long)iz * R + iy) * R + ix;
    }
    long long e = ((long long)seg * g.levels + l) * S + s;
    keys[e] = (uint32_t)(seg * g.nodes + g.noff[l] + cell);
    vals[e] = (uint32_t)e;
  }
}

// Row index of a key: seg * RS2 + (R_0^2 + ... + R_{l-1}^2) + z * R + y of
// the base cell (z, y, x).  Keys, node counts and row counts fit 32 bits.
// rstart[q] = first sorted entry whose row index is >= q, q = 0..nrows
// (rstart[nrows] = nent): one thread per row, a binary search for the row's
// first key (row r of level l in segment seg starts at key
// seg * nodes + noff[l] + r * R_l).
__global__ __launch_bounds__(256) void row_table_kernel(GridDev g, const uint32_t *__restrict__ keys,
                                                        int nent, uint32_t RS2, uint32_t nrows,
                                                        int *__restrict__ rstart) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q > nrows) return;
  if (q == nrows) {
    rstart[q] = nent;
    return;
  }
  const uint32_t seg = q / RS2;
  uint32_t r = q - seg * RS2;
  int l = 0;
  while (l + 1 < g.levels && r >= (uint32_t)(g.res[l] * g.res[l])) {
    r -= (uint32_t)(g.res[l] * g.res[l]);
    ++l;
  }
  const uint32_t k0 = seg * (uint32_t)g.nodes + (uint32_t)g.noff[l] + r * (uint32_t)g.res[l];
  int lo = 0, hi = nent;
  while (lo < hi) {
    const int mid = (int)(((unsigned)lo + (unsigned)hi) >> 1);
    if (keys[mid] < k0)
      lo = mid + 1;
    else
      hi = mid;
  }
  rstart[q] = lo;
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

// ent[i] = (fx, fy, fz, lam0), ent2[i] = (lam1, lam2) of sorted entry i.
// lam_only: the fractions staged by an earlier call on the same entries are
// kept (read back from ent) and only the adjoint values are staged anew.
__global__ __launch_bounds__(256) void scatter_stage_kernel(GridDev g, ScatterList L, int nent,
                                                            int lam_only) {
  // consecutive blocks (one segment's sorted entries) on one XCD
  const long long i = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= nent) return;
  const uint32_t e = L.vals[i], S = (uint32_t)L.S;
  const uint32_t segl = e / S;
  const uint32_t seg = segl / (uint32_t)g.levels;
  const int R = g.res[segl - seg * (uint32_t)g.levels];
  const uint32_t s = e - segl * S;
  const float *X = L.x + (long long)seg * L.xstride;
  const float *Lm = L.lam + (long long)seg * L.lstride;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  if (lam_only) {
    const float4 old = L.ent[i];
    fx = old.x;
    fy = old.y;
    fz = old.z;
  } else if (R > 1) {
    int ii;
    bool in;
    stencil1(R, X[s], ii, fx, in);
    stencil1(R, X[L.ldx + s], ii, fy, in);
    stencil1(R, X[2 * L.ldx + s], ii, fz, in);
  }
  L.ent[i] = make_float4(fx, fy, fz, Lm[s]);
  L.ent2[i] = make_float2(Lm[L.ldl + s], Lm[2 * L.ldl + s]);
}

// Gather form of the scatter: one block per (segment, level, node plane z,
// band of node rows y0..y1-1) writes all three channels of that band, every
// node exactly once (no zero fill, no read-modify-write in HBM).
//
// The band's nodes are corners of the cells in cell planes z-1 (corner
// dz = 1) and z (dz = 0) with cell rows y0-1..y1-1; the row table gives the
// entries of each (list, cell plane) as one contiguous range.  The ranges are
// walked 256 entries at a time: every thread forms its entry's 12 products
// w_k(s) * lam_c(s) (4 corners of its dz, 3 channels), a segmented inclusive
// scan over the chunk in float32 (segments = runs of equal (range, key)
// pairs, which are contiguous because every range is sorted; a fixed
// Hillis-Steele pattern inside rows of 16 lanes, then in row order across
// the wave, then across waves) leaves each run's sums at its last entry (a
// run cut by the chunk end hands its sums to the next chunk), and then, for
// each range (list, cell
// plane) and each (x, y) parity class in turn with a barrier in between, the
// runs that end there add level_scale times their sums to their corners inside
// the band held in LDS.  The runs of one range and class belong to distinct
// cells of one cell plane with equal (x, y) parity, so their corners are
// disjoint; every step's order is fixed by the sorted entries, so the result
// does not depend on scheduling.
constexpr int kGatherThreads = 256;
constexpr int kBandFloats = 2048;          // LDS floats per channel of a band
constexpr unsigned long long kNoSeg = ~0ull;   // no (range, key) pair takes this value
constexpr uint32_t kNoKey32 = 0xffffffffu;

// One Hillis-Steele step of a segmented inclusive scan inside rows of 16
// lanes: lane l adds lane l - D's partial when both lie in one row and one
// run (head = first lane of l's run).  The row shift is a DPP move, so all
// lanes must be active.
template <int D>
__device__ __forceinline__ void row_scan_step(float (&p)[12], int lane, int head) {
  const bool take = (lane & 15) >= D && lane - D >= head;
#pragma unroll
  for (int v = 0; v < 12; ++v) {
    const float o = __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(p[v]), 0x110 + D, 0xf, 0xf, false));
    p[v] = take ? p[v] + o : p[v];
  }
}

}  // namespace

// Gather plan: per level the band height, the bands per plane, the pieces K a
// band's entries are split into (K > 1 writes partial bands to scratch, summed
// in piece order afterwards), the first block and the scratch offset.
struct GatherPlan {
  int levels;
  int segs;
  int R[PDG_MAX_LEVELS];
  int B[PDG_MAX_LEVELS];                   // node rows per band
  int nb[PDG_MAX_LEVELS];                  // bands per plane
  int K[PDG_MAX_LEVELS];                   // pieces per band
  long long bfirst[PDG_MAX_LEVELS + 1];    // first block of each level
  long long roff2[PDG_MAX_LEVELS];         // first row of each level in a segment
  long long sof[PDG_MAX_LEVELS];           // scratch float offset of each level
  long long RS2;                           // rows per segment
  long long scratch;                       // scratch floats in all
  int ch0;                                 // first channel written (of g.ch)
};

namespace {

__global__ __launch_bounds__(kGatherThreads, 5) void gather_kernel(GridDev g, GatherPlan gp,
                                                                ScatterLists sl,
                                                                float *__restrict__ grad,
                                                                float *__restrict__ scratch) {
  __shared__ float band[3 * kBandFloats];
  __shared__ float wtail[kGatherThreads / 64][12];   // per-wave scan totals
  __shared__ unsigned long long skey[kGatherThreads + 1];   // (range << 32) | key
  __shared__ float carry[2][12];
  __shared__ unsigned s_mask[2];             // (range, class) rounds with runs ending
  const long long blk = blockIdx.x;
  int l = 0;
  while (l + 1 < gp.levels && blk >= gp.bfirst[l + 1]) ++l;
  const int R = gp.R[l], B = gp.B[l], nb = gp.nb[l], K = gp.K[l];
  long long local = blk - gp.bfirst[l];
  const int piece = (int)(local % K);
  local /= K;
  const int bi = (int)(local % nb);
  const long long rest = local / nb;
  const int z = (int)(rest % R);
  const long long seg = rest / R;
  const int y0 = bi * B, y1 = y0 + B < R ? y0 + B : R, rows = y1 - y0;
  const int t = threadIdx.x;
  const int band_n = rows * R;
  for (int i = t; i < 3 * band_n; i += kGatherThreads) band[i] = 0.f;

  // the (list, cell plane) ranges of this band, in a fixed order; their
  // bounds are fetched by eight threads at once
  __shared__ int rlo[4], rlen[4], rli[4], rdz[4], s_total, s_bound[8];
  const int zc_max = R > 1 ? R - 2 : 0;
  const int cy_lo = y0 > 0 ? y0 - 1 : 0, cy_hi = y1 - 1 < zc_max ? y1 - 1 : zc_max;
  if (t < 8) {
    const int li = t >> 2, pass = (t >> 1) & 1, hi = t & 1;
    const int zc = z - 1 + pass;
    int v = 0;
    if (li < sl.count && zc >= 0 && zc <= zc_max && cy_lo <= cy_hi) {
      const long long row = seg * gp.RS2 + gp.roff2[l] + (long long)zc * R;
      v = sl.list[li].pstart[row + (hi ? cy_hi + 1 : cy_lo)];
    }
    s_bound[t] = v;
  }
  __syncthreads();
  if (t == 0) {
    int nr = 0, total = 0;
    for (int q = 0; q < 4; ++q) {
      const int lo = s_bound[2 * q], hi = s_bound[2 * q + 1];
      if (hi <= lo) continue;
      rlo[nr] = lo;
      rlen[nr] = hi - lo;
      rli[nr] = q >> 1;
      rdz[nr] = 1 - (q & 1);                 // cell plane z - 1: dz = 1; z: dz = 0
      total += hi - lo;
      ++nr;
    }
    s_total = total;
  }
  const long long kbase = seg * g.nodes + g.noff[l];
  bool carried = false;
  __syncthreads();
  // this piece's part of the concatenated ranges: entries [cbeg, total)
  const int cbeg = (int)((long long)s_total * piece / K);
  const int total = (int)((long long)s_total * (piece + 1) / K);
  // entry v of the concatenated ranges: (range, sorted index)
  auto locate = [&](int v, int &r) {
    r = 0;
    while (v >= rlen[r]) v -= rlen[r++];
    return rlo[r] + v;
  };
  // this thread's entry of the next chunk, fetched one chunk ahead
  uint32_t nkey = kNoKey32;
  float4 ne = make_float4(0.f, 0.f, 0.f, 0.f);
  float2 ne2 = make_float2(0.f, 0.f);
  int nrng = 0;
  auto fetch = [&](int v) {
    if (v < total) {
      const int i = locate(v, nrng);
      const ScatterList &L = sl.list[rli[nrng]];
      nkey = L.keys[i];
      ne = L.ent[i];
      ne2 = L.ent2[i];
    }
  };
  fetch(cbeg + t);
  for (int c0 = cbeg, chunk = 0; c0 < total; c0 += kGatherThreads, ++chunk) {
    const int n = total - c0 < kGatherThreads ? total - c0 : kGatherThreads;
    const uint32_t ckey = nkey;
    const float4 ce = ne;
    const float2 ce2 = ne2;
    const int crng = nrng;
    nkey = kNoKey32;
    fetch(c0 + kGatherThreads + t);        // in flight during this chunk
    if (t == 0) s_mask[chunk & 1] = 0u;
    float p[12];
    unsigned long long key = kNoSeg;
    int my_range = -1;
    if (t < n) {
      my_range = crng;
      key = ((unsigned long long)crng << 32) | ckey;
      const float lv[3] = {ce.w, ce2.x, ce2.y};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float w = corner_weight(q | (rdz[crng] << 2), ce.x, ce.y, ce.z);
#pragma unroll
        for (int c = 0; c < 3; ++c) p[4 * c + q] = w * lv[c];
      }
      if (t == 0 && carried) {
#pragma unroll
        for (int v2 = 0; v2 < 12; ++v2) p[v2] = carry[(chunk + 1) & 1][v2] + p[v2];
      }
      skey[t] = key;
    }
    if (t == 0) {
      // the next chunk's first entry is this thread's prefetched one
      skey[n] = c0 + n < total ? (((unsigned long long)nrng << 32) | nkey) : kNoSeg;
    }
    if (t >= n) {
#pragma unroll
      for (int v2 = 0; v2 < 12; ++v2) p[v2] = 0.f;
    }
    // segmented inclusive scan within the wave (all lanes active here)
    const int lane = t & 63, wv = t >> 6;
    int head;                                // first lane of this lane's run
    {
      const unsigned klo = (unsigned)key, khi = (unsigned)(key >> 32);
      const unsigned plo = __shfl_up(klo, 1, 64), phi = __shfl_up(khi, 1, 64);
      const unsigned long long starts = __ballot(lane == 0 || plo != klo || phi != khi);
      const unsigned long long upto = lane == 63 ? ~0ull : (2ull << lane) - 1;
      head = 63 - __clzll(starts & upto);
    }
    row_scan_step<1>(p, lane, head);
    row_scan_step<2>(p, lane, head);
    row_scan_step<4>(p, lane, head);
    row_scan_step<8>(p, lane, head);
    // across rows in order: the last lane of row r - 1 already holds its
    // run's sum up to there
#pragma unroll
    for (int r = 1; r < 4; ++r) {
      const bool take = (lane >> 4) == r && head <= 16 * r - 1;
#pragma unroll
      for (int v2 = 0; v2 < 12; ++v2) {
        const float o = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(p[v2]), 16 * r - 1));
        p[v2] = take ? o + p[v2] : p[v2];
      }
    }
    if (lane == 63) {
#pragma unroll
      for (int v2 = 0; v2 < 12; ++v2) wtail[wv][v2] = p[v2];
    }
    __syncthreads();                         // skey, wave tails
    // carry into this wave's leading run from the (fully used) waves before it
    if (wv > 0 && 64 * wv < n) {
      const unsigned long long k0 = skey[64 * wv];
      if (key == k0) {
        float cin[12];
#pragma unroll
        for (int v2 = 0; v2 < 12; ++v2) cin[v2] = 0.f;
        for (int j = wv - 1; j >= 0; --j) {
          if (skey[64 * j + 63] != k0) break;
#pragma unroll
          for (int v2 = 0; v2 < 12; ++v2) cin[v2] += wtail[j][v2];
          if (skey[64 * j] != k0) break;       // the run starts inside wave j
        }
#pragma unroll
        for (int v2 = 0; v2 < 12; ++v2) p[v2] = cin[v2] + p[v2];
      }
    }
    const bool next_carried = skey[n - 1] == skey[n];
    const bool last = t < n && skey[t + 1] != key;     // last entry of its run in this chunk
    if (t == n - 1 && next_carried) {
#pragma unroll
      for (int v2 = 0; v2 < 12; ++v2) carry[chunk & 1][v2] = p[v2];
    }
    const int cell = last ? (int)((long long)(uint32_t)key - kbase) : 0;
    const int cx = cell % R, cy = (cell / R) % R;
    const int cls = last ? (cx & 1) | ((cy & 1) << 1) : -1;
    {
      // rounds present: OR over the wave first, then one LDS atomic per wave
      unsigned bits = cls >= 0 ? 1u << (4 * my_range + cls) : 0u;
      for (int o = 32; o > 0; o >>= 1) bits |= __shfl_xor(bits, o, 64);
      if (lane == 0 && bits) atomicOr(&s_mask[chunk & 1], bits);
    }
    __syncthreads();
    // only the (range, class) rounds that have runs ending in this chunk
    for (unsigned m = s_mask[chunk & 1]; m; m &= m - 1) {
      const int bit = __builtin_ctz(m);
      if (cls == (bit & 3) && my_range == (bit >> 2)) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int x = cx + (q & 1), y = cy + (q >> 1);
          if (x < R && y >= y0 && y < y1) {
            const int o = (y - y0) * R + x;
#pragma unroll
            for (int c = 0; c < 3; ++c)
              band[c * band_n + o] = __fmaf_rn(g.scale, p[4 * c + q], band[c * band_n + o]);
          }
        }
      }
      __syncthreads();
    }
    carried = next_carried;
  }
  __syncthreads();
  const long long R2 = (long long)R * R, R3 = R2 * R;
  float *Gd = (K == 1 ? grad + seg * g.size + g.off[l] + gp.ch0 * R3
                      : scratch + gp.sof[l] + ((long long)piece * gp.segs + seg) * 3 * R3) +
              (long long)z * R2 + (long long)y0 * R;
  for (int i = t; i < band_n; i += kGatherThreads) {
    __builtin_nontemporal_store(band[i], &Gd[i]);   // read once, by the next stage
    __builtin_nontemporal_store(band[band_n + i], &Gd[R3 + i]);
    __builtin_nontemporal_store(band[2 * band_n + i], &Gd[2 * R3 + i]);
  }
}

// grad = sum over pieces k (in order) of the partial bands, for the levels
// split into K > 1 pieces; one thread per (level part, float).
__global__ __launch_bounds__(256) void gather_reduce_kernel(GridDev g, GatherPlan gp,
                                                            const float *__restrict__ scratch,
                                                            float *__restrict__ grad) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  for (int l = 0; l < gp.levels; ++l) {
    if (gp.K[l] == 1) continue;
    const long long r3 = (long long)gp.R[l] * gp.R[l] * gp.R[l];
    const long long per = 3 * r3;                   // floats per segment (three channels)
    const long long n = per * gp.segs;
    if (i < n) {
      const long long seg = i / per, c = i - seg * per;
      const float *src = scratch + gp.sof[l] + i;
      // pieces added in order; their loads issued sixteen at a time
      const int K = gp.K[l];
      float v = src[0];
      int k = 1;
      for (; k + 16 <= K; k += 16) {
        float t[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) t[j] = src[(long long)(k + j) * n];
#pragma unroll
        for (int j = 0; j < 16; ++j) v += t[j];
      }
      for (; k < K; ++k) v += src[(long long)k * n];
      grad[seg * g.size + g.off[l] + gp.ch0 * r3 + c] = v;
      return;
    }
    i -= n;
  }
}

}  // namespace

pdg_status launch_warp(const GridDev &g, const float *grids, long long gstride, const float *x,
                       long long xstride, long long ldx, float *out, long long ostride,
                       long long ldo, long long n, int batch, hipStream_t st, const int *order,
                       long long order_stride) {
  if (n <= 0 || batch <= 0) return PDG_OK;
  const unsigned nb = div_up(n, 256);
  const unsigned long long blocks = job_grid(batch, nb);
  if (blocks >= (1ull << 31)) {
    set_error("warp: %llu workgroups exceed the launch limit", blocks);
    return PDG_EINVAL;
  }
  warp_kernel<<<(unsigned)blocks, 256, 0, st>>>(g, grids, gstride, x, xstride, ldx, out, ostride,
                                                ldo, n, order, order_stride, batch, nb);
  return launched("warp");
}

// Small launches (a template chain's single transition) take 64-thread
// workgroups so that the work spreads over every CU.
static int six_threads(long long n, int batch) {
  return div_up(n, 256) * (long long)batch < 1024 ? 64 : 256;
}

pdg_status launch_warp6_batch(const GridDev &g, const float *grids, long long gs, const float *x,
                              long long xs, float *out, long long os, long long n, int batch,
                              hipStream_t st) {
  if (n <= 0 || batch <= 0) return PDG_OK;
  const int nt = six_threads(n, batch);
  warp6_kernel<<<dim3(div_up(n, nt), batch), nt, 0, st>>>(g, grids, gs, x, xs, out, os, n);
  return launched("warp6");
}

pdg_status launch_warp6(const GridDev &g, const float *grids, const float *x, float *out,
                        long long n, hipStream_t st) {
  return launch_warp6_batch(g, grids, 0, x, 0, out, 0, n, 1, st);
}

pdg_status launch_adjoint6_batch(const GridDev &g, const float *grids, long long gs,
                                 const float *x, long long xs, const float *gout, long long gos,
                                 float *u, long long us, float *gx, const float *gx_add,
                                 long long gxs, long long n, int batch, hipStream_t st) {
  if (n <= 0 || batch <= 0 || (!u && !gx)) return PDG_OK;
  const int nt = six_threads(n, batch);
  adjoint6_kernel<<<dim3(div_up(n, nt), batch), nt, 0, st>>>(g, grids, gs, x, xs, gout, gos, u, us,
                                                             gx, gx ? gx_add : nullptr, gxs, n);
  return launched("adjoint6");
}

pdg_status launch_adjoint6(const GridDev &g, const float *grids, const float *x,
                           const float *gout, float *u, float *gx, long long n, hipStream_t st) {
  return launch_adjoint6_batch(g, grids, 0, x, 0, gout, 0, u, 0, gx, nullptr, 0, n, 1, st);
}

pdg_status launch_chain_warp6(const GridDev &g, const float *params, long long P, float *xhat,
                              long long V, int T, hipStream_t st) {
  if (V <= 0 || T <= 0) return PDG_OK;
  chain_warp6_kernel<<<div_up(V, 64), 64, 0, st>>>(g, params, P, xhat, V, T);
  return launched("chain_warp6");
}

pdg_status launch_chain_reverse6(const GridDev &g, const float *params, long long P,
                                 const float *xhat, const float *gd, float *lam, float *u,
                                 long long V, int T, hipStream_t st) {
  if (V <= 0 || T <= 0) return PDG_OK;
  chain_reverse6_kernel<<<div_up(V, 64), 64, 0, st>>>(g, params, P, xhat, gd, lam, u, V, T);
  return launched("chain_reverse6");
}

pdg_status launch_chain_adjoint(const GridDev &g, const float *grids, const float *x, long long ldx,
                                const float *lam, long long ldl, const float *gdir, long long ldd,
                                float *lam_out, long long ldo, long long n, hipStream_t st) {
  if (n <= 0) return PDG_OK;
  chain_adjoint_kernel<<<div_up(n, 256), 256, 0, st>>>(g, grids, x, ldx, lam, ldl, gdir, ldd,
                                                       lam_out, ldo, n);
  return launched("chain_adjoint");
}

pdg_status launch_chain_warp(const GridDev &g, const float *params, long long P, const float *x0,
                             float *xhat, long long V, int T, const int *order, hipStream_t st) {
  if (V <= 0) return PDG_OK;
  if (g.levels <= 8)
    chain_warp_kernel<8><<<div_up(V * 8, 256), 256, 0, st>>>(g, params, P, x0, xhat, V, T, order);
  else
    chain_warp_kernel<16><<<div_up(V * 16, 256), 256, 0, st>>>(g, params, P, x0, xhat, V, T, order);
  return launched("chain_warp");
}

pdg_status launch_chain_reverse(const GridDev &g, const float *params, long long P,
                                const float *xhat, const float *gd, float *lam, long long V, int T,
                                const int *order, hipStream_t st) {
  if (V <= 0 || T <= 0) return PDG_OK;
  if (g.levels <= 8)
    chain_reverse_kernel<8><<<div_up(V * 8, 256), 256, 0, st>>>(g, params, P, xhat, gd, lam, V, T,
                                                                order);
  else
    chain_reverse_kernel<16><<<div_up(V * 16, 256), 256, 0, st>>>(g, params, P, xhat, gd, lam, V,
                                                                  T, order);
  return launched("chain_reverse");
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

namespace {
__global__ __launch_bounds__(256) void add_kernel(float *__restrict__ dst,
                                                  const float *__restrict__ src, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] += src[i];
}
}  // namespace

pdg_status launch_add(float *dst, const float *src, long long count, hipStream_t st) {
  if (count <= 0) return PDG_OK;
  long long blocks = div_up(count, 256);
  if (blocks > 65536) blocks = 65536;
  add_kernel<<<(unsigned)blocks, 256, 0, st>>>(dst, src, count);
  return launched("add");
}

GridDev half_view(const GridDev &g, int half) {
  GridDev v = g;
  v.ch = 3;
  for (int l = 0; l < g.levels; ++l)
    v.off[l] = g.off[l] + (long long)half * 3 * g.res[l] * g.res[l] * g.res[l];
  return v;
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

long long row_count(const GridDev &g) {
  long long rs = 0;
  for (int l = 0; l < g.levels; ++l) rs += (long long)g.res[l] * g.res[l];
  return rs;
}

pdg_status launch_row_table(const GridDev &g, const uint32_t *keys, long long nent, int segs,
                            int *rstart, hipStream_t st) {
  const long long RS2 = row_count(g);
  const long long nrows = segs * RS2;
  row_table_kernel<<<div_up(nrows + 1, 256), 256, 0, st>>>(g, keys, (int)nent, (uint32_t)RS2,
                                                             (uint32_t)nrows, rstart);
  return launched("row_table");
}

pdg_status launch_scatter_stage(const GridDev &g, int segs, const ScatterList &L, hipStream_t st,
                                bool lam_only) {
  const long long nent = (long long)segs * g.levels * L.S;
  if (nent <= 0) return PDG_OK;
  scatter_stage_kernel<<<xcd_pad(div_up(nent, 256)), 256, 0, st>>>(g, L, (int)nent,
                                                                   lam_only ? 1 : 0);
  return launched("scatter_stage");
}

GatherPlan gather_plan(const GridDev &g, int segs, long long samples) {
  GatherPlan gp;
  memset(&gp, 0, sizeof gp);
  gp.levels = g.levels;
  gp.segs = segs;
  gp.RS2 = row_count(g);
  long long blocks = 0, roff = 0, sof = 0;
  for (int l = 0; l < g.levels; ++l) {
    const int R = g.res[l];
    int B = kBandFloats / R;
    if (B < 1) B = 1;
    if (B > R) B = R;
    // entries of a band if the samples spread evenly: two cell planes of
    // B + 1 rows; split into pieces of about six chunks, at most 16 or as
    // many as 2^22 floats of partial bands allow (coarse levels of many
    // samples), at most 512
    const double per_band = 2.0 * (double)samples * (B + 1) / ((double)R * R);
    const double per_piece = 3.0 * (double)R * R * R * segs;
    double kmax = (double)(1 << 22) / per_piece;
    kmax = kmax < 16.0 ? 16.0 : (kmax > 512.0 ? 512.0 : kmax);
    double kf = per_band / (6.0 * kGatherThreads);
    kf = kf < 1.0 ? 1.0 : (kf > kmax ? kmax : kf);
    const int K = (int)kf;
    gp.R[l] = R;
    gp.B[l] = B;
    gp.nb[l] = (R + B - 1) / B;
    gp.K[l] = K;
    gp.bfirst[l] = blocks;
    gp.roff2[l] = roff;
    gp.sof[l] = sof;
    blocks += (long long)segs * R * gp.nb[l] * K;
    roff += (long long)R * R;
    if (K > 1) sof += (long long)K * segs * 3 * R * R * R;
  }
  gp.bfirst[g.levels] = blocks;
  gp.scratch = sof;
  return gp;
}

size_t gather_scratch_bytes(const GridDev &g, int segs, long long samples) {
  return (size_t)gather_plan(g, segs, samples).scratch * sizeof(float);
}

pdg_status launch_gather(const GridDev &g, int segs, const ScatterLists &sl, long long samples,
                         float *grad, float *scratch, hipStream_t st, int ch0) {
  if (segs <= 0) return PDG_OK;
  if (ch0 < 0 || ch0 + 3 > g.ch) {
    set_error("gather: channels %d..%d outside the %d of the grid", ch0, ch0 + 2, g.ch);
    return PDG_EINVAL;
  }
  GatherPlan gp = gather_plan(g, segs, samples);
  gp.ch0 = ch0;
  const long long blocks = gp.bfirst[g.levels];
  if (blocks >= (1ll << 31)) {
    set_error("grid gather needs %lld blocks (limit 2^31)", blocks);
    return PDG_EINVAL;
  }
  if (gp.scratch > 0 && !scratch) {
    set_error("grid gather needs %lld floats of scratch", gp.scratch);
    return PDG_EINVAL;
  }
  gather_kernel<<<(unsigned)blocks, kGatherThreads, 0, st>>>(g, gp, sl, grad, scratch);
  PDG_TRY(launched("gather"));
  long long red = 0;
  for (int l = 0; l < g.levels; ++l)
    if (gp.K[l] > 1) red += 3ll * g.res[l] * g.res[l] * g.res[l] * segs;
  if (red > 0) {
    gather_reduce_kernel<<<div_up(red, 256), 256, 0, st>>>(g, gp, scratch, grad);
    PDG_TRY(launched("gather_reduce"));
  }
  return PDG_OK;
}

}  // namespace pdg
