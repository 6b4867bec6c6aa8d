// Grid Sobolev preconditioner (paper Sec. 3.2, Eq. 3): g <- (I + lam L)^-2 g
// per (stack, level, channel) system, L the 6-neighbour combinatorial
// Laplacian of the R^3 cell box with free boundary.
//
// Two conjugate-gradient solves per system, matrix-free, float32 vectors and
// float64 inner products, with a fixed per-level iteration count (so the whole
// solve is stream-ordered with no host synchronisation).
//
// Work decomposition: systems are numbered level-major (level, stack,
// channel); a tile is 2048 consecutive cells of one system (whole x-rows for
// R >= 64).  Each launch covers the tiles of the levels still iterating, with
// the workgroup -> tile map made XCD-aware (consecutive workgroups land on
// different XCDs, so each XCD gets a contiguous run of tiles and the z-planes
// its stencil touches stay in its L2).  A thread owns float4 quads along x;
// x-neighbours come from the quad itself plus two scalar loads, y/z
// neighbours are float4 loads served mostly from cache.
//
// Per iteration (p' = r + beta p, ping-pong buffers for p):
//   kernel A: p' from r and p, pq = <p', A p'> (A p' at the seven stencil
//             points from r and p), writes p';
//   reduce  : alpha = rr / pq;
//   kernel B: x += alpha p', r -= alpha A p' (stencil on p'), rr' = <r, r>;
//   reduce  : beta = rr' / rr.
// HBM traffic per cell and iteration: A reads r, p and writes p' (12 B);
// B reads p', x, r and writes x, r (20 B).
//
// Pruned grids (Sec. 3.6): with a mask the operator is I + lam L_S, L_S the
// Laplacian of the graph the kept cells induce.  The residual starts at zero
// on pruned cells and A p' is zero there, so r, p and x stay zero on them; a
// kept cell sees a pruned neighbour as missing (the neighbour's value is
// replaced by the cell's own, difference 0, selected and never multiplied, so
// stale values never enter).  Tiles without a kept cell return at once, and
// inside a kept tile a float4 quad without a kept cell is skipped (it adds
// exactly zero to both inner products): their p values are never written, and
// no kept cell uses them, so the traffic follows the kept quads.  The kept
// quads of a tile are listed in LDS (in index order) and dealt to the block's
// threads in turn, so that lanes do not idle on empty quads.
#include "common.h"

namespace pdg {
namespace {

constexpr int kThreads = 256;
constexpr int kQuads = 2;                            // float4 quads per thread
constexpr int kTileCells = kThreads * 4 * kQuads;    // 2048

struct CGState {
  float *x, *r, *p0, *p1;
  double *pq_part, *rr_part;   // [ntiles]
  double *rr, *alpha, *beta;   // [nsys]
};

struct Loc {                   // a workgroup's tile
  int l;                       // level
  int sys;                     // global system index
  int lt;                      // tile within the system
  long long base;              // float offset of the system
  const uint32_t *mk;          // the level's mask words of the system's stack
};

__device__ __forceinline__ bool locate(const CGPlanDev &P, int tile, Loc &o) {
  for (int l = 0; l < P.levels; ++l) {
    const CGLevel &L = P.lv[l];
    const int nt = P.batch * 3 * L.tps;
    if (tile >= L.tile0 && tile < L.tile0 + nt) {
      const int local = tile - L.tile0;
      const int s = local / L.tps;
      o.l = l;
      o.sys = L.sys0 + s;
      o.lt = local - s * L.tps;
      const long long r3 = (long long)L.R * L.R * L.R;
      o.base = (long long)(s / 3) * P.stack + L.off + (long long)(s % 3) * r3;
      o.mk = P.mask ? P.mask + (long long)(s / 3) * P.mstack + L.moff : nullptr;
      return true;
    }
  }
  return false;
}

// workgroup -> tile inside [lo, lo + n): each XCD gets a contiguous range
__device__ __forceinline__ int tile_of_block(int lo, int n) {
  const int per = (n + 7) >> 3;
  return lo + (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kThreads / 64; ++i) t += sh[i];
  return t;
}

__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ void st4(float *p, float4 v) { *reinterpret_cast<float4 *>(p) = v; }
// streams a pass reads or writes once (no stencil neighbour reads them in the
// same pass): past the caches
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld4nt(const float *p) {
  const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4nt(float *p, float4 x) {
  const nt_f4 v = {x.x, x.y, x.z, x.w};
  __builtin_nontemporal_store(v, reinterpret_cast<nt_f4 *>(p));
}
__device__ __forceinline__ float4 axpy4(float4 a, float b, float4 c) {
  return make_float4(a.x + b * c.x, a.y + b * c.y, a.z + b * c.z, a.w + b * c.w);
}

// Laplacian part sum_nbr (v - v_nbr) of a quad c given its neighbours; a
// missing neighbour is passed as the cell itself (difference 0).
__device__ __forceinline__ float4 lap4(float4 c, float xl, float xr, float4 ym, float4 yp,
                                       float4 zm, float4 zp) {
  float4 s;
  s.x = (c.x - xl) + (c.x - c.y) + (c.x - ym.x) + (c.x - yp.x) + (c.x - zm.x) + (c.x - zp.x);
  s.y = (c.y - c.x) + (c.y - c.z) + (c.y - ym.y) + (c.y - yp.y) + (c.y - zm.y) + (c.y - zp.y);
  s.z = (c.z - c.y) + (c.z - c.w) + (c.z - ym.z) + (c.z - yp.z) + (c.z - zm.z) + (c.z - zp.z);
  s.w = (c.w - c.z) + (c.w - xr) + (c.w - ym.w) + (c.w - yp.w) + (c.w - zm.w) + (c.w - zp.w);
  return s;
}

__device__ __forceinline__ double dot4(float4 a, float4 b) {
  return (double)a.x * b.x + (double)a.y * b.y + (double)a.z * b.z + (double)a.w * b.w;
}

// kept-cell bits (pruned grids)
__device__ __forceinline__ unsigned bit1(const uint32_t *mk, int c) { return (mk[c >> 5] >> (c & 31)) & 1u; }
// the four bits of cells q .. q + 3 (q % 4 == 0: one word)
__device__ __forceinline__ unsigned nib4(const uint32_t *mk, int q) { return (mk[q >> 5] >> (q & 31)) & 15u; }

// Laplacian part on the induced graph: as lap4, with a neighbour whose bit is
// clear (pruned, or outside the box) treated as missing.  xl/xr: bits of the
// x-neighbours of the quad's ends; own, ym..zp: four-bit masks.
__device__ __forceinline__ float4 lap4m(float4 c, float xl, float xr, float4 ym, float4 yp,
                                        float4 zm, float4 zp, unsigned own, unsigned bl,
                                        unsigned br, unsigned bym, unsigned byp, unsigned bzm,
                                        unsigned bzp) {
  auto d = [](float self, unsigned on, float nb) { return on ? self - nb : 0.0f; };
  float4 s;
  s.x = d(c.x, bl, xl) + d(c.x, own & 2u, c.y) + d(c.x, bym & 1u, ym.x) + d(c.x, byp & 1u, yp.x) +
        d(c.x, bzm & 1u, zm.x) + d(c.x, bzp & 1u, zp.x);
  s.y = d(c.y, own & 1u, c.x) + d(c.y, own & 4u, c.z) + d(c.y, bym & 2u, ym.y) +
        d(c.y, byp & 2u, yp.y) + d(c.y, bzm & 2u, zm.y) + d(c.y, bzp & 2u, zp.y);
  s.z = d(c.z, own & 2u, c.y) + d(c.z, own & 8u, c.w) + d(c.z, bym & 4u, ym.z) +
        d(c.z, byp & 4u, yp.z) + d(c.z, bzm & 4u, zm.z) + d(c.z, bzp & 4u, zp.z);
  s.w = d(c.w, own & 4u, c.z) + d(c.w, br, xr) + d(c.w, bym & 8u, ym.w) + d(c.w, byp & 8u, yp.w) +
        d(c.w, bzm & 8u, zm.w) + d(c.w, bzp & 8u, zp.w);
  return s;
}

// A p on the induced graph (zero on pruned cells)
__device__ __forceinline__ float4 apply4m(float4 c, float lam, float4 lap, unsigned own) {
  return make_float4((own & 1u) ? c.x + lam * lap.x : 0.0f, (own & 2u) ? c.y + lam * lap.y : 0.0f,
                     (own & 4u) ? c.z + lam * lap.z : 0.0f, (own & 8u) ? c.w + lam * lap.w : 0.0f);
}

__device__ __forceinline__ float4 keep4(float4 c, unsigned own) {
  return make_float4((own & 1u) ? c.x : 0.0f, (own & 2u) ? c.y : 0.0f, (own & 4u) ? c.z : 0.0f,
                     (own & 8u) ? c.w : 0.0f);
}

// true when the workgroup's tile holds a kept cell (block-uniform)
__device__ __forceinline__ bool tile_kept(const uint32_t *mk, int lt, int n) {
  const int w0 = lt * (kTileCells / 32);
  const int nw = (n + 31) / 32;
  const int w = w0 + (int)threadIdx.x;
  const uint32_t v = (threadIdx.x < kTileCells / 32 && w < nw) ? mk[w] : 0u;
  return __syncthreads_or(v != 0u) != 0;
}

// The kept quads of a tile, in index order: kq[0 .. count) are the tile's
// quad numbers u * kThreads + t (cells lt * kTileCells + 4 * (u * kThreads + t))
// whose four cells hold a kept one; the block's threads then take them in
// turn, so no lane idles on an empty quad.  gcount: kQuads * kThreads / 64
// ints of LDS.  Block-uniform count.
__device__ __forceinline__ int kept_quads(const uint32_t *mk, int lt, int n, unsigned short *kq,
                                          int *gcount) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int kW = kThreads / 64;
  unsigned long long m[kQuads];
#pragma unroll
  for (int u = 0; u < kQuads; ++u) {
    const int q = lt * kTileCells + 4 * (u * kThreads + (int)threadIdx.x);
    m[u] = __ballot(q < n && nib4(mk, q) != 0u);
    if (lane == 0) gcount[u * kW + w] = __popcll(m[u]);
  }
  __syncthreads();
  int total = 0;
#pragma unroll
  for (int g = 0; g < kQuads * kW; ++g) total += gcount[g];
#pragma unroll
  for (int u = 0; u < kQuads; ++u) {
    int off = 0;   // kept quads of the (u, wave) groups before this one
    for (int g = 0; g < u * kW + w; ++g) off += gcount[g];
    if ((m[u] >> lane) & 1ull)
      kq[off + __popcll(m[u] & ((1ull << lane) - 1ull))] =
          (unsigned short)(u * kThreads + (int)threadIdx.x);
  }
  __syncthreads();
  return total;
}

// generic cell coordinates (any R)
__device__ __forceinline__ void coords(const CGLevel &L, int c, int &x, int &y, int &z) {
  if (L.shift >= 0) {
    x = c & (L.R - 1);
    y = (c >> L.shift) & (L.R - 1);
    z = c >> (2 * L.shift);
  } else {
    x = c % L.R;
    y = (c / L.R) % L.R;
    z = c / (L.R * L.R);
  }
}

// r = src on the kept cells (all cells without a mask), x = 0.  On a pruned
// cell r is never read unselected and x only matters where it is the solve's
// output (zero_x_pruned): the other stores are left out there (a kept quad
// writes all four cells of r and x; only its kept cells enter <r, r>).
// list (nullable): the launched tiles are list[0 .. ntiles).
__global__ __launch_bounds__(kThreads) void cg_init_kernel(CGPlanDev P, int ntiles,
                                                           const int *__restrict__ list,
                                                           const float *__restrict__ src,
                                                           float *__restrict__ r,
                                                           float *__restrict__ x,
                                                           double *__restrict__ rr_part,
                                                           int zero_x_pruned) {
  __shared__ double sh[kThreads / 64];
  int tile = tile_of_block(0, ntiles);
  if (tile >= ntiles) return;
  if (list) tile = list[tile];
  Loc o;
  if (!locate(P, tile, o)) return;
  const CGLevel &L = P.lv[o.l];
  const int n = L.R * L.R * L.R;
  double acc = 0.0;
  if (L.vec) {
    for (int u = 0; u < kQuads; ++u) {
      const int q = o.lt * kTileCells + u * (4 * kThreads) + 4 * threadIdx.x;
      if (q >= n) continue;
      const unsigned own = o.mk ? nib4(o.mk, q) : 15u;
      if (own == 0u) {
        if (zero_x_pruned) st4(x + o.base + q, make_float4(0.f, 0.f, 0.f, 0.f));
        continue;
      }
      const float4 v = ld4(src + o.base + q);
      st4(r + o.base + q, v);
      st4(x + o.base + q, make_float4(0.f, 0.f, 0.f, 0.f));
      const float4 kv = keep4(v, own);
      acc += dot4(kv, kv);
    }
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) rr_part[tile] = t;
    return;
  }
  for (int k = 0; k < 4 * kQuads; ++k) {
    const int c = o.lt * kTileCells + k * kThreads + threadIdx.x;
    if (c < n) {
      if (o.mk && !bit1(o.mk, c)) {
        if (zero_x_pruned) x[o.base + c] = 0.f;
        continue;
      }
      const float v = src[o.base + c];
      r[o.base + c] = v;
      x[o.base + c] = 0.f;
      acc += (double)v * v;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) rr_part[tile] = t;
}

template <bool MASK>
__global__ __launch_bounds__(kThreads) void cg_a_kernel(CGPlanDev P, int k, int tile_lo, int nlaunch,
                                                        CGState s, const float *__restrict__ pin,
                                                        float *__restrict__ pout) {
  __shared__ double sh[kThreads / 64];
  __shared__ unsigned short kq[kQuads * kThreads];   // the tile's kept quads (masked)
  __shared__ int gcount[kQuads * kThreads / 64];
  int tile = tile_of_block(tile_lo, nlaunch);
  if (tile >= tile_lo + nlaunch) return;
  if (P.klist) tile = P.klist[tile];          // listed tiles hold a kept cell
  Loc o;
  if (!locate(P, tile, o)) return;
  const CGLevel &L = P.lv[o.l];
  if (k >= L.iters) return;
  const int R = L.R;
  const int n = R * R * R;
  if (MASK && !P.klist && !tile_kept(o.mk, o.lt, n)) {
    if (threadIdx.x == 0) s.pq_part[tile] = 0.0;
    return;
  }
  const float beta = k == 0 ? 0.f : (float)s.beta[o.sys];
  const float lam = L.lam;
  const float *rr = s.r + o.base;
  const float *pp = pin + o.base;
  float *po = pout + o.base;
  double acc = 0.0;
  if (L.vec) {
    const int RR = R * R;
    auto quad = [&](int q) {
      int x0, y, z;
      coords(L, q, x0, y, z);
      auto pn = [&](int i) { return k == 0 ? rr[i] : rr[i] + beta * pp[i]; };
      auto pn4 = [&](int i) { return k == 0 ? ld4(rr + i) : axpy4(ld4(rr + i), beta, ld4(pp + i)); };
      float4 c = pn4(q);
      const float xl = x0 > 0 ? pn(q - 1) : c.x;
      const float xr = x0 + 4 < R ? pn(q + 4) : c.w;
      const float4 ym = y > 0 ? pn4(q - R) : c;
      const float4 yp = y < R - 1 ? pn4(q + R) : c;
      const float4 zm = z > 0 ? pn4(q - RR) : c;
      const float4 zp = z < R - 1 ? pn4(q + RR) : c;
      float4 ap;
      if (MASK) {
        const unsigned own = nib4(o.mk, q);
        const unsigned bl = x0 > 0 ? bit1(o.mk, q - 1) : 0u;
        const unsigned br = x0 + 4 < R ? bit1(o.mk, q + 4) : 0u;
        const unsigned bym = y > 0 ? nib4(o.mk, q - R) : 0u;
        const unsigned byp = y < R - 1 ? nib4(o.mk, q + R) : 0u;
        const unsigned bzm = z > 0 ? nib4(o.mk, q - RR) : 0u;
        const unsigned bzp = z < R - 1 ? nib4(o.mk, q + RR) : 0u;
        c = keep4(c, own);
        ap = apply4m(c, lam, lap4m(c, xl, xr, ym, yp, zm, zp, own, bl, br, bym, byp, bzm, bzp), own);
      } else {
        ap = axpy4(c, lam, lap4(c, xl, xr, ym, yp, zm, zp));
      }
      st4nt(po + q, c);
      acc += dot4(c, ap);
    };
    if (MASK) {
      // a quad without a kept cell adds exactly zero to <p', A p'>: only the
      // kept quads are visited (the others' p values are never read
      // unselected)
      const int cnt = kept_quads(o.mk, o.lt, n, kq, gcount);
#pragma unroll 1
      for (int j = threadIdx.x; j < cnt; j += kThreads) quad(o.lt * kTileCells + 4 * (int)kq[j]);
    } else {
      for (int u = 0; u < kQuads; ++u) {
        const int q = o.lt * kTileCells + u * (4 * kThreads) + 4 * threadIdx.x;
        if (q < n) quad(q);
      }
    }
  } else {
    auto pn = [&](int i) { return k == 0 ? rr[i] : rr[i] + beta * pp[i]; };
    auto on = [&](int i) { return !MASK || bit1(o.mk, i) != 0u; };
    for (int e = 0; e < 4 * kQuads; ++e) {
      const int c = o.lt * kTileCells + e * kThreads + threadIdx.x;
      if (c >= n) continue;
      if (MASK && !on(c)) {
        po[c] = 0.f;
        continue;
      }
      int x, y, z;
      coords(L, c, x, y, z);
      const float v = pn(c);
      float sm = 0.f;
      if (x > 0 && on(c - 1)) sm += v - pn(c - 1);
      if (x < R - 1 && on(c + 1)) sm += v - pn(c + 1);
      if (y > 0 && on(c - R)) sm += v - pn(c - R);
      if (y < R - 1 && on(c + R)) sm += v - pn(c + R);
      if (z > 0 && on(c - R * R)) sm += v - pn(c - R * R);
      if (z < R - 1 && on(c + R * R)) sm += v - pn(c + R * R);
      po[c] = v;
      acc += (double)v * (double)(v + lam * sm);
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) s.pq_part[tile] = t;
}

template <bool MASK>
__global__ __launch_bounds__(kThreads, 8) void cg_b_kernel(CGPlanDev P, int k, int tile_lo, int nlaunch,
                                                        CGState s, const float *__restrict__ pcur) {
  __shared__ double sh[kThreads / 64];
  __shared__ unsigned short kq[kQuads * kThreads];   // the tile's kept quads (masked)
  __shared__ int gcount[kQuads * kThreads / 64];
  int tile = tile_of_block(tile_lo, nlaunch);
  if (tile >= tile_lo + nlaunch) return;
  if (P.klist) tile = P.klist[tile];
  Loc o;
  if (!locate(P, tile, o)) return;
  const CGLevel &L = P.lv[o.l];
  if (k >= L.iters) return;
  const int R = L.R;
  const int n = R * R * R;
  if (MASK && !P.klist && !tile_kept(o.mk, o.lt, n)) {
    if (threadIdx.x == 0) s.rr_part[tile] = 0.0;
    return;
  }
  const float alpha = (float)s.alpha[o.sys];
  const float lam = L.lam;
  const float *pp = pcur + o.base;
  float *xx = s.x + o.base;
  float *rr = s.r + o.base;
  double acc = 0.0;
  if (L.vec) {
    const int RR = R * R;
    auto quad = [&](int q) {
      int x0, y, z;
      coords(L, q, x0, y, z);
      const float4 c = ld4(pp + q);
      const float xl = x0 > 0 ? pp[q - 1] : c.x;
      const float xr = x0 + 4 < R ? pp[q + 4] : c.w;
      const float4 ym = y > 0 ? ld4(pp + q - R) : c;
      const float4 yp = y < R - 1 ? ld4(pp + q + R) : c;
      const float4 zm = z > 0 ? ld4(pp + q - RR) : c;
      const float4 zp = z < R - 1 ? ld4(pp + q + RR) : c;
      float4 ap;
      if (MASK) {
        const unsigned own = nib4(o.mk, q);
        const unsigned bl = x0 > 0 ? bit1(o.mk, q - 1) : 0u;
        const unsigned br = x0 + 4 < R ? bit1(o.mk, q + 4) : 0u;
        const unsigned bym = y > 0 ? nib4(o.mk, q - R) : 0u;
        const unsigned byp = y < R - 1 ? nib4(o.mk, q + R) : 0u;
        const unsigned bzm = z > 0 ? nib4(o.mk, q - RR) : 0u;
        const unsigned bzp = z < R - 1 ? nib4(o.mk, q + RR) : 0u;
        ap = apply4m(c, lam, lap4m(c, xl, xr, ym, yp, zm, zp, own, bl, br, bym, byp, bzm, bzp), own);
      } else {
        ap = axpy4(c, lam, lap4(c, xl, xr, ym, yp, zm, zp));
      }
      st4nt(xx + q, axpy4(ld4nt(xx + q), alpha, c));
      float4 rn = axpy4(ld4nt(rr + q), -alpha, ap);
      // the residual of a pruned cell is zero (its stored value is not kept
      // up to date: the set-up does not write it)
      if (MASK) rn = keep4(rn, nib4(o.mk, q));
      st4nt(rr + q, rn);
      acc += dot4(rn, rn);
    };
    if (MASK) {   // x and r stay zero on the quads without a kept cell
      const int cnt = kept_quads(o.mk, o.lt, n, kq, gcount);
#pragma unroll 1
      for (int j = threadIdx.x; j < cnt; j += kThreads) quad(o.lt * kTileCells + 4 * (int)kq[j]);
    } else {
      for (int u = 0; u < kQuads; ++u) {
        const int q = o.lt * kTileCells + u * (4 * kThreads) + 4 * threadIdx.x;
        if (q < n) quad(q);
      }
    }
  } else {
    auto on = [&](int i) { return !MASK || bit1(o.mk, i) != 0u; };
    for (int e = 0; e < 4 * kQuads; ++e) {
      const int c = o.lt * kTileCells + e * kThreads + threadIdx.x;
      if (c >= n) continue;
      if (MASK && !on(c)) continue;
      int x, y, z;
      coords(L, c, x, y, z);
      const float v = pp[c];
      float sm = 0.f;
      if (x > 0 && on(c - 1)) sm += v - pp[c - 1];
      if (x < R - 1 && on(c + 1)) sm += v - pp[c + 1];
      if (y > 0 && on(c - R)) sm += v - pp[c - R];
      if (y < R - 1 && on(c + R)) sm += v - pp[c + R];
      if (z > 0 && on(c - R * R)) sm += v - pp[c - R * R];
      if (z < R - 1 && on(c + R * R)) sm += v - pp[c + R * R];
      xx[c] += alpha * v;
      const float rn = rr[c] - alpha * (v + lam * sm);
      rr[c] = rn;
      acc += (double)rn * rn;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) s.rr_part[tile] = t;
}

// One workgroup per system of the launched levels.
// mode 0: rr = sum rr_part (after init); mode 1: alpha = rr / sum pq_part;
// mode 2: rr' = sum rr_part, beta = rr'/rr, rr = rr'.
__global__ __launch_bounds__(kThreads) void cg_reduce_kernel(CGPlanDev P, int k, int mode,
                                                             int sys_lo, CGState s) {
  __shared__ double sh[kThreads / 64];
  const int sys = sys_lo + blockIdx.x;
  int l = 0;
  while (l + 1 < P.levels && sys >= P.lv[l + 1].sys0) ++l;
  const CGLevel &L = P.lv[l];
  if (mode != 0 && k >= L.iters) return;
  const double *part = mode == 1 ? s.pq_part : s.rr_part;
  const int t0 = L.tile0 + (sys - L.sys0) * L.tps;
  double acc = 0.0;
  for (int i = threadIdx.x; i < L.tps; i += kThreads) acc += part[t0 + i];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    if (mode == 0) {
      s.rr[sys] = t;
    } else if (mode == 1) {
      s.alpha[sys] = t > 0.0 ? s.rr[sys] / t : 0.0;
    } else {
      const double old = s.rr[sys];
      s.beta[sys] = old > 0.0 ? t / old : 0.0;
      s.rr[sys] = t;
    }
  }
}


}  // namespace

CGPlanDev cg_make_plan(const GridDev &g, int batch, const float *lam, const int *iters,
                       bool aligned16) {
  CGPlanDev p;
  memset(&p, 0, sizeof p);
  p.levels = g.levels;
  p.batch = batch;
  p.stack = g.size;
  int tile = 0, sys = 0;
  for (int l = 0; l < g.levels; ++l) {
    CGLevel &L = p.lv[l];
    L.R = g.res[l];
    L.shift = -1;
    for (int s = 0; s < 12; ++s)
      if ((1 << s) == L.R) L.shift = s;
    L.iters = iters[l];
    L.lam = lam[l];
    L.off = g.off[l];
    L.tile0 = tile;
    const long long r3 = (long long)L.R * L.R * L.R;
    L.tps = (int)((r3 + kTileCells - 1) / kTileCells);
    L.sys0 = sys;
    L.vec = aligned16 && L.R % 4 == 0 && g.size % 4 == 0 && g.off[l] % 4 == 0 && L.R >= 4;
    tile += batch * 3 * L.tps;
    sys += batch * 3;
  }
  p.ntiles = tile;
  p.nsys = sys;
  return p;
}

size_t cg_bytes(long long floats, int nsys, int ntiles) {
  return 4 * a256((size_t)floats * 4) + 2 * a256((size_t)ntiles * 8) + 3 * a256((size_t)nsys * 8);
}

// The two reductions of an iteration whose span holds no kept tile (the
// partials stay as they are: alpha and beta follow from them unchanged).
static pdg_status run_reductions_only(const CGPlanDev &P, int k, int sys_lo, int sys_hi,
                                      const CGState &t, hipStream_t st) {
  cg_reduce_kernel<<<sys_hi - sys_lo, kThreads, 0, st>>>(P, k, 1, sys_lo, t);
  PDG_TRY(launched("cg_reduce"));
  cg_reduce_kernel<<<sys_hi - sys_lo, kThreads, 0, st>>>(P, k, 2, sys_lo, t);
  return launched("cg_reduce");
}

pdg_status run_cg(const CGPlanDev &P, float *g, long long floats, void *ws, hipStream_t st) {
  if (P.nsys <= 0 || P.ntiles <= 0) return PDG_OK;
  char *w = (char *)ws;
  CGState s;
  s.x = (float *)w;
  w += a256((size_t)floats * 4);
  s.r = (float *)w;
  w += a256((size_t)floats * 4);
  s.p0 = (float *)w;
  w += a256((size_t)floats * 4);
  s.p1 = (float *)w;
  w += a256((size_t)floats * 4);
  s.pq_part = (double *)w;
  w += a256((size_t)P.ntiles * 8);
  s.rr_part = (double *)w;
  w += a256((size_t)P.ntiles * 8);
  s.rr = (double *)w;
  w += a256((size_t)P.nsys * 8);
  s.alpha = (double *)w;
  w += a256((size_t)P.nsys * 8);
  s.beta = (double *)w;
  int kmax = 0;
  for (int l = 0; l < P.levels; ++l) kmax = P.lv[l].iters > kmax ? P.lv[l].iters : kmax;
  auto padded = [](int n) { return (unsigned)(((n + 7) / 8) * 8); };
  // listed launches leave the partials of unlisted tiles untouched: both dot
  // partials start at zero
  int nlisted = 0;
  if (P.klist) {
    for (int l = 0; l < P.levels; ++l) nlisted += P.kcount[l];
    PDG_TRY(launch_fill((float *)s.pq_part, 2LL * P.ntiles, 0.f, st));
    PDG_TRY(launch_fill((float *)s.rr_part, 2LL * P.ntiles, 0.f, st));
  }
  // solve 1: (I + lam L) y = g, y in s.x ; solve 2: (I + lam L) z = y, z in g
  for (int solve = 0; solve < 2; ++solve) {
    const float *src = solve == 0 ? g : s.x;
    CGState t = s;
    t.x = solve == 0 ? s.x : g;
    // solve 1's x feeds solve 2 through its kept cells only (its set-up visits
    // the listed tiles); solve 2's x is the output (every tile, zeros on the
    // pruned cells)
    if (P.klist && solve == 0)
      cg_init_kernel<<<padded(nlisted), kThreads, 0, st>>>(P, nlisted, P.klist, src, t.r, t.x,
                                                           t.rr_part, 0);
    else
      cg_init_kernel<<<padded(P.ntiles), kThreads, 0, st>>>(P, P.ntiles, nullptr, src, t.r, t.x,
                                                            t.rr_part, solve == 1);
    PDG_TRY(launched("cg_init"));
    cg_reduce_kernel<<<P.nsys, kThreads, 0, st>>>(P, 0, 0, 0, t);
    PDG_TRY(launched("cg_reduce"));
    for (int k = 0; k < kmax; ++k) {
      // launch only the span of levels that are still iterating
      int lo = -1, hi = -1;
      for (int l = 0; l < P.levels; ++l)
        if (P.lv[l].iters > k) {
          if (lo < 0) lo = l;
          hi = l;
        }
      int tile_lo = P.lv[lo].tile0;
      int tile_hi = P.lv[hi].tile0 + P.batch * 3 * P.lv[hi].tps;
      if (P.klist) {                       // positions in the kept-tile list
        tile_lo = P.kfirst[lo];
        tile_hi = P.kfirst[hi] + P.kcount[hi];
      }
      const int sys_lo = P.lv[lo].sys0;
      const int sys_hi = P.lv[hi].sys0 + P.batch * 3;
      float *pin = (k & 1) ? t.p1 : t.p0;
      float *pout = (k & 1) ? t.p0 : t.p1;
      if (tile_hi <= tile_lo) {            // no kept tile in the span: nothing to update
        PDG_TRY(run_reductions_only(P, k, sys_lo, sys_hi, t, st));
        continue;
      }
      if (P.mask)
        cg_a_kernel<true><<<padded(tile_hi - tile_lo), kThreads, 0, st>>>(
            P, k, tile_lo, tile_hi - tile_lo, t, pin, pout);
      else
        cg_a_kernel<false><<<padded(tile_hi - tile_lo), kThreads, 0, st>>>(
            P, k, tile_lo, tile_hi - tile_lo, t, pin, pout);
      PDG_TRY(launched("cg_a"));
      cg_reduce_kernel<<<sys_hi - sys_lo, kThreads, 0, st>>>(P, k, 1, sys_lo, t);
      PDG_TRY(launched("cg_reduce"));
      if (P.mask)
        cg_b_kernel<true><<<padded(tile_hi - tile_lo), kThreads, 0, st>>>(
            P, k, tile_lo, tile_hi - tile_lo, t, pout);
      else
        cg_b_kernel<false><<<padded(tile_hi - tile_lo), kThreads, 0, st>>>(
            P, k, tile_lo, tile_hi - tile_lo, t, pout);
      PDG_TRY(launched("cg_b"));
      cg_reduce_kernel<<<sys_hi - sys_lo, kThreads, 0, st>>>(P, k, 2, sys_lo, t);
      PDG_TRY(launched("cg_reduce"));
    }
  }
  return PDG_OK;
}

}  // namespace pdg
