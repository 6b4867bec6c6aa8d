// Pruned grids (paper Sec. 3.6, implementation details): a cell of a level is
// kept when a point of the frames its stack connects lies in it or within
// `halo` cells of such a cell (Chebyshev distance, the cube around it).  The
// kept set is a bit per cell; pruned cells hold zero.
//
// Occupancy: one thread per point and frame sets the bit of its cell at every
// level in each stack that uses the frame (integer atomics; the result does
// not depend on their order).  The cube dilation is separable: three passes,
// one per axis, each a bitwise OR over 2 halo + 1 shifted copies.  Rows of
// R % 32 == 0 levels are whole words, so those passes work on words (shifts
// along x, word ORs along y and z); other levels go cell by cell.
#include <algorithm>

#include "common.h"

namespace pdg {
namespace {

struct PruneLevels {
  int levels;
  int R[PDG_MAX_LEVELS];
  long long moff[PDG_MAX_LEVELS];   // word offset of the level in a stack
  long long mstack;                 // words per stack
};

PruneLevels prune_levels(const GridDev &g) {
  PruneLevels p;
  memset(&p, 0, sizeof p);
  p.levels = g.levels;
  long long w = 0;
  for (int l = 0; l < g.levels; ++l) {
    p.R[l] = g.res[l];
    p.moff[l] = w;
    w += mask_words(g.res[l]);
  }
  p.mstack = w;
  return p;
}

// Cell of coordinate s along an axis: floor((s + 1) R / 2) clamped to
// 0..R-1, decided in float32 ((s + 1) rounded, then the product by R/2
// rounded); a NaN coordinate falls in cell 0.
__device__ __forceinline__ int cell1(float s, int R) {
  float u = (s + 1.0f) * ((float)R * 0.5f);
  u = fminf(fmaxf(u, 0.0f), (float)(R - 1));
  return (int)floorf(u);
}

__global__ __launch_bounds__(256) void occupy_cells_kernel(PruneLevels pl, int stacks, int span,
                                                           const float *__restrict__ points,
                                                           long long n,
                                                           uint32_t *__restrict__ occ) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int f = blockIdx.y;
  const float *P = points + (long long)f * 3 * n;
  const float sx = P[i], sy = P[n + i], sz = P[2 * n + i];
  const int b0 = f - span + 1 > 0 ? f - span + 1 : 0;
  const int b1 = f < stacks - 1 ? f : stacks - 1;
  for (int l = 0; l < pl.levels; ++l) {
    const int R = pl.R[l];
    const long long id = ((long long)cell1(sz, R) * R + cell1(sy, R)) * R + cell1(sx, R);
    const uint32_t bit = 1u << (id & 31);
    for (int b = b0; b <= b1; ++b)
      atomicOr(&occ[(long long)b * pl.mstack + pl.moff[l] + (id >> 5)], bit);
  }
}

// One pass of the cube dilation along `axis` (0 = x, 1 = y, 2 = z): a cell is
// set in out when a cell at most `halo` cells away along the axis is set in
// in.  One thread per output word.
__global__ __launch_bounds__(256) void dilate_kernel(PruneLevels pl, int stacks, int axis, int halo,
                                                     const uint32_t *__restrict__ in,
                                                     uint32_t *__restrict__ out) {
  const long long gw = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gw >= (long long)stacks * pl.mstack) return;
  const long long b = gw / pl.mstack;
  const long long wl = gw - b * pl.mstack;
  int l = 0;
  while (l + 1 < pl.levels && wl >= pl.moff[l + 1]) ++l;
  const int R = pl.R[l];
  const long long w = wl - pl.moff[l];                  // word within the level
  const uint32_t *L = in + b * pl.mstack + pl.moff[l];  // the level's words
  const long long n = (long long)R * R * R;
  uint32_t v = 0;
  if (R % 32 == 0) {
    const long long wpr = R / 32;                       // words per x-row
    if (axis == 0) {
      const long long m = w % wpr;
      const uint32_t cur = L[w];
      const uint32_t prev = m > 0 ? L[w - 1] : 0u;
      const uint32_t next = m < wpr - 1 ? L[w + 1] : 0u;
      v = cur;
      for (int d = 1; d <= halo; ++d)
        v |= (cur << d) | (prev >> (32 - d)) | (cur >> d) | (next << (32 - d));
    } else {
      const long long row = w / wpr;                    // z R + y
      const int c = axis == 1 ? (int)(row % R) : (int)(row / R);
      const long long step = axis == 1 ? wpr : wpr * R;
      for (int d = -halo; d <= halo; ++d)
        if (c + d >= 0 && c + d < R) v |= L[w + d * step];
    }
  } else {
    const long long stride = axis == 0 ? 1 : (axis == 1 ? R : (long long)R * R);
    for (int j = 0; j < 32; ++j) {
      const long long c = 32 * w + j;
      if (c >= n) break;
      const long long x = c % R, y = (c / R) % R, z = c / ((long long)R * R);
      const long long k = axis == 0 ? x : (axis == 1 ? y : z);
      const long long lo = k - halo > 0 ? -halo : -k;
      const long long hi = k + halo < R - 1 ? halo : R - 1 - k;
      bool on = false;
      for (long long d = lo; d <= hi && !on; ++d) {
        const long long e = c + d * stride;
        on = (L[e >> 5] >> (e & 31)) & 1u;
      }
      if (on) v |= 1u << j;
    }
  }
  out[gw] = v;
}

// active[b * levels + l] = kept cells of level l of stack b (one workgroup each)
__global__ __launch_bounds__(256) void mask_count_kernel(PruneLevels pl,
                                                         const uint32_t *__restrict__ mask,
                                                         long long *__restrict__ active) {
  __shared__ long long part[256];
  const int b = blockIdx.x / pl.levels, l = blockIdx.x % pl.levels;
  const uint32_t *W = mask + (long long)b * pl.mstack + pl.moff[l];
  const long long nw = mask_words(pl.R[l]);
  long long c = 0;
  for (long long w = threadIdx.x; w < nw; w += blockDim.x) c += __popc(W[w]);
  part[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) active[blockIdx.x] = part[0];
}

// data <- 0 on pruned cells (every channel).  One thread per value.
__global__ __launch_bounds__(256) void mask_apply_kernel(GridDev g, PruneLevels pl, int batch,
                                                         const uint32_t *__restrict__ mask,
                                                         float *__restrict__ data) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)batch * g.size) return;
  const long long b = i / g.size;
  const long long k = i - b * g.size;
  int l = 0;
  while (l + 1 < g.levels && k >= g.off[l + 1]) ++l;
  const long long r3 = (long long)g.res[l] * g.res[l] * g.res[l];
  const long long c = (k - g.off[l]) % r3;
  const uint32_t w = mask[b * pl.mstack + pl.moff[l] + (c >> 5)];
  if (!((w >> (c & 31)) & 1u)) data[i] = 0.0f;
}

}  // namespace

long long mask_stack_words(const GridDev &g) { return prune_levels(g).mstack; }

size_t prune_bytes(const GridDev &g, int stacks) {
  return 2 * a256((size_t)stacks * (size_t)mask_stack_words(g) * sizeof(uint32_t));
}

pdg_status launch_prune_mask(const GridDev &g, int stacks, int span, const float *points,
                             long long n, int halo, uint32_t *mask, long long *active, void *ws,
                             hipStream_t st) {
  const PruneLevels pl = prune_levels(g);
  const long long words = (long long)stacks * pl.mstack;
  uint32_t *t0 = (uint32_t *)ws;
  uint32_t *t1 = (uint32_t *)((char *)ws + a256((size_t)words * sizeof(uint32_t)));
  PDG_TRY(launch_fill((float *)mask, words, 0.f, st));
  const int frames = stacks + span - 1;
  if (n > 0) {
    occupy_cells_kernel<<<dim3(div_up(n, 256), frames), 256, 0, st>>>(pl, stacks, span, points, n,
                                                                      mask);
    PDG_TRY(launched("occupy_cells"));
  }
  const unsigned blocks = div_up(words, 256);
  dilate_kernel<<<blocks, 256, 0, st>>>(pl, stacks, 0, halo, mask, t0);
  PDG_TRY(launched("dilate_x"));
  dilate_kernel<<<blocks, 256, 0, st>>>(pl, stacks, 1, halo, t0, t1);
  PDG_TRY(launched("dilate_y"));
  dilate_kernel<<<blocks, 256, 0, st>>>(pl, stacks, 2, halo, t1, mask);
  PDG_TRY(launched("dilate_z"));
  if (active) {
    mask_count_kernel<<<stacks * pl.levels, 256, 0, st>>>(pl, mask, active);
    PDG_TRY(launched("mask_count"));
  }
  return PDG_OK;
}

pdg_status launch_mask_apply(const GridDev &g, int batch, const uint32_t *mask, float *data,
                             hipStream_t st) {
  if (batch <= 0) return PDG_OK;
  mask_apply_kernel<<<div_up((long long)batch * g.size, 256), 256, 0, st>>>(g, prune_levels(g),
                                                                           batch, mask, data);
  return launched("mask_apply");
}

int cg_kept_tiles(CGPlanDev &p, const GridDev &g, const uint32_t *hmask, int *list) {
  const PruneLevels pl = prune_levels(g);
  const long long tw = 2048 / 32;              // mask words per 2048-cell CG tile
  int n = 0;
  for (int l = 0; l < p.levels; ++l) {
    const CGLevel &L = p.lv[l];
    const long long nw = mask_words(L.R);
    p.kfirst[l] = n;
    for (int b = 0; b < p.batch; ++b) {
      const uint32_t *W = hmask + (long long)b * pl.mstack + pl.moff[l];
      for (int lt = 0; lt < L.tps; ++lt) {
        bool kept = false;
        for (long long w = lt * tw; w < (lt + 1) * tw && w < nw && !kept; ++w) kept = W[w] != 0u;
        if (!kept) continue;
        for (int c = 0; c < 3; ++c) list[n++] = L.tile0 + (b * 3 + c) * L.tps + lt;
      }
    }
    p.kcount[l] = n - p.kfirst[l];
  }
  // ascending: systems are (stack, channel) within a level
  std::sort(list + 0, list + n);
  return n;
}

void adam_set_mask(AdamLevels &lv, const GridDev &g, const uint32_t *mask) {
  const PruneLevels pl = prune_levels(g);
  lv.mask = mask;
  lv.mstack = pl.mstack;
  for (int l = 0; l < g.levels; ++l) {
    lv.moff[l] = pl.moff[l];
    lv.r3[l] = (long long)g.res[l] * g.res[l] * g.res[l];
  }
}

void cg_set_mask(CGPlanDev &p, const GridDev &g, const uint32_t *mask) {
  const PruneLevels pl = prune_levels(g);
  p.mask = mask;
  p.mstack = pl.mstack;
  for (int l = 0; l < g.levels; ++l) p.lv[l].moff = pl.moff[l];
}

}  // namespace pdg
