// kern_all.hip -- per-tile kernels of a batch launched once over the tiles
// of every dimension class: each tile's system selects the
// dimension-templated body (update, binning, subcell sort, list build,
// forces).  One launch per kernel instead of one per class keeps the launch
// count of a batch iteration independent of how many dimensions it mixes.
#include "kernels.h"
#include "dispatch.h"

namespace hdmd {

#define HDMD_EACH_D(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)
// classes of the all-class list build and forces: the d = 9, 10 bodies need
// more registers than four waves per SIMD allow, so those classes keep
// launches of their own
#define HDMD_BUILD_D(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8)

// The rebuild chain's kernels (binning, subcell sort, list build) run in
// every iteration but find work only in the systems that rebuild, often one
// of hundreds.  Their workgroups therefore test many tiles at once, one per
// lane (tile entry, system pointer, flags: three dependent loads), and then
// walk the tiles that rebuild; a workgroup's tiles are strided by the grid
// so that a rebuilding system's tiles spread over the workgroups.
__device__ inline bool tile_rebuilds(const Table* tab, const int2* tiles, int t, int n, int2& e,
                                     int dmax = kMaxD) {
  if (t >= n) return false;
  e = tiles[t];
  const SysDev* s = tab->sys[e.x];
  return running(s) && need_rebuild(s) && s->d <= dmax;
}

// The flags f of a 256-thread workgroup, as four 64-bit ballots handed to
// every wave (uniform); false when no flag is set.  xch is 32 bytes of LDS
// that no wave uses on entry or exit.
__device__ inline bool block_ballots(bool f, unsigned long long* xch, unsigned long long (&mk)[4]) {
  const unsigned long long bal = __ballot(f);
  if ((threadIdx.x & 63) == 0) xch[threadIdx.x >> 6] = bal;
  __syncthreads();
  unsigned long long any = 0;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const unsigned long long v = xch[q];
    mk[q] = ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
            (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
    any |= mk[q];
  }
  __syncthreads();
  return any != 0;
}

__global__ __launch_bounds__(kTile) void k_bin_all(KArgs a) {
  const int n = a.tab->n_atom[0], g = gridDim.x, lane = threadIdx.x;
  const int2* tiles = a.tab->atom_tiles[0];
  for (int base = blockIdx.x; base < n; base += 64 * g) {
    int2 e = make_int2(0, 0);
    unsigned long long m = __ballot(tile_rebuilds(a.tab, tiles, base + lane * g, n, e));
    while (m) {
      const int k = __builtin_ctzll(m);
      m &= m - 1;
      SysDev* s = uniform_ptr(a.tab->sys[__builtin_amdgcn_readlane(e.x, k)]);
      const int tile = __builtin_amdgcn_readlane(e.y, k);
      switch (s->d) {
#define HDMD_CASE(DD)      \
  case DD:                 \
    bin_tile<DD>(s, tile); \
    break;
        HDMD_EACH_D(HDMD_CASE)
#undef HDMD_CASE
      }
    }
  }
}

__global__ __launch_bounds__(kTile) void k_fire_update_all(KArgs a) {
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int tile;
    if (!fetch_atom_tile(a, t, s, tile)) break;
    if (!running(s) || s->mode != MODE_FIRE) continue;
    const bool mix = s->precision != 0;
    switch (s->d) {
#define HDMD_CASE(DD)                                    \
  case DD:                                               \
    if (mix) fire_update_tile<DD, true>(s, tile);        \
    else fire_update_tile<DD, false>(s, tile);           \
    break;
      HDMD_EACH_D(HDMD_CASE)
#undef HDMD_CASE
    }
  }
}

__global__ __launch_bounds__(256) void k_cellsort_all(KArgs a) {
  __shared__ int sk[kSortCap];
  __shared__ int sv[kSortCap];
  const int n = a.tab->n_cell[0], g = gridDim.x;
  const int2* tiles = a.tab->cell_tiles[0];
  for (int base = blockIdx.x; base < n; base += 256 * g) {
    int2 e;
    unsigned long long mk[4];
    if (!block_ballots(tile_rebuilds(a.tab, tiles, base + (int)threadIdx.x * g, n, e),
                       reinterpret_cast<unsigned long long*>(sk), mk))
      continue;
    for (int q = 0; q < 4; q++) {
      unsigned long long mq = mk[q];
      while (mq) {
        const int k = 64 * q + __builtin_ctzll(mq);
        mq &= mq - 1;
        const int2 ek = tiles[base + k * g];
        SysDev* s = a.tab->sys[ek.x];
        const int c = ek.y;
        const bool mix = s->precision != 0;
        switch (s->d) {
#define HDMD_CASE(DD)                                \
  case DD:                                           \
    if (mix) cellsort_tile<DD, float>(s, c, sk, sv); \
    else cellsort_tile<DD, double>(s, c, sk, sv);    \
    break;
          HDMD_EACH_D(HDMD_CASE)
#undef HDMD_CASE
        }
      }
    }
    __syncthreads();  // the LDS exchange area is free again
  }
}

// FIRE forces of every class d <= kBuildAllMaxD (larger d: per-class launches)
template <bool MORSE>
__global__ __launch_bounds__(kTile) void k_force_all(KArgs a, int fire) {
  __shared__ double sh[kPart];
  __shared__ vd2 stage[kStage16];
  for (int t = xcd_tile(blockIdx.x, gridDim.x);; t += gridDim.x) {
    SysDev* s;
    int tile;
    if (!fetch_atom_tile(a, t, s, tile)) break;
    if (!running(s) || (s->potential == kPotMorse) != MORSE || s->lpa != 1) continue;
    if (fire && s->mode != MODE_FIRE) continue;
    const bool mix = s->precision != 0;
    switch (s->d) {
#define HDMD_CASE(DD)                                           \
  case DD:                                                      \
    if (mix) force_tile<DD, true, 1, MORSE>(s, tile, fire, sh, stage); \
    else force_tile<DD, false, 1, MORSE>(s, tile, fire, sh, stage);    \
    break;
      HDMD_BUILD_D(HDMD_CASE)
#undef HDMD_CASE
    }
  }
}

// Verlet-list build of every rebuilding system with d <= kBuildAllMaxD (the
// d = 9, 10 bodies need more registers than four waves per SIMD allow, so
// those classes keep launches of their own): a subcell of an n_cell >= 3
// system is one wave's work (four such per workgroup), a subcell of an
// n_cell <= 2 system (crowded: it holds the atoms of 1/2^d of the box) is
// split over the four waves of a workgroup.  One launch per stencil radius
// present (RAD 1: subcells of side >= r_l,max; RAD 2: half-size subcells),
// each passing over the subcells of the other radius.
template <int RAD>
__global__ __launch_bounds__(256) void k_build_all(KArgs a) {
  __shared__ unsigned long long msk_all[4][8 * 128];
  __shared__ int cand_all[4][8 * 64];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nnw = a.tab->n_cell_nowrap[0], ntot = a.tab->n_cell[0];
  const int unw = (nnw + 3) / 4;
  const int units = unw + (ntot - nnw);
  const int2* tiles = a.tab->cell_tiles[0];
  const int g = gridDim.x;
  for (int base = xcd_tile(blockIdx.x, g); base < units; base += 256 * g) {
    unsigned long long mk[4];
    {
      // unit u: subcells 4u..4u+3 of the n_cell >= 3 part, or one wrapped subcell
      const int u = base + (int)threadIdx.x * g;
      bool act = false;
      int2 e;
      if (u < unw) {
        for (int q = 0; q < 4; q++) act |= tile_rebuilds(a.tab, tiles, 4 * u + q, nnw, e, kBuildAllMaxD);
      } else if (u < units) {
        act = tile_rebuilds(a.tab, tiles, nnw + (u - unw), ntot, e, kBuildAllMaxD);
      }
      if (!block_ballots(act, reinterpret_cast<unsigned long long*>(cand_all[0]), mk)) continue;
    }
    for (int q = 0; q < 4; q++) {
      unsigned long long mq = mk[q];
      while (mq) {
        const int u = base + (64 * q + __builtin_ctzll(mq)) * g;
        mq &= mq - 1;
        const bool wr = u >= unw;
        const int idx = wr ? nnw + (u - unw) : 4 * u + wv;
        if (idx >= ntot || (!wr && idx >= nnw)) continue;
        const int2 e = tiles[idx];
        SysDev* s = uniform_ptr(a.tab->sys[uniform_int(e.x)]);
        const int hc = uniform_int(e.y);
        if (!running(s) || !need_rebuild(s) || uniform_int(s->reach) != RAD) continue;
        switch (s->d) {
#define HDMD_CASE(DD)                                                             \
  case DD:                                                                        \
    if (RAD == 2) build_t_tile<DD, 1, false, 2>(s, hc, 0, msk_all[wv], cand_all[wv]); \
    else if (wr) build_t_tile<DD, 4, true>(s, hc, wv, msk_all[wv], cand_all[wv]); \
    else build_t_tile<DD, 1, false>(s, hc, 0, msk_all[wv], cand_all[wv]);         \
    break;
          HDMD_BUILD_D(HDMD_CASE)
#undef HDMD_CASE
        }
      }
    }
    __syncthreads();  // the LDS exchange area is free again
  }
}

void launch_build_all(const KArgs& a, int grid, int reach, hipStream_t st) {
  if (reach == 2) k_build_all<2><<<grid, 256, 0, st>>>(a);
  else k_build_all<1><<<grid, 256, 0, st>>>(a);
}
void launch_bin_all(const KArgs& a, int grid, hipStream_t st) { k_bin_all<<<grid, kTile, 0, st>>>(a); }
void launch_force_all(const KArgs& a, int grid, int fire, bool morse, hipStream_t st) {
  if (morse) k_force_all<true><<<grid, kTile, 0, st>>>(a, fire);
  else k_force_all<false><<<grid, kTile, 0, st>>>(a, fire);
}
void launch_fire_update_all(const KArgs& a, int grid, hipStream_t st) {
  k_fire_update_all<<<grid, kTile, 0, st>>>(a);
}
void launch_cellsort_all(const KArgs& a, int grid, hipStream_t st) {
  k_cellsort_all<<<grid, 256, 0, st>>>(a);
}

}  // namespace hdmd
