// kern_all.hip -- per-tile kernels of a batch launched once over the tiles
// of every dimension class: each tile's system selects the
// dimension-templated body (update, binning, subcell sort, list build,
// forces).  One launch per kernel instead of one per class keeps the launch
// count of a batch iteration independent of how many dimensions it mixes.
#include "kernels.h"
#include "dispatch.h"

namespace hdmd {

#define HDMD_EACH_D(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)

__global__ __launch_bounds__(kTile) void k_bin_all(KArgs a) {
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int tile;
    if (!fetch_atom_tile(a, t, s, tile)) break;
    if (!running(s) || !need_rebuild(s)) continue;
    switch (s->d) {
#define HDMD_CASE(DD) \
  case DD:            \
    bin_tile<DD>(s, tile); \
    break;
      HDMD_EACH_D(HDMD_CASE)
#undef HDMD_CASE
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
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int c;
    if (!fetch_cell_tile(a, t, s, c)) break;
    if (!running(s) || !need_rebuild(s)) continue;
    const bool mix = s->precision != 0;
    switch (s->d) {
#define HDMD_CASE(DD)                                         \
  case DD:                                                    \
    if (mix) cellsort_tile<DD, float>(s, c, sk, sv);          \
    else cellsort_tile<DD, double>(s, c, sk, sv);             \
    break;
      HDMD_EACH_D(HDMD_CASE)
#undef HDMD_CASE
    }
  }
}

__global__ __launch_bounds__(kTile) void k_force_all(KArgs a, int fire) {
  __shared__ double sh[kPart];
  for (int t = xcd_tile(blockIdx.x, gridDim.x);; t += gridDim.x) {
    SysDev* s;
    int tile;
    if (!fetch_atom_tile(a, t, s, tile)) break;
    if (!running(s)) continue;
    if (fire && s->mode != MODE_FIRE) continue;
    const bool mix = s->precision != 0;
    switch (s->d) {
#define HDMD_CASE(DD)                                           \
  case DD:                                                      \
    if (mix) force_tile<DD, true, 1>(s, tile, fire, sh);        \
    else force_tile<DD, false, 1>(s, tile, fire, sh);           \
    break;
      HDMD_EACH_D(HDMD_CASE)
#undef HDMD_CASE
    }
  }
}

// Verlet-list build of every rebuilding system: a subcell of an n_cell >= 3
// system is one wave's work (four such per workgroup), a subcell of an
// n_cell <= 2 system (crowded: it holds the atoms of 1/2^d of the box) is
// split over the four waves of a workgroup.
__global__ __launch_bounds__(256) void k_build_all(KArgs a) {
  __shared__ unsigned long long msk_all[4][8 * 128];
  __shared__ int cand_all[4][8 * 64];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nnw = a.tab->n_cell_nowrap[0], ntot = a.tab->n_cell[0];
  const int unw = (nnw + 3) / 4;
  const int units = unw + (ntot - nnw);
  const int2* tiles = a.tab->cell_tiles[0];
  for (int u = xcd_tile(blockIdx.x, gridDim.x); u < units; u += gridDim.x) {
    const bool wr = u >= unw;
    const int idx = wr ? nnw + (u - unw) : 4 * u + wv;
    if (idx >= ntot || (!wr && idx >= nnw)) continue;
    const int2 e = tiles[idx];
    SysDev* s = uniform_ptr(a.tab->sys[uniform_int(e.x)]);
    const int hc = uniform_int(e.y);
    if (!running(s) || !need_rebuild(s)) continue;
    switch (s->d) {
#define HDMD_CASE(DD)                                              \
  case DD:                                                         \
    if (wr) build_t_tile<DD, 4, true>(s, hc, wv, msk_all[wv], cand_all[wv]); \
    else build_t_tile<DD, 1, false>(s, hc, 0, msk_all[wv], cand_all[wv]);    \
    break;
      HDMD_EACH_D(HDMD_CASE)
#undef HDMD_CASE
    }
  }
}

void launch_build_all(const KArgs& a, int grid, hipStream_t st) { k_build_all<<<grid, 256, 0, st>>>(a); }
void launch_bin_all(const KArgs& a, int grid, hipStream_t st) { k_bin_all<<<grid, kTile, 0, st>>>(a); }
void launch_force_all(const KArgs& a, int grid, int fire, hipStream_t st) {
  k_force_all<<<grid, kTile, 0, st>>>(a, fire);
}
void launch_fire_update_all(const KArgs& a, int grid, hipStream_t st) {
  k_fire_update_all<<<grid, kTile, 0, st>>>(a);
}
void launch_cellsort_all(const KArgs& a, int grid, hipStream_t st) {
  k_cellsort_all<<<grid, 256, 0, st>>>(a);
}

}  // namespace hdmd
