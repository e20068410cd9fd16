// kern_all.hip -- per-tile kernels of a batch launched once over the tiles
// of every dimension class: each tile's system selects the
// dimension-templated body (update, binning, subcell sort, forces).  One launch per
// kernel instead of one per class keeps the launch count of a batch
// iteration independent of how many dimensions it mixes.
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
  for (int t = blockIdx.x;; t += gridDim.x) {
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
