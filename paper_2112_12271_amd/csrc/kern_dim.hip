// kern_dim.hip -- instantiates the kernels for one dimension HDMD_DIM and
// exports their launchers.  Built once per d = 2..10.
#include "kernels.h"
#include "dispatch.h"

#ifndef HDMD_DIM
#error "HDMD_DIM must be defined"
#endif

namespace hdmd {
namespace {
constexpr int D = HDMD_DIM;

void l_load(bool mix, SysDev* s, int grid, hipStream_t st, const double* pos, const double* diam,
            const double* vel) {
  if (mix) k_load<D, float><<<grid, kTile, 0, st>>>(s, pos, diam, vel);
  else k_load<D, double><<<grid, kTile, 0, st>>>(s, pos, diam, vel);
}
void l_unload(bool mix, const SysDev* s, int grid, hipStream_t st, double* pos, double* vel,
              double* force) {
  if (mix) k_unload<D, float><<<grid, kTile, 0, st>>>(s, pos, vel, force);
  else k_unload<D, double><<<grid, kTile, 0, st>>>(s, pos, vel, force);
}
void l_same_state(bool mix, SysDev* s, int grid, hipStream_t st, const double* pos, const double* vel,
                  const double* diam) {
  if (mix) k_same_state<D, float><<<grid, kTile, 0, st>>>(s, pos, vel, diam);
  else k_same_state<D, double><<<grid, kTile, 0, st>>>(s, pos, vel, diam);
}
void l_disp_restart(SysDev* s, int grid, hipStream_t st) {
  k_disp_restart<D><<<grid, kTile, 0, st>>>(s);
}
void l_bin(const KArgs& a, int grid, hipStream_t st) { k_bin<D><<<grid, kTile, 0, st>>>(a); }
void l_cellsort(bool mix, const KArgs& a, int grid, hipStream_t st) {
  if (mix) k_cellsort<D, float><<<grid, 256, 0, st>>>(a);
  else k_cellsort<D, double><<<grid, 256, 0, st>>>(a);
}
void l_build(int reach, bool wrap, int blk, const KArgs& a, int grid, hipStream_t st) {
  if ((blk & kBuildMF) && !wrap) {
    // candidate-lane build with the pair tests on the matrix cores
    blk &= ~kBuildMF;
    if (reach == 2) {
      if (blk == 1) k_build_t<D, 1, false, 2, true><<<grid, 64, 0, st>>>(a);
      else if (blk == 2) k_build_t<D, 2, false, 2, true><<<grid, 128, 0, st>>>(a);
      else k_build_t<D, 4, false, 2, true><<<grid, 256, 0, st>>>(a);
    } else {
      if (blk == 1) k_build_t<D, 1, false, 1, true><<<grid, 64, 0, st>>>(a);
      else if (blk == 2) k_build_t<D, 2, false, 1, true><<<grid, 128, 0, st>>>(a);
      else k_build_t<D, 4, false, 1, true><<<grid, 256, 0, st>>>(a);
    }
    return;
  }
  blk &= ~kBuildMF;  // wrapped systems: the vector form
  if (reach == 2) {
    // half-size subcells, 5^d stencil (never wrapped)
    if (blk == 1) k_build_t<D, 1, false, 2><<<grid, 64, 0, st>>>(a);
    else if (blk == 2) k_build_t<D, 2, false, 2><<<grid, 128, 0, st>>>(a);
    else if (blk == 4 || blk == 8 || blk == 16) k_build_t<D, 4, false, 2><<<grid, 256, 0, st>>>(a);
    else if (blk <= 64) k_build<D, false, 64><<<grid, 64, 0, st>>>(a);
    else if (blk <= 128) k_build<D, false, 128><<<grid, 128, 0, st>>>(a);
    else k_build<D, false, 256><<<grid, 256, 0, st>>>(a);
  } else if (wrap) {
    // crowded subcells (n_cell <= 2): up to 16 waves share one
    if (blk == 1) k_build_t<D, 1, true><<<grid, 64, 0, st>>>(a);
    else if (blk == 2) k_build_t<D, 2, true><<<grid, 128, 0, st>>>(a);
    else if (blk == 4) k_build_t<D, 4, true><<<grid, 256, 0, st>>>(a);
    else if (blk == 8) k_build_t<D, 8, true><<<grid, 512, 0, st>>>(a);
    else if (blk == 16) k_build_t<D, 16, true><<<grid, 1024, 0, st>>>(a);
    else if (blk <= 64) k_build<D, true, 64><<<grid, 64, 0, st>>>(a);
    else if (blk <= 128) k_build<D, true, 128><<<grid, 128, 0, st>>>(a);
    else k_build<D, true, 256><<<grid, 256, 0, st>>>(a);
  } else {
    if (blk == 1) k_build_t<D, 1, false><<<grid, 64, 0, st>>>(a);
    else if (blk == 2) k_build_t<D, 2, false><<<grid, 128, 0, st>>>(a);
    else if (blk == 4 || blk == 8 || blk == 16) k_build_t<D, 4, false><<<grid, 256, 0, st>>>(a);
    else if (blk <= 64) k_build<D, false, 64><<<grid, 64, 0, st>>>(a);
    else if (blk <= 128) k_build<D, false, 128><<<grid, 128, 0, st>>>(a);
    else k_build<D, false, 256><<<grid, 256, 0, st>>>(a);
  }
}
template <bool MIX, int LPA, bool MORSE = false>
void force_lpa(const KArgs& a, int grid, int fire, hipStream_t st) {
  k_force<D, MIX, LPA, MORSE><<<grid, kTile * LPA, 0, st>>>(a, fire);
}
template <bool MIX, int LPA, bool MORSE = false>
void step_lpa(const KArgs& a, int grid, hipStream_t st) {
  k_step<D, MIX, LPA, MORSE><<<grid, kTile * LPA, 0, st>>>(a);
}
// Morse systems run one lane per atom
void l_force(bool mix, int lpa, bool morse, const KArgs& a, int grid, int fire, hipStream_t st) {
  if (morse) {
    if (mix) force_lpa<true, 1, true>(a, grid, fire, st);
    else force_lpa<false, 1, true>(a, grid, fire, st);
  } else if (mix) {
    if (lpa >= 4) force_lpa<true, 4>(a, grid, fire, st);
    else if (lpa == 2) force_lpa<true, 2>(a, grid, fire, st);
    else force_lpa<true, 1>(a, grid, fire, st);
  } else {
    if (lpa >= 4) force_lpa<false, 4>(a, grid, fire, st);
    else if (lpa == 2) force_lpa<false, 2>(a, grid, fire, st);
    else force_lpa<false, 1>(a, grid, fire, st);
  }
}
void l_step(bool mix, int lpa, bool morse, const KArgs& a, int grid, hipStream_t st) {
  if (morse) {
    if (mix) step_lpa<true, 1, true>(a, grid, st);
    else step_lpa<false, 1, true>(a, grid, st);
  } else if (mix) {
    if (lpa >= 4) step_lpa<true, 4>(a, grid, st);
    else if (lpa == 2) step_lpa<true, 2>(a, grid, st);
    else step_lpa<true, 1>(a, grid, st);
  } else {
    if (lpa >= 4) step_lpa<false, 4>(a, grid, st);
    else if (lpa == 2) step_lpa<false, 2>(a, grid, st);
    else step_lpa<false, 1>(a, grid, st);
  }
}
void l_fire_update(bool mix, const KArgs& a, int grid, hipStream_t st) {
  if (mix) k_fire_update<D, true><<<grid, kTile, 0, st>>>(a);
  else k_fire_update<D, false><<<grid, kTile, 0, st>>>(a);
}
void l_vanhove(const SysDev* s, int grid, hipStream_t st, int nbins, double w,
               unsigned long long* hist, double* disp) {
  k_vanhove<D><<<grid, kTile, 0, st>>>(s, nbins, w, hist, disp);
}
void l_swap_de(const SysDev* s, hipStream_t st, const long long* ctl, const int32_t* off_in,
               int64_t n_att, const int32_t* pairs, const int32_t* slot_of, double* de,
               unsigned long long* conf) {
  k_swap_de<D><<<kSwapBatch, 1024, 0, st>>>(s, ctl, off_in, n_att, pairs, slot_of, de, conf);
}
void l_swap_settle(SysDev* s, hipStream_t st, long long* ctl, const int32_t* off_in,
                   int32_t* off_out, int64_t n_att, const int32_t* pairs, const double* u, double T,
                   const int32_t* slot_of, const double* de, const unsigned long long* conf,
                   int32_t* acc, double* diam) {
  k_swap_settle<D><<<1, 1024, 0, st>>>(s, ctl, off_in, off_out, n_att, pairs, u, T, slot_of, de,
                                       conf, acc, diam);
}
const DKernels table = {l_load, l_unload, l_same_state, l_disp_restart, l_bin, l_cellsort, l_build, l_force, l_step,
                        l_fire_update, l_vanhove, l_swap_de, l_swap_settle};
}  // namespace

#define HDMD_CAT2(a, b) a##b
#define HDMD_CAT(a, b) HDMD_CAT2(a, b)
const DKernels* HDMD_CAT(dkernels_d, HDMD_DIM)() { return &table; }

}  // namespace hdmd
