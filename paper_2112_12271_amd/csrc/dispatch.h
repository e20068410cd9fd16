// dispatch.h -- host-side launchers of the dimension-templated kernels.
#pragma once
#include <hip/hip_runtime.h>
#include "hdmd_dev.h"

namespace hdmd {

struct DKernels {
  void (*load)(bool mix, SysDev* s, int grid, hipStream_t st, const double* pos,
               const double* diam, const double* vel);
  void (*unload)(bool mix, const SysDev* s, int grid, hipStream_t st, double* pos, double* vel,
                 double* force);
  // resume check (caller arrays == workspace state) and displacement restart
  void (*same_state)(bool mix, SysDev* s, int grid, hipStream_t st, const double* pos,
                     const double* vel, const double* diam);
  void (*disp_restart)(SysDev* s, int grid, hipStream_t st);
  void (*bin)(const KArgs& a, int grid, hipStream_t st);
  void (*cellsort)(bool mix, const KArgs& a, int grid, hipStream_t st);
  // reach: stencil radius in subcells (1: subcells of side >= r_l,max, 3^d
  // stencil; 2: half-size subcells, 5^d stencil); blk: workgroup size of the
  // home-atom-lane build (64/128/256), or 1, 2, 4 waves per subcell of the
  // candidate-lane build.  Each launch serves the systems of its own reach.
  void (*build)(int reach, bool wrap, int blk, const KArgs& a, int grid, hipStream_t st);
  // the force kernels serve the systems of one precision form (mix) and one
  // potential class (morse: the Morse form; otherwise WCA and harmonic)
  void (*force)(bool mix, int lpa, bool morse, const KArgs& a, int grid, int fire, hipStream_t st);
  void (*step)(bool mix, int lpa, bool morse, const KArgs& a, int grid, hipStream_t st);
  void (*fire_update)(bool mix, const KArgs& a, int grid, hipStream_t st);
  void (*vanhove)(const SysDev* s, int grid, hipStream_t st, int nbins, double w,
                  unsigned long long* hist, double* disp);
  // SWAP Monte Carlo: dE of a round's batch, then its settlement (kernels.h)
  void (*swap_de)(const SysDev* s, hipStream_t st, const long long* ctl, const int32_t* off_in,
                  int64_t n_att, const int32_t* pairs, const int32_t* slot_of, double* de,
                  unsigned long long* conf);
  void (*swap_settle)(SysDev* s, hipStream_t st, long long* ctl, const int32_t* off_in,
                      int32_t* off_out, int64_t n_att, const int32_t* pairs, const double* u,
                      double T, const int32_t* slot_of, const double* de,
                      const unsigned long long* conf, int32_t* acc, double* diam);
};

const DKernels* dkernels(int d);

// per-tile kernels over the tiles of every dimension class of a batch
// (KArgs.cls = 0; kern_all.hip)
void launch_bin_all(const KArgs& a, int grid, hipStream_t st);
void launch_fire_update_all(const KArgs& a, int grid, hipStream_t st);
void launch_cellsort_all(const KArgs& a, int grid, hipStream_t st);
void launch_force_all(const KArgs& a, int grid, int fire, bool morse, hipStream_t st);
// list build and FIRE forces of the classes d <= kBuildAllMaxD; larger d keep
// per-class launches
constexpr int kBuildAllMaxD = 8;
void launch_build_all(const KArgs& a, int grid, int reach, hipStream_t st);

// dimension-independent kernels (common.hip)
void launch_setdesc(SysDev* dst, const SysDev& val, hipStream_t st);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
void launch_scan1(const KArgs& a, int grid, hipStream_t st);
void launch_scan2(const KArgs& a, int grid, hipStream_t st);
void launch_scatter(const KArgs& a, int grid, hipStream_t st);
void launch_finalize(const KArgs& a, int grid, hipStream_t st);
void launch_fire_ctrl(const KArgs& a, int grid, hipStream_t st);
void launch_reduce_pe(const SysDev* s, double* out, hipStream_t st);
void launch_slot_of(const SysDev* s, int n, int32_t* slot_of, hipStream_t st);
// SWAP set-up: every pair id in [0, n) (else ctl[3] = 1), counters zeroed
void launch_swap_init(int64_t n_att, const int32_t* pairs, int n, long long* ctl, hipStream_t st);
void launch_export(const SysDev* s, int n, int64_t* row_ptr, int32_t* cols, hipStream_t st,
                   int phase);
void launch_set_status(SysDev* s, int32_t status, hipStream_t st);
void launch_poll(const Table* t, int max_slots, int32_t* state, int64_t* iters, hipStream_t st);

}  // namespace hdmd
