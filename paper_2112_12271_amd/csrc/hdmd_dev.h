// hdmd_dev.h -- device-side data structures and helpers of the HIP hot path.
//
// Internal layout of one system (all in the caller's workspace):
//   x[2]      atom records [npad][DR] FP64: the d coordinates, the diameter,
//             zero padding; DR = 4, 8 or 16 doubles so that a record is whole
//             16-byte loads and never straddles more cache lines than needed
//             (one 64-byte half line for 4 <= d <= 7).  Double-buffered: a
//             step reads x[cur] and writes x[cur^1].
//   q[2]      (mixed precision only) the same records as 32-bit fixed-point
//             coordinates u = (x + L/2) 2^32 / L and the FP64 diameter,
//             [npad][DQ] int32; u_j - u_i in two's complement is the exact
//             minimum-image displacement, so gathers carry half the bytes.
//   v[2]      velocities, axis-major (SoA) [d][npad], FP64 or FP32.
//   oid[2]    caller id of each slot; the [2] buffers of v and oid are the
//             source and destination of the permutation at a rebuild.
//   f         forces [d][npad] (FP64 or FP32), written by the force kernels.
//   xref      positions at the last build [d][npad] FP64 (rebuild trigger).
//   qc        offsets from the subcell centre quantised to int8 in units of
//             L_sc/250, packed four per int32 (prefilter of the list build
//             when n_cell >= 3); qc16 the same as int16 pairs with |q|^2 in
//             the last word read, or, when n_cell <= 2, 16-bit coordinates
//             wrapping at L; ycell the offsets in FP32 (home-lane build when
//             n_cell <= 2).
//   nl, nlen  Verlet rows in ELL form, column-major nl[k*npad + i], i.e. entry
//             k of every row is contiguous so a wave reads it coalesced.
// Atoms are stored in subcell order (canonical: by subcell, then caller id),
// rebuilt at every list build.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace hdmd {

constexpr int kMaxD = 10;
constexpr int kMinD = 2;
constexpr int kTile = 64;       // atoms per atom tile (one wave at one lane per atom)
constexpr int kWave = 64;
constexpr int kChunk = 1024;    // subcells per scan chunk
constexpr int kSortCap = 4096;  // subcell occupancy sorted in LDS (larger: in global memory)
constexpr int kPart = 11;       // doubles per wave in the partial-sum array
// step, KE, PE, KE+PE, virial W, coordination Z, <|Delta|^2>, <|Delta|^4>,
// non-Gaussian alpha_2, overlap f_ov
constexpr int kThermoCols = 10;
constexpr int kMaxSlots = 1024;
constexpr int kQCap = 16;       // per-lane prefilter queue of the build
constexpr int kSwapBatch = 256;   // SWAP attempts per batch (a multiple of 64)
constexpr int kPotMorse = 2;     // hdmd_system.potential of the Morse form
constexpr int kQScale = 250;    // int8 quantisation: subcell side = 250 units
constexpr int kBuildMF = 1024;  // build-variant flag: candidate-lane build, pair tests on the matrix cores

enum Mode : int32_t { MODE_NONE = 0, MODE_FIRE = 1, MODE_MD = 2, MODE_STATIC = 3 };
enum Slot : int32_t { SLOT_EMPTY = 0, SLOT_RUNNING = 1, SLOT_DONE = 2 };
enum Err : int32_t {
  ERR_ARG = 1,        // position far outside the box, bad diameter
  ERR_NONFINITE = 2,  // NaN/Inf in inputs
  ERR_OVERFLOW = 4,   // a Verlet row longer than the ELL width
  ERR_RUN_NAN = 8,    // non-finite energy during a run
};
// partial-sum record of one wave
// P_VIR: sum over the atom's row of fc r^2 / 2 (the pair virial r_ij . F_ij shared
// between the two rows of a pair); P_NC: neighbours inside the interaction cutoff
// P_M2, P_M4: |Delta|^2 and |Delta|^4 of the unwrapped displacement since the
// run's start; P_OV: atoms with |Delta| < 0.1 d (thermo steps only)
enum Part : int {
  P_PE = 0, P_KE = 1, P_FV = 2, P_FF = 3, P_VV = 4, P_FMAX2 = 5, P_VIR = 6, P_NC = 7,
  P_M2 = 8, P_M4 = 9, P_OV = 10
};

struct FireCtl {
  double dt0, dtmax, dtmin, finc, fdec, alpha0, falpha, ftol, etol;
  int64_t ndelay, nnegmax, maxiter, initdelay;
};

struct SysDev {
  // ---- static, written by the host
  int32_t d, potential, precision, n;
  int32_t npad, ncell, radix, ncells;
  int32_t nstencil, width, nchunks, ntiles;
  int32_t mode, wrap, nwaves;
  int32_t reach;  // stencil radius in subcells: 1 (side >= r_l,max), 2 (half-size subcells)
  int32_t lpa;    // lanes per atom of the force kernels (1, 2 or 4)
  int32_t pad0;
  double L, hL, cutoff, skin, eps, sigma_max;
  double rlmax, lsc, inv_lsc, halfskin2;
  double fxscale, qinv;  // 2^32 / L; 250 / L_sc
  double fxinv;          // L / 2^32
  double qmarg;          // sqrt(d)/2 with slack: half the quantisation error bound
  double morse_a;        // Morse stiffness (potential 2)
  double tau_t, temp_t;  // Berendsen time constant (0: NVE) and target temperature
  float rl2f, lscf, Lf, pad3;
  int32_t tq, tcull;     // int8 prefilter threshold; row-culling threshold
                         // (squared quantised units)
  int32_t ysort, pad5;   // 1: subcells ordered by last-axis offset, then caller id
  double* x[2];
  int32_t* q[2];
  void* v[2];
  int32_t* oid[2];
  void* f;
  double* xref;
  double* disp[2];  // unwrapped displacement since the run's start up to the
                    // last build, [d][npad] (MD; permuted with the atoms)
  float* ycell;
  int32_t* qc;
  int32_t* qc16;  // int16 offsets or wrapped 16-bit coordinates, [npad][8];
                  // n_cell >= 3: words 0.. the offsets as int16 pairs, word
                  // 3 (d <= 6) or 7 the home term |q|^2 - T, word 5 the
                  // row-cull threshold, word 6 the threshold share T
  int32_t* cell_of;
  int32_t* rank;
  int32_t* cell_count;
  int32_t* cell_flat;  // start of every subcell, [ncells + 1], written at each rebuild
  int32_t* cell_local;
  int32_t* chunk_sum;
  int32_t* chunk_off;
  int32_t* key;
  int32_t* src;
  int32_t* nl;
  int32_t* nlen;
  double* part;
  double* thermo;
  double dt;
  int64_t nsteps, thermo_every;
  FireCtl fc;
  // ---- dynamic, written by the kernels
  int32_t xcur, pcur, force_rebuild, err;
  unsigned long long maxdisp2;  // bit pattern of a non-negative double
  int32_t max_row, max_cell, status, fstatus;
  int64_t step, builds, iters;
  double ke, pe;
  double fdt, falpha, fmax, c_dt, c_keep, c_mix;
  double vscale;  // Berendsen factor of the next full-step kick (1: none)
  int32_t npos, nneg, c_zero;
  int32_t differ;  // set by k_same_state when the caller's arrays differ from the state
};

// Tile tables of a batch: one list per dimension class (index d).
struct Table {
  int32_t max_slots, pad;
  // index d: dimension class d; index 0: all classes (atom tiles of class d
  // follow those of class d-1 in one array, so class 0 covers them all; the
  // cell tiles of class 0 are an array of their own that lists the n_cell >= 3
  // subcells of every class before the wrap ones)
  int32_t n_atom[kMaxD + 1];
  int32_t n_cell[kMaxD + 1];
  int32_t n_cell_nowrap[kMaxD + 1];  // cell tiles of systems with n_cell >= 3 come first
  int32_t n_chunk;
  int32_t n_sys;
  int2* atom_tiles[kMaxD + 1];  // (slot, tile)
  int2* cell_tiles[kMaxD + 1];  // (slot, cell)
  int2* chunk_tiles;            // (slot, chunk)
  int32_t* sys_list;            // slots of the current composition
  SysDev* sys[kMaxSlots];
};

// Kernel arguments: either one system (tile = blockIdx) or a batch table.
// part selects a sub-range of the cell tiles: 0 all, 1 systems with
// n_cell >= 3, 2 systems with n_cell <= 2 (the two list-build variants).
struct KArgs {
  SysDev* single;
  Table* tab;
  int32_t cls;
  int32_t part;
};

// Workgroups of a launch are handed to the eight XCDs in turn (workgroup b to
// XCD b mod 8), each XCD with its own L2.  For a grid that is a multiple of
// eight, this maps workgroup b to tile (b mod 8)·(grid/8) + b/8, so that each
// XCD takes one contiguous run of tiles (neighbouring subcells, whose linked
// subcells overlap) instead of every eighth tile.  A bijection on [0, grid).
__device__ inline int xcd_tile(int b, int g) {
#ifdef HDMD_NO_XCD
  return b;
#else
  return (g & 7) ? b : (b & 7) * (g >> 3) + (b >> 3);
#endif
}

__device__ inline bool fetch_atom_tile(const KArgs& a, int t, SysDev*& s, int& tile) {
  if (a.single) {
    s = a.single;
    tile = t;
    return t < s->ntiles;
  }
  if (t >= a.tab->n_atom[a.cls]) return false;
  int2 e = a.tab->atom_tiles[a.cls][t];
  s = a.tab->sys[e.x];
  tile = e.y;
  return true;
}

__device__ inline bool fetch_cell_tile(const KArgs& a, int t, SysDev*& s, int& cell) {
  if (a.single) {
    s = a.single;
    cell = t;
    return t < s->ncells;
  }
  int lo = 0, hi = a.tab->n_cell[a.cls];
  if (a.part == 1) hi = a.tab->n_cell_nowrap[a.cls];
  else if (a.part == 2) lo = a.tab->n_cell_nowrap[a.cls];
  if (t >= hi - lo) return false;
  int2 e = a.tab->cell_tiles[a.cls][lo + t];
  s = a.tab->sys[e.x];
  cell = e.y;
  return true;
}

__device__ inline bool fetch_chunk_tile(const KArgs& a, int t, SysDev*& s, int& chunk) {
  if (a.single) {
    s = a.single;
    chunk = t;
    return t < s->nchunks;
  }
  if (t >= a.tab->n_chunk) return false;
  int2 e = a.tab->chunk_tiles[t];
  s = a.tab->sys[e.x];
  chunk = e.y;
  return true;
}

__device__ inline bool fetch_sys(const KArgs& a, int t, SysDev*& s) {
  if (a.single) {
    s = a.single;
    return t == 0;
  }
  if (t >= a.tab->n_sys) return false;
  s = a.tab->sys[a.tab->sys_list[t]];
  return true;
}

__device__ inline bool running(const SysDev* s) { return s->status == SLOT_RUNNING; }

__device__ inline bool need_rebuild(const SysDev* s) {
  return s->force_rebuild != 0 || __longlong_as_double((long long)s->maxdisp2) > s->halfskin2;
}

// Subcell start (exclusive prefix of occupancies), split in chunk-local part
// and chunk offset; start(ncells) = n.
__device__ inline int cell_start(const SysDev* s, int c) {
  if (c >= s->ncells) return s->n;
  return s->cell_local[c] + s->chunk_off[c / kChunk];
}

// One periodic shift into [-L/2, L/2), then a guard for x + L rounding onto
// +L/2 (same rule as the per-step wrap of positions).
__device__ inline double wrap1(double x, double L, double h) {
  if (x >= h) x = x - L;
  else if (x < -h) x = x + L;
  if (x >= h) x = -h;
  return x;
}

// Nearest image for the pair forces: dx - L k with k = rint(dx / L), one
// rounding (for k = +-1 the same value as dx -+ L).  It can pick the other
// image only for |dx| within rounding of L/2, far beyond any cutoff, so the
// force sums are those of the definition; the list test keeps min_image.
__device__ inline double near_image(double dx, double L, double invL) {
  return __builtin_fma(-L, rint(dx * invL), dx);
}

// dx - L when dx > L/2, dx + L (= dx - (-L)) when dx < -L/2, else dx - 0 = dx:
// one subtraction after selecting the shift (no branches, same values).
__device__ inline double min_image(double dx, double L, double h) {
  const double sh = dx > h ? L : (dx < -h ? -L : 0.0);
  return dx - sh;
}

__host__ __device__ constexpr int rec_stride(int d) { return d <= 3 ? 4 : (d <= 7 ? 8 : 16); }

template <int D>
struct Dims {
  static constexpr int DR = rec_stride(D);                    // FP64 record stride (doubles)
  static constexpr int NR = (D + 2) / 2;                      // double2 loads per record
  static constexpr int SQ = (D + 1) & ~1;                     // FP64 sigma slot (in ints)
  static constexpr int DQ = D <= 2 ? 4 : (D <= 6 ? 8 : 16);  // fixed-point record stride (ints)
  static constexpr int NQ = (SQ + 2 + 3) / 4;                 // int4 loads per record
  static constexpr int DY = (D + 3) & ~3;                     // FP32 offset stride
  static constexpr int QW = (D + 3) / 4;                      // int8x4 words of the offsets
};

// int8 offset from the subcell centre in units of L_sc / 250; |y| <= L_sc/2
// up to binning rounding, so |q| <= 125 and the clamp never bites.
__device__ inline int quant8(double y, double qinv) {
  int q = (int)rint(y * qinv);
  return q < -127 ? -127 : (q > 127 ? 127 : q);
}

// Centre of subcell c along the last axis (the fastest-varying digit).
__device__ inline double last_centre(const SysDev* s, int c) {
  return ((double)(c % s->ncell) + 0.5) * s->lsc - s->hL;
}

// An atom's share T of the candidate-lane prefilter threshold (squared
// quantised units): a = (c sigma + s)/2, alpha = a/Delta + sqrt(d)/2 (with
// slack), T = floor(2 alpha^2) + 1; non-decreasing in sigma.
__device__ inline int thresh_share(const SysDev* s, double sg) {
  const double ai = 0.5 * (s->cutoff * sg + s->skin);
  const double al = ai * s->qinv + s->qmarg;
  return (int)floor(2.0 * al * al) + 1;
}

// Device arrays are global memory: accessing them through the global
// address space gives global_load/store instead of flat ones.
#define HDMD_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ inline const HDMD_GLOBAL T* gbl(const T* p) {
  return (const HDMD_GLOBAL T*)p;
}
template <typename T>
__device__ inline HDMD_GLOBAL T* gbl(T* p) {
  return (HDMD_GLOBAL T*)p;
}
// plain vector types for loads and stores through those pointers
typedef double vd2 __attribute__((ext_vector_type(2)));
typedef int vi4 __attribute__((ext_vector_type(4)));

// record = (x_0 .. x_{D-1}, sigma, 0 ...)
template <int D>
__device__ inline void load_rec(const double* __restrict__ xb, int i, double (&x)[D], double& sg) {
  const HDMD_GLOBAL vd2* p = gbl(reinterpret_cast<const vd2*>(xb + (size_t)i * Dims<D>::DR));
#pragma unroll
  for (int k = 0; k < Dims<D>::NR; k++) {
    if (2 * k == D) {
      // (sigma, padding): sigma alone
      sg = *reinterpret_cast<const HDMD_GLOBAL double*>(p + k);
      continue;
    }
    const vd2 t = p[k];
    if (2 * k < D) x[2 * k] = t.x;
    else sg = t.x;
    if (2 * k + 1 < D) x[2 * k + 1] = t.y;
    else if (2 * k + 1 == D) sg = t.y;
  }
}

template <int D>
__device__ inline void load_x(const double* __restrict__ xb, int i, double (&x)[D]) {
  double sg;
  load_rec<D>(xb, i, x, sg);
}

template <int D>
__device__ inline void store_rec(double* __restrict__ xb, int i, const double (&x)[D], double sg) {
  HDMD_GLOBAL vd2* p = gbl(reinterpret_cast<vd2*>(xb + (size_t)i * Dims<D>::DR));
#pragma unroll
  for (int k = 0; k < Dims<D>::NR; k++) {
    vd2 t;
    t.x = 2 * k < D ? x[2 * k] : (2 * k == D ? sg : 0.0);
    t.y = 2 * k + 1 < D ? x[2 * k + 1] : (2 * k + 1 == D ? sg : 0.0);
    p[k] = t;
  }
}

// fixed-point record = (u_0 .. u_{D-1}, [0], sigma as FP64 at int slot SQ, 0 ...)
__device__ inline int32_t to_fixed(double x, double hL, double scale) {
  return (int32_t)(uint32_t)(long long)rint((x + hL) * scale);
}

template <int D>
__device__ inline void store_q(int32_t* __restrict__ qb, int i, const double (&x)[D], double sg,
                               double hL, double scale) {
  constexpr int SQ = Dims<D>::SQ;
  int v[4 * Dims<D>::NQ];
#pragma unroll
  for (int k = 0; k < 4 * Dims<D>::NQ; k++) v[k] = 0;
#pragma unroll
  for (int k = 0; k < D; k++) v[k] = to_fixed(x[k], hL, scale);
  const long long sb = __double_as_longlong(sg);
  v[SQ] = (int)(unsigned)(sb & 0xffffffffll);
  v[SQ + 1] = (int)(unsigned)((unsigned long long)sb >> 32);
  HDMD_GLOBAL vi4* p = gbl(reinterpret_cast<vi4*>(qb + (size_t)i * Dims<D>::DQ));
#pragma unroll
  for (int k = 0; k < Dims<D>::NQ; k++) {
    vi4 t;
    t.x = v[4 * k];
    t.y = v[4 * k + 1];
    t.z = v[4 * k + 2];
    t.w = v[4 * k + 3];
    p[k] = t;
  }
}

template <int D>
__device__ inline void load_q(const int32_t* __restrict__ qb, int i, int (&u)[D], double& sg) {
  constexpr int SQ = Dims<D>::SQ;
  const HDMD_GLOBAL vi4* p = gbl(reinterpret_cast<const vi4*>(qb + (size_t)i * Dims<D>::DQ));
  int v[4 * Dims<D>::NQ];
#pragma unroll
  for (int k = 0; k < Dims<D>::NQ; k++) {
    const vi4 t = p[k];
    v[4 * k] = t.x;
    v[4 * k + 1] = t.y;
    v[4 * k + 2] = t.z;
    v[4 * k + 3] = t.w;
  }
#pragma unroll
  for (int k = 0; k < D; k++) u[k] = v[k];
  sg = __longlong_as_double((long long)(((unsigned long long)(unsigned)v[SQ + 1] << 32) |
                                        (unsigned)v[SQ]));
}

// Squared minimum-image distance accumulated axis by axis with a fused
// multiply-add; identical operation sequence to the list definition.
template <int D>
__device__ inline double dist2_exact(const double (&xi)[D], const double (&xj)[D], double L,
                                     double h) {
  double r2 = 0.0;
#pragma unroll
  for (int k = 0; k < D; k++) {
    double dx = min_image(xj[k] - xi[k], L, h);
    r2 = __builtin_fma(dx, dx, r2);
  }
  return r2;
}

// Per-pair list radius squared: (c * (si+sj)/2 + s)^2, each op rounded once.
__device__ inline double list_r2(double si, double sj, double c, double s) {
  double sij = 0.5 * (si + sj);
  double rl = c * sij + s;
  return rl * rl;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide deterministic sum of per-thread values (fixed tree order).
template <int BS>
__device__ inline double block_sum(double v, double* sh) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = BS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = sh[t] + sh[t + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}
template <int BS>
__device__ inline double block_max(double v, double* sh) {
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = BS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

}  // namespace hdmd
