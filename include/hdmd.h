/*
 * hdmd.h -- C ABI of the MI355X (gfx950) hot path of d-dimensional molecular
 * dynamics after Hoy & Interiano-Alberto, "Efficient d-dimensional molecular
 * dynamics simulations for studies of the glass-jamming transition"
 * (arXiv:2112.12271).
 *
 * The library (libhdmd.so) runs every step on the GPU in hand-written HIP
 * kernels.  It never allocates device memory: the caller owns positions,
 * velocities, diameters, outputs and one opaque workspace per system (and one
 * table workspace per batch), all device pointers.  Work is enqueued on the
 * caller's stream (a hipStream_t passed as void*; NULL = the null stream).
 *
 * Layouts (caller side): positions, velocities and forces are row-major
 * [n][d] FP64 (atom i, axis k at p[i*d + k]); diameters are [n] FP64.  The
 * box is the periodic hypercube [-L/2, L/2)^d centred at the origin (Sec.
 * II.A); positions are wrapped into it on entry.  Masses are 1 and the pair
 * energy scale epsilon is one global value.
 *
 * Errors: every entry point returns an int status (hdmd_status).  Calls that
 * report host-side results (required widths, statistics, FIRE results)
 * synchronise the stream.  No C++ exception crosses this boundary; the text
 * of the last failure on the calling thread is returned by hdmd_last_error().
 * A workspace may be used by one stream at a time.
 */
#ifndef HDMD_H
#define HDMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HDMD_OK = 0,
  HDMD_NOT_CONVERGED = 1,      /* FIRE stopped at maxiter or after too many P<=0 steps */
  HDMD_ERR_ARG = -1,           /* bad d (2..10), n < 2, L <= 0, skin < 0, null pointer, diameter
                                  outside (0, sigma_max], position outside [-3L/2, 3L/2) */
  HDMD_ERR_BOX = -2,           /* L < 2 c sigma_max: the minimum-image rule would be ambiguous */
  HDMD_ERR_WORKSPACE = -3,     /* workspace smaller than hdmd_workspace_bytes() */
  HDMD_ERR_NLIST_OVERFLOW = -4,/* a Verlet row exceeded max_neighbors; *required_width is set */
  HDMD_ERR_NONFINITE = -5,     /* NaN/Inf in inputs or in the energy during a run */
  HDMD_ERR_HIP = -6,           /* a HIP runtime call failed */
  HDMD_ERR_STATE = -7          /* workspace not initialised for this system, or batch misuse */
} hdmd_status;

typedef enum { HDMD_WCA = 0, HDMD_HARMONIC = 1, HDMD_MORSE = 2 } hdmd_potential;
typedef enum { HDMD_FP64 = 0, HDMD_MIXED = 1 } hdmd_precision;
typedef enum { HDMD_SUBCELLS_AUTO = 0, HDMD_SUBCELLS_FULL = 1, HDMD_SUBCELLS_HALF = 2 } hdmd_subcells;

/* One system (Sec. II.A-C).  Pair (i,j) interacts for r < r_c = cutoff*sigma_ij
 * with sigma_ij = (sigma_i + sigma_j)/2 (Lorentz-Berthelot, Sec. II.A) and is
 * in the Verlet list for r < cutoff*sigma_ij + skin (Sec. II.C).
 *   potential  HDMD_WCA: U = 4 eps [(sigma/r)^12 - (sigma/r)^6] + eps (the
 *              paper's Mie n=6 form, Sec. II.A, with cutoff 2^(1/6));
 *              HDMD_HARMONIC: U = eps/2 (1 - r/sigma)^2 (cutoff 1);
 *              HDMD_MORSE: U = eps [e^{-2a(r-sigma)} - 2 e^{-a(r-sigma)} + 1],
 *              the paper's truncated and shifted Morse form (Sec. II.A,
 *              eq. morsepot), with cutoff 1 and a = morse_a (the paper: 30).
 *   precision  HDMD_FP64: everything in FP64.  HDMD_MIXED: neighbour
 *              positions are gathered as 32-bit fixed-point coordinates whose
 *              integer difference is the exact minimum-image displacement;
 *              pair distances, coefficients and the force sums are FP64, the
 *              stored forces and the velocities FP32; positions, energy sums
 *              and FIRE's reductions FP64.  Verlet lists are FP64-exact in
 *              both.  (A departure from a form with FP32 distances and
 *              forces: computed in FP32, the pair coefficient's error reached
 *              5.9e-5 and FP32 force sums 5.3e-5 of F_rms, above the 1e-5
 *              bound; the FP32 part here is what is stored and gathered.)
 *   sigma_max  largest diameter present; it sizes the subcells (eq. setnc).
 *   max_neighbors  Verlet row capacity W of the workspace.
 *   morse_a    Morse stiffness a in 1/length (read for HDMD_MORSE only; > 0). */
typedef struct {
  int32_t d;
  int32_t potential;
  int32_t precision;
  int32_t max_neighbors;
  int64_t n;
  double box_l;
  double cutoff;
  double skin;
  double epsilon;
  double sigma_max;
  double morse_a;
  /* Berendsen thermostat of the MD calls (Sec. II.B, II.E): with
   * thermostat_tau > 0 every velocity kick that completes a full step is
   * followed by the rescaling v *= lambda, lambda^2 = 1 + (dt/tau)(T_t/T - 1),
   * T = 2 KE / (d (n-1)) of the previous full step (1 when that KE is 0);
   * tau must be >= dt.  thermostat_tau = 0: NVE.  Unused by FIRE. */
  double thermostat_tau;
  double target_temp;
  /* Subcell grid of the list build (Sec. II.C).  HDMD_SUBCELLS_FULL:
   * n_cell = floor(L / r_l,max) per axis (eq. setnc) and the 3^d stencil.
   * HDMD_SUBCELLS_HALF: the half-size subcells the paper describes as the
   * common alternative, side >= r_l,max/2 (floor(2L / r_l,max) per axis,
   * at least 5) and the 5^d stencil; HDMD_ERR_ARG when L < 5 r_l,max/2.
   * HDMD_SUBCELLS_AUTO (0): the autotuner times both grids (where the half
   * grid applies and has at most max(64, 4n) subcells) on the first list
   * build of each key (d, n_cell <= 2, log2 of the atoms per subcell) in the
   * process and keeps the faster for every later call with that key.  The
   * lists are the same on either grid; the atom order, and so the rounding
   * of the force sums, follows the grid. */
  int32_t subcells;
  int32_t pad;
} hdmd_system;

/* FIRE 2.0 controls (Sec. II.B cites FIRE 2.0 with the semi-implicit Euler
 * integrator but prints no values; hdmd_fire_defaults() fills the published
 * defaults: N_delay 20, f_inc 1.1, f_dec 0.5, alpha_start 0.25, f_alpha 0.99,
 * dt_max = 10 dt0, dt_min = 0.02 dt0, N_neg_max 2000, initial delay on). */
typedef struct {
  double dt0, dt_max, dt_min;
  double f_inc, f_dec, alpha0, f_alpha;
  int64_t n_delay, n_neg_max, max_iter;
  int64_t initial_delay;
  double f_tol;  /* stop when max_i |F_i| < f_tol */
  double e_tol;  /* or when E/N < e_tol (0 disables; the paper's pushoff rule) */
} hdmd_fire_params;

typedef struct {
  int64_t iterations;
  int64_t builds;
  double fmax;
  double energy;
  int32_t status;  /* HDMD_OK, HDMD_NOT_CONVERGED or an error */
  int32_t pad;
} hdmd_fire_result;

typedef struct {
  int64_t steps_done;
  int64_t builds;     /* Verlet-list builds during the call */
  double ke, pe;      /* at the last full step */
  int32_t max_row;    /* longest Verlet row at the last build */
  int32_t pad;
  /* Filled only when the environment variable HDMD_PROFILE=1 is set: the call
   * then launches kernels one by one (no graph) and brackets every fused-step
   * kernel and every list-build kernel that did build with HIP events on the
   * caller's stream. */
  double step_kernel_ms;   /* summed duration of the fused-step kernels */
  int64_t step_kernels;    /* their number */
  double build_kernel_ms;  /* summed duration of the list-build kernels that built */
  int64_t build_kernels;
} hdmd_step_stats;

/* Fills *p with the FIRE 2.0 defaults for initial step dt0 and tolerance f_tol. */
void hdmd_fire_defaults(hdmd_fire_params* p, double dt0, double f_tol, int64_t max_iter);

/* Bytes of the per-system workspace (256-byte aligned device memory). */
size_t hdmd_workspace_bytes(const hdmd_system* sys);

/* Subcells per axis of sys's grid of side >= r_l,max (eq. setnc with a
 * rounding guard; the half-size grid's for HDMD_SUBCELLS_HALF), or <= 0 with
 * the status of the failed validation.  hdmd_build_config reports the grid
 * an autotuned system builds on. */
int hdmd_cells_per_axis(const hdmd_system* sys);

/* The kernel configuration calls on sys use now.  List build (Sec. II.C):
 * *reach 1 (subcells of side >= r_l,max, 3^d stencil) or 2 (half-size
 * subcells, 5^d stencil), *cells_per_axis of that grid, and *variant 1, 2 or
 * 4 (waves per subcell of the candidate-lane build; plus 1024: its pair
 * prefilter as f16 matrix-core products, exact in f32, n_cell >= 3 only; 8
 * or 16 for crowded subcells, n_cell <= 2) or 64, 128, 256 (lanes per
 * workgroup of the home-lane build); every variant builds the same lists,
 * and the environment variable HDMD_BUILD_BLK forces one.  Forces (Sec. II.B
 * getforce): *lanes_per_atom 1, 2 or 4 lanes sharing an atom's row; the
 * autotuner times them on the first list built for each (d, precision form,
 * expected row length n V_d(r_l,max) / L^d in half-octaves), and every later system with
 * that key, alone or in a batch, takes its choice (the lane count fixes the
 * rounding of the force sums); Morse systems and systems of fewer than 16384
 * atoms take one.
 * Returns 1 when the autotuner has decided the list build for sys's key, 0
 * when not yet (the defaults are reported: what the next build would time),
 * or a negative status.  Any pointer may be null. */
int hdmd_build_config(const hdmd_system* sys, int32_t* reach, int32_t* cells_per_axis,
                      int32_t* variant, int32_t* lanes_per_atom);

/* Verlet-list build, Sec. II.C (Fig. 1): loads pos/diam into ws, bins atoms
 * into n_cell^d subcells (flat index sum_k C_k n^(d-1-k)), sorts them by
 * (subcell, atom id), and lists j for i iff r_ij^2 < (c sigma_ij + s)^2 over
 * the 3^d linked subcells (deduplicated per axis when n_cell < 3).  On
 * HDMD_ERR_NLIST_OVERFLOW *required_width holds the longest row; grow
 * max_neighbors (and the workspace) and call again.  Synchronises. */
int hdmd_build_nlist(const hdmd_system* sys, const double* pos, const double* diam, void* ws,
                     size_t ws_bytes, int32_t* required_width, void* stream);

/* Exports the list held in ws as canonical CSR in caller atom ids, each row
 * ascending: row_ptr [n+1] int64 (device), cols [cols_cap] int32 (device).
 * *nnz (host) receives the entry count; cols untouched beyond cols_cap
 * (HDMD_ERR_WORKSPACE if too small).  Synchronises. */
int hdmd_nlist_export(const hdmd_system* sys, void* ws, int64_t* row_ptr, int32_t* cols,
                      int64_t cols_cap, int64_t* nnz, void* stream);

/* Forces and energy, Sec. II.B (getforce): builds the list for pos, then
 * F_i = sum_j -U'(r_ij)/r_ij (x_i - x_j) over listed pairs with r < r_c, in
 * caller order [n][d] FP64 (device); *energy (device FP64) = sum_{i<j} U_ij.
 * Synchronises (to report list overflow). */
int hdmd_forces(const hdmd_system* sys, const double* pos, const double* diam, void* ws,
                size_t ws_bytes, double* force, double* energy, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * hdmd_forces with no workspace argument.  The workspace lives in a scratch
 * array the library holds on each device it runs on until the process ends,
 * hdmd_forces_noalloc_bytes() bytes (16 MiB); a system whose
 * hdmd_workspace_bytes() exceeds it is refused with HDMD_ERR_WORKSPACE
 * before any device work.  The call allocates nothing and does not time
 * list-build variants (it takes the one an earlier call tuned for this kind
 * of system, else the default); results are those of hdmd_forces with the
 * same arguments.  Every call on one device shares that device's array and
 * leaves its contents behind (the next call rewrites what it reads): calls
 * that overlap on one device (other streams, other threads) race.  Other
 * arguments, outputs and errors as hdmd_forces.  Synchronises. */
size_t hdmd_forces_noalloc_bytes(void);
int hdmd_forces_noalloc(const hdmd_system* sys, const double* pos, const double* diam,
                        double* force, double* energy, void* stream);

#define HDMD_THERMO_COLS 10

/* Velocity Verlet, the kick-drift-kick leapfrog of Sec. II.B: per step
 * v += dt/2 F; x += dt v (wrapped); rebuild the list when the largest
 * displacement since the last build exceeds skin/2; F = F(x); v += dt/2 F
 * (times the Berendsen factor when sys->thermostat_tau > 0; NVE otherwise).
 * pos and vel ([n][d] FP64, device) are read on entry and written on exit.
 * thermo (device, may be NULL) receives floor(nsteps/thermo_every)+1 rows of
 * HDMD_THERMO_COLS FP64 at steps 0, thermo_every, ...:
 *   (step, KE, PE, KE+PE, W, Z, <|dr|^2>, <|dr|^4>, alpha_2, f_ov)
 * W is the virial, the sum over pairs inside the cutoff of r_ij . F_ij
 * (pressure P = (2 KE + W) / (d L^d)), and Z the mean number of neighbours
 * inside the cutoff per atom (getthermo, Sec. II.E).  dr is each atom's
 * unwrapped displacement since the call's step 0 (the reference state of
 * the displacement observables, Sec. II.E): its second and fourth moments,
 * the non-Gaussian parameter alpha_2 = d <|dr|^4> / ((d+2) <|dr|^2>^2) - 1
 * (eq. ngp; 0 at step 0) and the overlap f_ov, the fraction of atoms with
 * |dr| < 0.1 d (eq. fov, sigma~ = 1).  Synchronises. */
int hdmd_step(const hdmd_system* sys, double* pos, double* vel, const double* diam, void* ws,
              size_t ws_bytes, int64_t nsteps, double dt, int64_t thermo_every, double* thermo,
              hdmd_step_stats* stats, void* stream);

/* Continues the velocity-Verlet run (Sec. II.B, as hdmd_step) that the last
 * hdmd_step or hdmd_step_resume call left in ws, without reloading the state
 * or rebuilding the Verlet list: the list, the subcell order and the
 * reference positions of the rebuild trigger carry over, so a run split into
 * calls costs no extra list build per call.  pos, vel and diam must be the
 * arrays that call returned (checked bit for bit on the device; else
 * HDMD_ERR_STATE, arrays untouched), sys the same system (else
 * HDMD_ERR_STATE); thermostat_tau and target_temp may change.  The
 * displacement observables restart from zero at this call's step 0.  The
 * trajectory equals that of one longer call up to rounding of the force sums
 * (the atoms' order and the list differ from a fresh build's).  Other
 * arguments, outputs and errors as hdmd_step.  Synchronises. */
int hdmd_step_resume(const hdmd_system* sys, double* pos, double* vel, const double* diam,
                     void* ws, size_t ws_bytes, int64_t nsteps, double dt, int64_t thermo_every,
                     double* thermo, hdmd_step_stats* stats, void* stream);

/* Self part of the van Hove function (eq. VGC, Sec. II.E) after an
 * hdmd_step call that returned HDMD_OK on this workspace (no other call on it
 * since): with dr_i the unwrapped displacement of atom i from that call's
 * step 0 to its last step,
 *   hist[b] = #{i : b w <= |dr_i| < (b+1) w},  b < nbins, hist[nbins] = the
 *   atoms with |dr_i| >= nbins w, so G_s(r_b) = hist[b] / (n w);
 *   disp = dr in caller order ([n][d] FP64).
 * hist (nbins + 1 int64, device) and disp (device) are optional (not both
 * NULL); w = bin_width > 0 and nbins >= 1 when hist is given.  Errors:
 * HDMD_ERR_ARG, HDMD_ERR_WORKSPACE, HDMD_ERR_STATE (the workspace holds no
 * completed MD run of this system).  Synchronises. */
int hdmd_van_hove(const hdmd_system* sys, void* ws, size_t ws_bytes, int32_t nbins,
                  double bin_width, int64_t* hist, double* disp, void* stream);

/* SWAP Monte Carlo (Sec. II.D): n_att attempts, in order, each exchanging
 * the diameters of atoms pairs[2k] and pairs[2k+1] (caller ids, int32,
 * device).  With the diameters the earlier attempts left, dE = E_a - E_b is
 * the change of the energy of every pair that involves either atom (eq.
 * ebefore; their mutual pair keeps its diameter and cancels), and the swap is
 * kept when dE <= 0 or u[k] < exp(-dE / temperature) (Metropolis; u: n_att
 * uniforms in [0, 1), FP64, device, drawn by the caller).  Masses are 1, so
 * velocities need no rescaling.  pos ([n][d] FP64, device) is read; diam
 * ([n] FP64, device) is updated in place; accepted (n_att int32, device,
 * optional) receives 1 or 0 per attempt and *n_accepted (host) the count.
 * The outcome is that of the serial walk the paper runs on one thread; the
 * attempts are evaluated in batches and settled in order (an attempt waits
 * for the next batch when an earlier kept or waiting attempt of its batch
 * has an atom within cutoff * sigma_max of one of its atoms).  Its scratch
 * (round counters, the queues of put-off attempts, a batch's dE and
 * conflict masks: about 16 KiB, whatever n_att) is part of ws; the library
 * allocates nothing.  The pair ids are checked on the device before any
 * change.  Errors: HDMD_ERR_ARG (an id outside [0, n), temperature <= 0,
 * ...), HDMD_ERR_WORKSPACE, HDMD_ERR_HIP and the load errors of
 * hdmd_build_nlist.  Synchronises. */
int hdmd_swap(const hdmd_system* sys, const double* pos, double* diam, void* ws, size_t ws_bytes,
              int64_t n_att, const int32_t* pairs, const double* u, double temperature,
              int32_t* accepted, int64_t* n_accepted, void* stream);

/* FIRE 2.0 energy minimisation with the semi-implicit Euler update (Sec.
 * II.B), unit masses, global norms: pos ([n][d] FP64, device) in and out.
 * Synchronises. */
int hdmd_fire_minimize(const hdmd_system* sys, double* pos, const double* diam, void* ws,
                       size_t ws_bytes, const hdmd_fire_params* params, hdmd_fire_result* result,
                       void* stream);

/* ---- Batches of uneven replicas (one persistent launch per kernel and
 * d, replayed from a captured hipGraph).  A batch table holds up to
 * max_slots systems; each slot has its own system workspace.  Slots are
 * filled and emptied while other slots keep running (continuous batching). */

#define HDMD_SLOT_EMPTY 0
#define HDMD_SLOT_RUNNING 1
#define HDMD_SLOT_DONE 2

size_t hdmd_batch_bytes(int32_t max_slots, int64_t max_atoms, int64_t max_cells);
/* Initialises a batch table in table_ws (device). */
int hdmd_batch_init(void* table_ws, size_t table_bytes, int32_t max_slots, int64_t max_atoms,
                    int64_t max_cells, void* stream);
/* Loads a FIRE minimisation into slot: copies pos/diam into ws, builds the
 * list and the initial forces.  pos/diam may be freed after the call returns
 * (the stream is synchronised). */
int hdmd_batch_add_fire(void* table_ws, int32_t slot, const hdmd_system* sys, const double* pos,
                        const double* diam, void* ws, size_t ws_bytes,
                        const hdmd_fire_params* params, void* stream);
/* Loads a run of nsteps velocity-Verlet steps of size dt into slot (NVE, or
 * with the Berendsen thermostat of sys, as hdmd_step). */
int hdmd_batch_add_md(void* table_ws, int32_t slot, const hdmd_system* sys, const double* pos,
                      const double* vel, const double* diam, void* ws, size_t ws_bytes,
                      int64_t nsteps, double dt, void* stream);
/* Advances every running slot by `iterations` FIRE iterations or MD steps
 * (asynchronous: enqueued as a captured graph). */
int hdmd_batch_run(void* table_ws, int32_t iterations, void* stream);
/* Synchronises and fills state[max_slots] (HDMD_SLOT_*) and, where non-NULL,
 * iters[max_slots] (iterations or steps done). */
int hdmd_batch_poll(void* table_ws, int32_t* state, int64_t* iters, void* stream);
/* Copies a finished slot out (pos [n][d], vel may be NULL), fills *result,
 * and empties the slot.  Synchronises. */
int hdmd_batch_take(void* table_ws, int32_t slot, double* pos, double* vel,
                    hdmd_fire_result* result, void* stream);

/* Text of the last non-OK status on this thread. */
const char* hdmd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HDMD_H */
