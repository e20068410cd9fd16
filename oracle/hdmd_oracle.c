/*
 * hdmd_oracle.c -- plain, slow, single-threaded CPU oracle for the
 * d-dimensional MD hot path of Hoy & Interiano-Alberto (arXiv:2112.12271).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the HIP
 * library.  Compile with -O2 -ffp-contract=off (no -march=native, no fast-math)
 * so that every operation below is rounded exactly as written.
 *
 * Conventions (all FP64):
 *   positions x[n*d], row-major (atom i, axis k at x[i*d+k]), wrapped into
 *   the periodic hypercube [-L/2, L/2)^d centred at the origin (Sec. II.A).
 *   diameters sig[n]; masses are 1 and epsilon is one global value.
 *
 * Each function names the passage of the paper it follows.  Where the paper is
 * silent or garbled the reading taken is stated next to the code.
 *
 * Built with -fopenmp (a second library, used only to time the CPU baseline),
 * the per-atom force loop and the per-subcell list loop run on all host
 * threads: the paper's own parallelisation (per-atom getforce and per-subcell
 * list build over threads, Sec. II intro).  Rows are sorted and forces summed
 * per atom in the same order either way; only the total energy's summation
 * order changes under OpenMP.
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_WCA 0
#define ORC_HARMONIC 1
#define ORC_MORSE 2

/* ------------------------------------------------------------------------- */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------- */

/* Volume of a d-dimensional ball of diameter sigma, Sec. II.A eq. (vofsigma):
 * pi^(d/2) sigma^d / (2^d Gamma(1 + d/2)). */
double orc_sphere_volume(int d, double sigma) {
  return pow(3.14159265358979323846, 0.5 * d) * pow(sigma, d) / (pow(2.0, d) * tgamma(1.0 + 0.5 * d));
}

/* Subcells per axis, Sec. II.C eq. (setnc): floor(L / r_list_max), at least
 * one.  The paper's r_c^max is the largest interaction range plus the skin.
 * Reading: the count is lowered while a subcell would be narrower than the
 * list radius by more than rounding can explain, so that two atoms closer
 * than r_list_max along an axis never land two subcells apart. */
int orc_ncell(double L, double rlmax) {
  double q = floor(L / rlmax);
  int n = q < 1.0 ? 1 : (q > 1.0e6 ? 1000000 : (int)q);
  while (n > 1 && L / (double)n < rlmax * (1.0 + 1.0e-9)) n--;
  return n;
}

/* Wrap one coordinate into [-L/2, L/2): one periodic shift, then a guard for
 * the case where x + L rounds up onto +L/2 (periodic boundaries, Sec. II.A). */
double orc_wrap1(double x, double L) {
  double h = 0.5 * L;
  if (x >= h) x = x - L;
  else if (x < -h) x = x + L;
  if (x >= h) x = -h;
  return x;
}

/* Minimum-image displacement along one axis, dx = x_j - x_i shifted by one box
 * length when it exceeds half the box.  The paper's distance formula (Sec.
 * II.B, the pair-distance equation) is printed as a plain sum of components;
 * the reading taken is the Euclidean norm of the minimum-image vector. */
static double min_image(double dx, double L) {
  double h = 0.5 * L;
  if (dx > h) dx = dx - L;
  else if (dx < -h) dx = dx + L;
  return dx;
}

/* Squared minimum-image distance, accumulated axis by axis as a fused
 * multiply-add (the sum of squares, each term added with one rounding). */
static double dist2(int d, const double* xi, const double* xj, double L) {
  double r2 = 0.0;
  for (int k = 0; k < d; k++) {
    double dx = min_image(xj[k] - xi[k], L);
    r2 = fma(dx, dx, r2);
  }
  return r2;
}

/* Verlet-list radius for one pair: r_l = c * sigma_ij + s with the
 * Lorentz-Berthelot diameter sigma_ij = (sigma_i + sigma_j)/2 (Sec. II.A) and
 * the skin s (Sec. II.C).  Reading: the radius is per pair, not the global
 * r_c^max; the global value only sizes the subcells. */
static double list_radius2(double si, double sj, double c, double s) {
  double sij = 0.5 * (si + sj);
  double rl = c * sij + s;
  return rl * rl;
}

/* ------------------------------------------------------------------------- */
/* Neighbour lists                                                           */
/* ------------------------------------------------------------------------- */

typedef struct {
  int64_t n;
  int64_t* row_ptr; /* n+1 */
  int32_t* cols;
  int64_t nnz, cap;
} orc_list;

static orc_list* list_new(int64_t n) {
  orc_list* l = (orc_list*)calloc(1, sizeof(orc_list));
  l->n = n;
  l->row_ptr = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  l->cap = 16 * (n > 0 ? n : 1);
  l->cols = (int32_t*)malloc((size_t)l->cap * sizeof(int32_t));
  return l;
}

static void list_push(orc_list* l, int32_t j) {
  if (l->nnz == l->cap) {
    l->cap *= 2;
    l->cols = (int32_t*)realloc(l->cols, (size_t)l->cap * sizeof(int32_t));
  }
  l->cols[l->nnz++] = j;
}

void orc_list_free(orc_list* l) {
  if (!l) return;
  free(l->row_ptr);
  free(l->cols);
  free(l);
}
int64_t orc_list_nnz(const orc_list* l) { return l->nnz; }
void orc_list_copy(const orc_list* l, int64_t* row_ptr, int32_t* cols) {
  memcpy(row_ptr, l->row_ptr, (size_t)(l->n + 1) * sizeof(int64_t));
  memcpy(cols, l->cols, (size_t)l->nnz * sizeof(int32_t));
}

/* The definition of the Verlet list: j is in the list of i iff j != i and the
 * squared minimum-image distance is strictly below r_l,ij^2.  Every pair is
 * examined; rows come out in ascending j. */
orc_list* orc_nlist_brute(int d, int64_t n, double L, const double* x, const double* sig, double c,
                          double s) {
  orc_list* l = list_new(n);
  for (int64_t i = 0; i < n; i++) {
    l->row_ptr[i] = l->nnz;
    for (int64_t j = 0; j < n; j++) {
      if (j == i) continue;
      double r2 = dist2(d, x + i * d, x + j * d, L);
      if (r2 < list_radius2(sig[i], sig[j], c, s)) list_push(l, (int32_t)j);
    }
  }
  l->row_ptr[n] = l->nnz;
  return l;
}

/* One row of the definition above (for sampled checks on large systems). */
int64_t orc_nlist_row(int d, int64_t n, double L, const double* x, const double* sig, double c,
                      double s, int64_t i, int32_t* out, int64_t cap) {
  int64_t m = 0;
  for (int64_t j = 0; j < n; j++) {
    if (j == i) continue;
    double r2 = dist2(d, x + i * d, x + j * d, L);
    if (r2 < list_radius2(sig[i], sig[j], c, s)) {
      if (m < cap) out[m] = (int32_t)j;
      m++;
    }
  }
  return m;
}

static int cmp_i32(const void* a, const void* b) {
  int32_t u = *(const int32_t*)a, v = *(const int32_t*)b;
  return (u > v) - (u < v);
}

/* Subcell of one atom along one axis: C = floor((x + L/2) n / L), clamped to
 * [0, n-1] (Sec. II.C; subcells are numbered from the box corner). */
static int cell_coord(double x, double L, int nc) {
  int c = (int)floor((x + 0.5 * L) * ((double)nc / L));
  if (c < 0) c = 0;
  if (c > nc - 1) c = nc - 1;
  return c;
}

/* The paper's cell path (Sec. II.C, Fig. 1): subcells of side L/n_cell with
 * flat index I = sum_k C_k n^(d-1-k); an outer loop over subcells, a second
 * loop over the 3^d linked subcells found on the fly by decoding a mixed-radix
 * counter, then the atoms of the subcell and the atoms of the linked subcell.
 * Reading for n_cell < 3 (the paper switches to an O(N^2) routine there): the
 * per-axis offsets -1, 0, +1 taken modulo n_cell are deduplicated, so each
 * linked subcell is visited once; with n_cell = 1 or 2 this visits every
 * subcell, which is the all-pairs search.  Rows are then sorted so the result
 * can be compared with the definition as a set.
 * ncell_override > 0 forces a smaller subcell count (any count whose subcells
 * are at least r_list_max wide gives the same list). */
orc_list* orc_nlist_cells(int d, int64_t n, double L, const double* x, const double* sig, double c,
                          double s, int ncell_override) {
  double smax = 0.0;
  for (int64_t i = 0; i < n; i++)
    if (sig[i] > smax) smax = sig[i];
  double rlmax = c * smax + s;
  int nc = orc_ncell(L, rlmax);
  if (ncell_override > 0 && ncell_override < nc) nc = ncell_override;
  int64_t ncells = 1;
  for (int k = 0; k < d; k++) ncells *= nc;

  /* linked subcells: atoms of each subcell in ascending id */
  int64_t* cell_of = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  int64_t* start = (int64_t*)calloc((size_t)ncells + 1, sizeof(int64_t));
  int64_t* members = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  for (int64_t i = 0; i < n; i++) {
    int64_t I = 0;
    for (int k = 0; k < d; k++) I = I * nc + cell_coord(x[i * d + k], L, nc);
    cell_of[i] = I;
    start[I + 1]++;
  }
  for (int64_t I = 0; I < ncells; I++) start[I + 1] += start[I];
  int64_t* fill = (int64_t*)malloc((size_t)ncells * sizeof(int64_t));
  memcpy(fill, start, (size_t)ncells * sizeof(int64_t));
  for (int64_t i = 0; i < n; i++) members[fill[cell_of[i]]++] = i;
  free(fill);

  /* per-axis offsets after deduplication */
  int radix = nc < 3 ? nc : 3;
  int offs[3];
  if (nc >= 3) { offs[0] = -1; offs[1] = 0; offs[2] = 1; }
  else if (nc == 2) { offs[0] = 0; offs[1] = 1; }
  else { offs[0] = 0; }
  int64_t nstencil = 1;
  for (int k = 0; k < d; k++) nstencil *= radix;

  /* gather hits per atom (one buffer per thread), then emit sorted rows */
  int64_t* cnt = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  int nthr = 1;
#ifdef _OPENMP
  nthr = omp_get_max_threads();
#endif
  int64_t* hcaps = (int64_t*)malloc((size_t)nthr * sizeof(int64_t));
  int64_t* nhs = (int64_t*)calloc((size_t)nthr, sizeof(int64_t));
  int32_t** his = (int32_t**)malloc((size_t)nthr * sizeof(int32_t*));
  int32_t** hjs = (int32_t**)malloc((size_t)nthr * sizeof(int32_t*));
  for (int t = 0; t < nthr; t++) {
    hcaps[t] = 16 * (n > 0 ? n : 1) / nthr + 16;
    his[t] = (int32_t*)malloc((size_t)hcaps[t] * sizeof(int32_t));
    hjs[t] = (int32_t*)malloc((size_t)hcaps[t] * sizeof(int32_t));
  }

#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t I = 0; I < ncells; I++) {
    if (start[I] == start[I + 1]) continue; /* no atom i in this subcell */
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    int C[16];
    /* decode I into subcell coordinates, axis 0 most significant */
    int64_t t = I;
    for (int k = d - 1; k >= 0; k--) { C[k] = (int)(t % nc); t /= nc; }
    for (int64_t q = 0; q < nstencil; q++) {
      /* decode the stencil counter and form the linked subcell index */
      int64_t u = q, J = 0, w = 1;
      for (int k = d - 1; k >= 0; k--) {
        int o = offs[u % radix];
        u /= radix;
        int cj = ((C[k] + o) % nc + nc) % nc;
        J += cj * w;
        w *= nc;
      }
      for (int64_t a = start[I]; a < start[I + 1]; a++) {
        int64_t i = members[a];
        for (int64_t b = start[J]; b < start[J + 1]; b++) {
          int64_t j = members[b];
          if (j == i) continue;
          double r2 = dist2(d, x + i * d, x + j * d, L);
          if (r2 < list_radius2(sig[i], sig[j], c, s)) {
            if (nhs[tid] == hcaps[tid]) {
              hcaps[tid] *= 2;
              his[tid] = (int32_t*)realloc(his[tid], (size_t)hcaps[tid] * sizeof(int32_t));
              hjs[tid] = (int32_t*)realloc(hjs[tid], (size_t)hcaps[tid] * sizeof(int32_t));
            }
            his[tid][nhs[tid]] = (int32_t)i;
            hjs[tid][nhs[tid]] = (int32_t)j;
            nhs[tid]++;
            cnt[i]++; /* atom i has one home subcell: one thread counts its row */
          }
        }
      }
    }
  }
  int64_t nh = 0;
  for (int t = 0; t < nthr; t++) nh += nhs[t];
  orc_list* l = list_new(n);
  for (int64_t i = 0; i < n; i++) l->row_ptr[i + 1] = l->row_ptr[i] + cnt[i];
  l->cap = nh > 0 ? nh : 1;
  l->cols = (int32_t*)realloc(l->cols, (size_t)l->cap * sizeof(int32_t));
  int64_t* pos = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  for (int64_t i = 0; i < n; i++) pos[i] = l->row_ptr[i];
  for (int t = 0; t < nthr; t++)
    for (int64_t h = 0; h < nhs[t]; h++) l->cols[pos[his[t][h]]++] = hjs[t][h];
  l->nnz = nh;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
  for (int64_t i = 0; i < n; i++)
    qsort(l->cols + l->row_ptr[i], (size_t)(l->row_ptr[i + 1] - l->row_ptr[i]), sizeof(int32_t),
          cmp_i32);
  for (int t = 0; t < nthr; t++) { free(his[t]); free(hjs[t]); }
  free(his); free(hjs); free(nhs); free(hcaps);
  free(pos); free(cnt);
  free(cell_of); free(start); free(members);
  return l;
}

/* ------------------------------------------------------------------------- */
/* Pair potentials and forces                                                */
/* ------------------------------------------------------------------------- */

/* One pair: returns U and sets *fcoef = -U'(r)/r, so that the force on i is
 * fcoef * (x_i - x_j).  Interaction iff r < r_c = c * sigma_ij.
 *  WCA: U = 4 eps [(sigma/r)^12 - (sigma/r)^6] + eps, the paper's Mie form with
 *       n = 6 (Sec. II.A) rewritten with sigma at the zero crossing and shifted
 *       so that U(2^(1/6) sigma) = 0.
 *  Harmonic soft spheres: U = eps/2 (1 - r/sigma)^2.
 *  Morse (Sec. II.A, eq. morsepot): U = eps [exp(-2a(r - sigma))
 *       - 2 exp(-a(r - sigma)) + 1] for r <= sigma, zero beyond (cutoff 1);
 *       -U'(r)/r = 2 a eps [exp(-2a(r - sigma)) - exp(-a(r - sigma))] / r. */
static double g_morse_a = 30.0;

/* Morse stiffness a used by every later call (the paper's value is 30). */
void orc_set_morse_a(double a) { g_morse_a = a; }

static double pair(int pot, double r2, double sij, double eps, double* fcoef) {
  if (pot == ORC_WCA) {
    double s2 = sij * sij / r2;
    double s6 = s2 * s2 * s2;
    *fcoef = 24.0 * eps * (2.0 * s6 * s6 - s6) / r2;
    return 4.0 * eps * (s6 * s6 - s6) + eps;
  } else if (pot == ORC_MORSE) {
    double r = sqrt(r2);
    double e1 = exp(-g_morse_a * (r - sij));
    double e2 = exp(-2.0 * g_morse_a * (r - sij));
    *fcoef = 2.0 * g_morse_a * eps * (e2 - e1) / r;
    return eps * (e2 - 2.0 * e1 + 1.0);
  } else {
    double r = sqrt(r2);
    double g = 1.0 - r / sij;
    *fcoef = eps * g / (sij * r);
    return 0.5 * eps * g * g;
  }
}

/* Force and per-atom energy from a full Verlet list (the paper's getforce,
 * Sec. II.B): F_i = sum over j in the row, in row order, of fcoef*(x_i - x_j)
 * for pairs inside the cutoff; e_i = half the sum of the pair energies.
 * Returns the total energy sum_{i<j} U_ij accumulated in ascending (i, j). */
double orc_forces(int d, int64_t n, double L, const double* x, const double* sig, int pot, double c,
                  double eps, const int64_t* row_ptr, const int32_t* cols, double* F,
                  double* e_atom) {
  double etot = 0.0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(+ : etot)
#endif
  for (int64_t i = 0; i < n; i++) {
    double ei = 0.0;
    for (int k = 0; k < d; k++) F[i * d + k] = 0.0;
    for (int64_t a = row_ptr[i]; a < row_ptr[i + 1]; a++) {
      int64_t j = cols[a];
      double sij = 0.5 * (sig[i] + sig[j]);
      double rc = c * sij;
      double r2 = dist2(d, x + i * d, x + j * d, L);
      if (!(r2 < rc * rc)) continue;
      double fc;
      double u = pair(pot, r2, sij, eps, &fc);
      for (int k = 0; k < d; k++) {
        double dx = min_image(x[j * d + k] - x[i * d + k], L);
        F[i * d + k] -= fc * dx;
      }
      ei += 0.5 * u;
      if (j > i) etot += u;
    }
    if (e_atom) e_atom[i] = ei;
  }
  return etot;
}

/* Energy of atom i with every other atom (brute force over all n), with i
 * given diameter si and the atoms a and b given diameters sa and sb instead
 * of their own (a, b < 0: none): sum_k U(r_ik, (si + s_k)/2) inside the
 * cutoff c (si + s_k)/2. */
static double swap_energy(int d, int64_t n, double L, const double* x, const double* sig, int pot,
                          double c, double eps, int64_t i, double si, int64_t a, double sa,
                          int64_t b, double sb) {
  double e = 0.0;
  for (int64_t k = 0; k < n; k++) {
    if (k == i) continue;
    const double sk = k == a ? sa : (k == b ? sb : sig[k]);
    const double sij = 0.5 * (si + sk);
    const double rc = c * sij;
    const double r2 = dist2(d, x + i * d, x + k * d, L);
    if (!(r2 < rc * rc)) continue;
    double fc;
    e += pair(pot, r2, sij, eps, &fc);
  }
  return e;
}

/* SWAP Monte Carlo (Sec. II.D): attempts k = 0 .. n_att-1 in order, each
 * exchanging the diameters of atoms i = pairs[2k] and j = pairs[2k+1] with
 * the diameters left by the earlier attempts.  The energy of the
 * interactions that involve i or j is summed before (eq. ebefore, E_b) and
 * after (E_a) the exchange, each sum over i's partners plus j's partners;
 * the pair i-j itself keeps its diameter sigma_ij and cancels.  The swap is
 * kept on the Metropolis rule: dE = E_a - E_b <= 0, or u_k < exp(-dE / T).
 * Unit masses: the kinetic energy is unchanged and no velocity is rescaled.
 * sig is updated in place; accepted[k] (optional) gets 1 or 0 and dE[k]
 * (optional) the energy change.  Returns the number of accepted swaps. */
int64_t orc_swap(int d, int64_t n, double L, const double* x, double* sig, int pot, double c,
                 double eps, int64_t n_att, const int32_t* pairs, const double* u, double T,
                 int32_t* accepted, double* dE) {
  int64_t nacc = 0;
  for (int64_t k = 0; k < n_att; k++) {
    const int64_t i = pairs[2 * k], j = pairs[2 * k + 1];
    const double si = sig[i], sj = sig[j];
    const double eb = swap_energy(d, n, L, x, sig, pot, c, eps, i, si, -1, 0.0, -1, 0.0) +
                      swap_energy(d, n, L, x, sig, pot, c, eps, j, sj, -1, 0.0, -1, 0.0);
    const double ea = swap_energy(d, n, L, x, sig, pot, c, eps, i, sj, j, si, -1, 0.0) +
                      swap_energy(d, n, L, x, sig, pot, c, eps, j, si, i, sj, -1, 0.0);
    const double de = i == j ? 0.0 : ea - eb;
    const int acc = de <= 0.0 || u[k] < exp(-de / T);
    if (acc) {
      sig[i] = sj;
      sig[j] = si;
      nacc++;
    }
    if (accepted) accepted[k] = acc;
    if (dE) dE[k] = de;
  }
  return nacc;
}

/* The virial and the coordination number of getthermo (Sec. II.E) from a
 * full CSR list: out[0] = W = sum over pairs i<j inside the cutoff of
 * r_ij . F_ij = fcoef r^2 (so that P = (2 KE + W) / (d V)); out[1] = Z, the
 * mean number of neighbours inside the cutoff per atom. */
void orc_virial(int d, int64_t n, double L, const double* x, const double* sig, int pot, double c,
                double eps, const int64_t* row_ptr, const int32_t* cols, double* out) {
  double w = 0.0, pairs = 0.0;
  for (int64_t i = 0; i < n; i++) {
    for (int64_t a = row_ptr[i]; a < row_ptr[i + 1]; a++) {
      int64_t j = cols[a];
      if (j <= i) continue;
      double sij = 0.5 * (sig[i] + sig[j]);
      double rc = c * sij;
      double r2 = dist2(d, x + i * d, x + j * d, L);
      if (!(r2 < rc * rc)) continue;
      double fc;
      pair(pot, r2, sij, eps, &fc);
      w += fc * r2;
      pairs += 1.0;
    }
  }
  out[0] = w;
  out[1] = 2.0 * pairs / (double)n;
}

/* Force on one atom by the definition (every other atom, ascending j). */
double orc_force_one(int d, int64_t n, double L, const double* x, const double* sig, int pot,
                     double c, double eps, int64_t i, double* Fi) {
  double ei = 0.0;
  for (int k = 0; k < d; k++) Fi[k] = 0.0;
  for (int64_t j = 0; j < n; j++) {
    if (j == i) continue;
    double sij = 0.5 * (sig[i] + sig[j]);
    double rc = c * sij;
    double r2 = dist2(d, x + i * d, x + j * d, L);
    if (!(r2 < rc * rc)) continue;
    double fc;
    double u = pair(pot, r2, sij, eps, &fc);
    for (int k = 0; k < d; k++) {
      double dx = min_image(x[j * d + k] - x[i * d + k], L);
      Fi[k] -= fc * dx;
    }
    ei += 0.5 * u;
  }
  return ei;
}

/* ------------------------------------------------------------------------- */
/* Integrators                                                               */
/* ------------------------------------------------------------------------- */

typedef struct {
  int d;
  int64_t n;
  double L;
  int pot;
  double c, s, eps;
} orc_sys;

typedef struct {
  orc_list* nl;
  double* xref;
  int64_t builds;
} orc_nlstate;

static void rebuild(const orc_sys* S, const double* x, const double* sig, orc_nlstate* st) {
  orc_list_free(st->nl);
  st->nl = orc_nlist_cells(S->d, S->n, S->L, x, sig, S->c, S->s, 0);
  memcpy(st->xref, x, (size_t)(S->n * S->d) * sizeof(double));
  st->builds++;
}

/* Rebuild trigger: the largest minimum-image displacement since the last
 * build exceeds half the skin (compared squared).  This is the rule the
 * hot path uses; the paper's own needsrebuild (Sec. II.C) checks a 0.1 %
 * quantile as well and only every n_bet steps. */
static int needs_rebuild(const orc_sys* S, const double* x, const orc_nlstate* st) {
  double hs2 = 0.25 * S->s * S->s, dmax = 0.0;
  for (int64_t i = 0; i < S->n; i++) {
    double r2 = dist2(S->d, st->xref + i * S->d, x + i * S->d, S->L);
    if (r2 > dmax) dmax = r2;
  }
  return dmax > hs2;
}

static double kinetic(int64_t m, const double* v) {
  double ke = 0.0;
  for (int64_t a = 0; a < m; a++) ke += v[a] * v[a];
  return 0.5 * ke;
}

/* Displacement observables of Sec. II.E over the unwrapped displacements
 * dr[n*d] of every atom since the reference state:
 *   out[0] = <|dr|^2>, out[1] = <|dr|^4>  (averages over the n atoms),
 *   out[2] = alpha_2 = d <|dr|^4> / ((d+2) <|dr|^2>^2) - 1   (eq. ngp),
 *   out[3] = f_ov = (1/n) sum_i Theta(0.1 d - |dr_i|)        (eq. fov),
 * with the diameter scale sigma~ = 1 (Sec. II.A) and Theta(0) = 0.  Reading:
 * alpha_2 is undefined while nothing has moved; it is reported as 0. */
void orc_disp_moments(int d, int64_t n, const double* dr, double* out) {
  double m2 = 0.0, m4 = 0.0, ov = 0.0;
  const double a = 0.1 * d;
  for (int64_t i = 0; i < n; i++) {
    double r2 = 0.0;
    for (int k = 0; k < d; k++) r2 += dr[i * d + k] * dr[i * d + k];
    m2 += r2;
    m4 += r2 * r2;
    if (sqrt(r2) < a) ov += 1.0;
  }
  m2 /= (double)n;
  m4 /= (double)n;
  out[0] = m2;
  out[1] = m4;
  out[2] = m2 > 0.0 ? d * m4 / ((d + 2) * m2 * m2) - 1.0 : 0.0;
  out[3] = ov / (double)n;
}

/* Self part of the van Hove function (eq. VGC, Sec. II.E) as a histogram of
 * the displacement lengths: hist[b] = #{i : b w <= |dr_i| < (b+1) w} for
 * b < nbins and hist[nbins] = #{i : |dr_i| >= nbins w}; G_s(r_b) is
 * hist[b] / (n w). */
void orc_van_hove(int d, int64_t n, const double* dr, int32_t nbins, double w, int64_t* hist) {
  for (int32_t b = 0; b <= nbins; b++) hist[b] = 0;
  for (int64_t i = 0; i < n; i++) {
    double r2 = 0.0;
    for (int k = 0; k < d; k++) r2 += dr[i * d + k] * dr[i * d + k];
    const double r = sqrt(r2);
    int32_t b = nbins;
    for (int32_t c = 0; c < nbins; c++)
      if (r >= c * w && r < (c + 1) * w) { b = c; break; }
    hist[b]++;
  }
}

/* Velocity Verlet, the kick-drift-kick leapfrog of Sec. II.B with unit masses:
 * per step v += dt/2 F; x += dt v; wrap; rebuild if needed; F = F(x);
 * v += dt/2 F.  The first list is built at step 0.
 * With tau > 0 the second kick carries the Berendsen thermostat (the paper
 * folds it into that kick, Sec. II.B and II.E): v = lambda (v + dt/2 F) with
 * lambda^2 = 1 + (dt/tau)(T0/T - 1), T = 2 KE / (d (n-1)) at the previous
 * full step (reading: a single pass over the atoms knows only that T; lambda
 * is 1 when that KE is 0).  tau = 0: NVE.
 * thermo (optional) receives nsteps+1 rows of (KE, PE) at the full steps;
 * obs (optional) nsteps+1 rows of orc_disp_moments of the unwrapped
 * displacement since step 0, which advances by dt v with every drift (the
 * wrap only relabels the image); dr_out (optional, [n*d]) that displacement
 * at the end.  Returns the number of list builds. */
int64_t orc_vv(int d, int64_t n, double L, int pot, double c, double s, double eps, double* x,
               double* v, const double* sig, int64_t nsteps, double dt, double tau, double T0,
               double* thermo, double* obs, double* dr_out) {
  orc_sys S = {d, n, L, pot, c, s, eps};
  int64_t m = n * d;
  orc_nlstate st = {0};
  st.xref = (double*)malloc((size_t)m * sizeof(double));
  double* F = (double*)malloc((size_t)m * sizeof(double));
  double* dr = (double*)calloc((size_t)m, sizeof(double));
  for (int64_t a = 0; a < m; a++) x[a] = orc_wrap1(x[a], L);
  rebuild(&S, x, sig, &st);
  double pe = orc_forces(d, n, L, x, sig, pot, c, eps, st.nl->row_ptr, st.nl->cols, F, NULL);
  double ke = kinetic(m, v);
  if (thermo) { thermo[0] = ke; thermo[1] = pe; }
  if (obs) orc_disp_moments(d, n, dr, obs);
  for (int64_t t = 1; t <= nsteps; t++) {
    double lam = 1.0;
    if (tau > 0.0 && ke > 0.0) {
      const double T = 2.0 * ke / ((double)d * (double)(n - 1));
      lam = sqrt(1.0 + dt / tau * (T0 / T - 1.0));
    }
    for (int64_t a = 0; a < m; a++) v[a] += 0.5 * dt * F[a];
    for (int64_t a = 0; a < m; a++) {
      x[a] = orc_wrap1(x[a] + dt * v[a], L);
      dr[a] += dt * v[a];
    }
    if (needs_rebuild(&S, x, &st)) rebuild(&S, x, sig, &st);
    pe = orc_forces(d, n, L, x, sig, pot, c, eps, st.nl->row_ptr, st.nl->cols, F, NULL);
    for (int64_t a = 0; a < m; a++) v[a] = lam * (v[a] + 0.5 * dt * F[a]);
    ke = kinetic(m, v);
    if (thermo) { thermo[2 * t] = ke; thermo[2 * t + 1] = pe; }
    if (obs) orc_disp_moments(d, n, dr, obs + 4 * t);
  }
  int64_t b = st.builds;
  if (dr_out) memcpy(dr_out, dr, (size_t)m * sizeof(double));
  orc_list_free(st.nl);
  free(st.xref);
  free(F);
  free(dr);
  return b;
}

/* FIRE 2.0 parameters.  The paper (Sec. II.B) uses the semi-implicit-Euler
 * variant of FIRE 2.0 but prints no parameter values; these fields carry the
 * values of the FIRE 2.0 publication it cites. */
typedef struct {
  double dt0, dtmax, dtmin;
  double finc, fdec, alpha0, falpha;
  int64_t ndelay, nneg_max, maxiter;
  int64_t initial_delay;
  double ftol; /* stop when max_i |F_i| < ftol */
  double etol; /* or when PE/N < etol (0 disables) */
} orc_fire_params;

typedef struct {
  int64_t iters;
  int64_t builds;
  double fmax;
  double energy;
  int64_t status; /* 0 converged, 1 not converged */
} orc_fire_result;

/* FIRE 2.0 with the semi-implicit Euler integrator (unit masses), Sec. II.B.
 * Each iteration: P = F.v; on P > 0 count up and, after the delay, grow dt
 * and shrink alpha; on P <= 0 count down, shrink dt and reset alpha (except
 * inside the initial delay), step back x -= dt/2 v and zero v; then
 * v += dt F, mix v = (1-alpha) v + alpha |v| F/|F| with norms over all dN
 * components, x += dt v, wrap, rebuild if needed, recompute F.
 * Convergence is checked on the fresh force before each iteration.
 * trace (optional, trace_cap rows of ORC_FIRE_TRACE doubles) receives one
 * row per iteration: P, the dt and alpha the update used, the counts of
 * consecutive P > 0 and P <= 0 iterations after the control step, and 1 when
 * the iteration stepped back and zeroed v (else 0). */
#define ORC_FIRE_TRACE 6
void orc_fire_traced(int d, int64_t n, double L, int pot, double c, double s, double eps, double* x,
                     const double* sig, const orc_fire_params* p, orc_fire_result* res,
                     double* trace, int64_t trace_cap) {
  orc_sys S = {d, n, L, pot, c, s, eps};
  int64_t m = n * d;
  orc_nlstate st = {0};
  st.xref = (double*)malloc((size_t)m * sizeof(double));
  double* F = (double*)malloc((size_t)m * sizeof(double));
  double* v = (double*)calloc((size_t)m, sizeof(double));
  for (int64_t a = 0; a < m; a++) x[a] = orc_wrap1(x[a], L);
  rebuild(&S, x, sig, &st);
  double pe = orc_forces(d, n, L, x, sig, pot, c, eps, st.nl->row_ptr, st.nl->cols, F, NULL);
  double dt = p->dt0, alpha = p->alpha0;
  int64_t npos = 0, nneg = 0, it = 0;
  int64_t status = 1;
  double fmax2 = 0.0;
  for (;;) {
    fmax2 = 0.0;
    for (int64_t i = 0; i < n; i++) {
      double f2 = 0.0;
      for (int k = 0; k < d; k++) f2 += F[i * d + k] * F[i * d + k];
      if (f2 > fmax2) fmax2 = f2;
    }
    if (sqrt(fmax2) < p->ftol || (p->etol > 0.0 && pe / (double)n < p->etol)) { status = 0; break; }
    if (it >= p->maxiter) break;
    double P = 0.0;
    for (int64_t a = 0; a < m; a++) P += F[a] * v[a];
    int back = 0;
    if (P > 0.0) {
      npos++;
      nneg = 0;
      if (npos > p->ndelay) {
        dt = fmin(dt * p->finc, p->dtmax);
        alpha *= p->falpha;
      }
    } else {
      npos = 0;
      nneg++;
      if (nneg > p->nneg_max) break;
      if (!(p->initial_delay && it < p->ndelay)) {
        if (dt * p->fdec >= p->dtmin) dt *= p->fdec;
        alpha = p->alpha0;
      }
      for (int64_t a = 0; a < m; a++) x[a] = x[a] - 0.5 * dt * v[a];
      for (int64_t a = 0; a < m; a++) v[a] = 0.0;
      back = 1;
    }
    if (trace && it < trace_cap) {
      double* row = trace + it * ORC_FIRE_TRACE;
      row[0] = P;
      row[1] = dt;
      row[2] = alpha;
      row[3] = (double)npos;
      row[4] = (double)nneg;
      row[5] = (double)back;
    }
    for (int64_t a = 0; a < m; a++) v[a] += dt * F[a];
    double vv = 0.0, ff = 0.0;
    for (int64_t a = 0; a < m; a++) { vv += v[a] * v[a]; ff += F[a] * F[a]; }
    double vn = sqrt(vv), fn = sqrt(ff);
    if (fn > 0.0) {
      double mixf = alpha * vn / fn;
      for (int64_t a = 0; a < m; a++) v[a] = (1.0 - alpha) * v[a] + mixf * F[a];
    }
    for (int64_t a = 0; a < m; a++) x[a] = orc_wrap1(x[a] + dt * v[a], L);
    if (needs_rebuild(&S, x, &st)) rebuild(&S, x, sig, &st);
    pe = orc_forces(d, n, L, x, sig, pot, c, eps, st.nl->row_ptr, st.nl->cols, F, NULL);
    it++;
  }
  res->iters = it;
  res->builds = st.builds;
  res->fmax = sqrt(fmax2);
  res->energy = pe;
  res->status = status;
  orc_list_free(st.nl);
  free(st.xref);
  free(F);
  free(v);
}

void orc_fire(int d, int64_t n, double L, int pot, double c, double s, double eps, double* x,
              const double* sig, const orc_fire_params* p, orc_fire_result* res) {
  orc_fire_traced(d, n, L, pot, c, s, eps, x, sig, p, res, NULL, 0);
}
