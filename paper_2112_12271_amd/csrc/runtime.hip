// runtime.hip -- host runtime behind the C ABI (include/hdmd.h): workspace
// layout, validation, launch sequences, hipGraph capture of step / iteration
// chunks, the build-tile autotuner, and the batch tables of uneven replicas.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "dispatch.h"
#include "hdmd.h"

namespace hdmd {

static_assert(kThermoCols == HDMD_THERMO_COLS, "thermo row layout");

static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) return fail(HDMD_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

static inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// SWAP Monte Carlo scratch (fixed size, whatever the number of attempts):
// round counters, the two put-off queues, a batch's dE and conflict masks.
struct SwapScratch {
  long long* ctl;      // [0] attempts put off, [1] kept, [2] next attempt not begun, [3] bad id
  int32_t* off[2];     // put-off queues, kSwapBatch each
  double* de;          // 3 kSwapBatch
  unsigned long long* conf;  // kSwapBatch x kSwapBatch/64
};
constexpr size_t kSwapCtlBytes = 256, kSwapOffBytes = kSwapBatch * 4;
constexpr size_t kSwapDeBytes = 3 * kSwapBatch * 8, kSwapConfBytes = kSwapBatch * (kSwapBatch / 64) * 8;
constexpr size_t kSwapScratchBytes = kSwapCtlBytes + 2 * kSwapOffBytes + kSwapDeBytes + kSwapConfBytes;

static SwapScratch swap_scratch(void* base) {
  char* b = static_cast<char*>(base);
  SwapScratch w;
  w.ctl = reinterpret_cast<long long*>(b);
  w.off[0] = reinterpret_cast<int32_t*>(b + kSwapCtlBytes);
  w.off[1] = reinterpret_cast<int32_t*>(b + kSwapCtlBytes + kSwapOffBytes);
  w.de = reinterpret_cast<double*>(b + kSwapCtlBytes + 2 * kSwapOffBytes);
  w.conf = reinterpret_cast<unsigned long long*>(b + kSwapCtlBytes + 2 * kSwapOffBytes + kSwapDeBytes);
  return w;
}

// ---------------------------------------------------------------------------
// geometry and workspace plan
// ---------------------------------------------------------------------------
struct Plan {
  int d = 0, dr = 0, dq = 0, dy = 0;
  int n = 0, npad = 0, ncell = 0, radix = 0, ncells = 0, nstencil = 0, nchunks = 0;
  int ntiles = 0, nwaves = 0, width = 0;
  bool wrap = false, mix = false, morse = false;
  // reach: stencil radius in subcells (1: side >= r_l,max, 3^d stencil; 2:
  // half-size subcells, 5^d stencil); key_wrap/key_occ: the autotuner's key,
  // taken from the grid of side >= r_l,max; nh_auto: half-size subcells per
  // axis the autotuner may take (0: none)
  int reach = 1, key_wrap = 0, key_occ = 0, nh_auto = 0;
  int lpa = 1, row_key = 0;  // lanes per atom of the force kernels and their key
  double rlmax = 0;
  size_t off_desc = 0, off_x[2] = {0, 0}, off_q[2] = {0, 0}, off_v[2] = {0, 0},
         off_oid[2] = {0, 0}, off_f = 0, off_xref = 0, off_disp[2] = {0, 0}, off_ycell = 0, off_qc = 0, off_qc16 = 0,
         off_cell_of = 0,
         off_rank = 0, off_cell_count = 0, off_cell_flat = 0, off_cell_local = 0, off_chunk_sum = 0,
         off_chunk_off = 0, off_key = 0, off_src = 0, off_nl = 0, off_nlen = 0, off_part = 0,
         off_swap = 0;
  size_t bytes = 0;
};

static int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; i++) {
    r *= b;
    if (r > (int64_t(1) << 40)) return r;
  }
  return r;
}

// Subcells per axis: floor(L / r_list_max) (eq. setnc with the largest
// diameter sigma_max and skin s), lowered while a subcell would be narrower
// than the list radius by more than rounding, and while the subcell count
// would exceed 2^26 or four per atom (fewer, wider subcells list the same
// pairs).
static int64_t cell_cap(const hdmd_system& s) {
  return std::min<int64_t>(int64_t(1) << 26, std::max<int64_t>(64, 4 * s.n));
}

static int choose_ncell(const hdmd_system& s, double rlmax) {
  double q = std::floor(s.box_l / rlmax);
  int nc = q < 1.0 ? 1 : (q > 4096.0 ? 4096 : (int)q);
  while (nc > 1 && s.box_l / (double)nc < rlmax * (1.0 + 1.0e-9)) nc--;
  const int64_t cap = cell_cap(s);
  while (nc > 1 && ipow(nc, s.d) > cap) nc--;
  return nc;
}

// Half-size subcells (Sec. II.C: side at least r_l,max/2, each linked to the
// 5^d - 1 around it): floor(2 L / r_l,max) per axis with the same rounding
// guard, lowered while the count exceeds cap.  0 where fewer than 5 per axis
// would remain: there the 5^d stencil would meet a subcell twice.
static int half_ncell(const hdmd_system& s, double rlmax, int64_t cap) {
  const double hr = 0.5 * rlmax;
  const double q = std::floor(s.box_l / hr);
  int nc = q < 1.0 ? 1 : (q > 4096.0 ? 4096 : (int)q);
  while (nc > 1 && s.box_l / (double)nc < hr * (1.0 + 1.0e-9)) nc--;
  while (nc > 5 && ipow(nc, s.d) > cap) nc--;
  return (nc >= 5 && ipow(nc, s.d) <= cap) ? nc : 0;
}

static int occ_bucket(int64_t n, int64_t ncells) {
  double occ = (double)n / (double)ncells;
  int b = 0;
  while (occ >= 2.0 && b < 20) {
    occ *= 0.5;
    b++;
  }
  return b;
}

// the autotuner's grid for a key: 0 (not tuned yet), 1 or 2 (reach)
static int tuned_reach(int d, int wrap, int occ);
// lanes per atom of the force kernels for a system (the autotuner's, or 1),
// keyed by the row-length bucket
static int lanes_for(const hdmd_system* s, int d, int rowkey);

// The force kernels' key: half-octaves of the expected row length, the atoms
// in a ball of the largest list radius at the mean number density, n V_d(r)
// / L^d (rows, not the subcell occupancy, decide how many lanes pay).
static int row_bucket(const hdmd_system& s, double rlmax) {
  const double vd = std::pow(M_PI, 0.5 * s.d) / std::tgamma(0.5 * s.d + 1.0) * std::pow(rlmax, s.d);
  const double rows = (double)s.n * vd / std::pow(s.box_l, s.d);
  return (int)std::lround(2.0 * std::log2(std::max(rows, 1.0)));
}

static int make_plan(const hdmd_system* s, Plan& p) {
  if (!s) return fail(HDMD_ERR_ARG, "null system");
  if (s->d < kMinD || s->d > kMaxD) return fail(HDMD_ERR_ARG, "d must be in [2, 10]");
  if (s->n < 2 || s->n > (int64_t(1) << 30)) return fail(HDMD_ERR_ARG, "n must be in [2, 2^30]");
  if (!(s->box_l > 0) || !std::isfinite(s->box_l)) return fail(HDMD_ERR_ARG, "box_l must be > 0");
  if (!(s->cutoff > 0) || !std::isfinite(s->cutoff)) return fail(HDMD_ERR_ARG, "cutoff must be > 0");
  if (!(s->skin >= 0) || !std::isfinite(s->skin)) return fail(HDMD_ERR_ARG, "skin must be >= 0");
  if (!(s->epsilon > 0) || !std::isfinite(s->epsilon)) return fail(HDMD_ERR_ARG, "epsilon must be > 0");
  if (!(s->sigma_max > 0) || !std::isfinite(s->sigma_max)) return fail(HDMD_ERR_ARG, "sigma_max must be > 0");
  if (s->potential != HDMD_WCA && s->potential != HDMD_HARMONIC && s->potential != HDMD_MORSE)
    return fail(HDMD_ERR_ARG, "bad potential");
  if (s->potential == HDMD_MORSE && !(s->morse_a > 0.0 && std::isfinite(s->morse_a)))
    return fail(HDMD_ERR_ARG, "morse_a must be positive");
  if (s->precision != HDMD_FP64 && s->precision != HDMD_MIXED) return fail(HDMD_ERR_ARG, "bad precision");
  if (!(s->thermostat_tau >= 0) || !std::isfinite(s->thermostat_tau) || !(s->target_temp >= 0) ||
      !std::isfinite(s->target_temp))
    return fail(HDMD_ERR_ARG, "thermostat_tau and target_temp must be >= 0");
  if (s->max_neighbors < 1 || s->max_neighbors > (1 << 20)) return fail(HDMD_ERR_ARG, "max_neighbors must be in [1, 2^20]");
  if (s->box_l < 2.0 * s->cutoff * s->sigma_max)
    return fail(HDMD_ERR_BOX, "box_l < 2 * cutoff * sigma_max: minimum image is ambiguous");
  p.d = s->d;
  p.dr = s->d <= 3 ? 4 : (s->d <= 7 ? 8 : 16);
  p.dq = s->d <= 2 ? 4 : (s->d <= 6 ? 8 : 16);
  p.dy = (s->d + 3) & ~3;
  p.n = (int)s->n;
  p.npad = (int)((s->n + kTile - 1) / kTile * kTile);  // whole 64-atom tiles
  p.rlmax = s->cutoff * s->sigma_max + s->skin;
  // the grid: subcells of side >= r_l,max (3^d stencil) or half-size ones
  // (5^d stencil), by request or, for HDMD_SUBCELLS_AUTO, as the autotuner
  // chose for the key; the workspace holds the cell arrays of either grid
  // the system may take, so its layout does not depend on the choice
  const int ncf = choose_ncell(*s, p.rlmax);
  const int64_t cells_full = ipow(ncf, p.d);
  p.key_wrap = ncf <= 2;
  p.key_occ = occ_bucket(p.n, cells_full);
  int64_t cells_alloc = cells_full;
  bool need_ycell = ncf <= 2, need_qc = ncf > 2;
  p.reach = 1;
  p.ncell = ncf;
  if (s->subcells == HDMD_SUBCELLS_HALF) {
    const int nh = half_ncell(*s, p.rlmax, int64_t(1) << 26);
    if (!nh)
      return fail(HDMD_ERR_ARG, "half-size subcells need box_l >= 5 r_l,max / 2 (five per axis) "
                                "and at most 2^26 of them");
    p.reach = 2;
    p.ncell = nh;
    cells_alloc = ipow(nh, p.d);
    need_ycell = false;
    need_qc = true;
  } else if (s->subcells == HDMD_SUBCELLS_AUTO) {
    p.nh_auto = half_ncell(*s, p.rlmax, cell_cap(*s));
    if (p.nh_auto) {
      cells_alloc = std::max<int64_t>(cells_alloc, ipow(p.nh_auto, p.d));
      need_qc = true;
      if (tuned_reach(p.d, p.key_wrap, p.key_occ) == 2) {
        p.reach = 2;
        p.ncell = p.nh_auto;
      }
    }
  } else if (s->subcells != HDMD_SUBCELLS_FULL) {
    return fail(HDMD_ERR_ARG, "subcells must be HDMD_SUBCELLS_AUTO, _FULL or _HALF");
  }
  p.radix = p.reach == 2 ? 5 : (p.ncell < 3 ? p.ncell : 3);
  p.ncells = (int)ipow(p.ncell, p.d);
  p.nstencil = (int)ipow(p.radix, p.d);
  p.nchunks = (p.ncells + kChunk - 1) / kChunk;
  const int64_t chunks_alloc = (cells_alloc + kChunk - 1) / kChunk;
  p.ntiles = p.npad / kTile;
  p.nwaves = p.npad / kWave;
  p.width = s->max_neighbors;
  p.wrap = p.reach == 1 && p.ncell <= 2;
  p.mix = s->precision == HDMD_MIXED;
  p.row_key = row_bucket(*s, p.rlmax);
  p.lpa = lanes_for(s, p.d, p.row_key);
  p.morse = s->potential == HDMD_MORSE;
  const size_t np = (size_t)p.npad, vsz = p.mix ? 4 : 8;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  p.off_desc = take(sizeof(SysDev));
  for (int b = 0; b < 2; b++) p.off_x[b] = take(np * p.dr * 8);
  for (int b = 0; b < 2; b++) p.off_q[b] = take(p.mix ? np * p.dq * 4 : 0);
  for (int b = 0; b < 2; b++) p.off_v[b] = take(np * p.d * vsz);
  for (int b = 0; b < 2; b++) p.off_oid[b] = take(np * 4);
  p.off_f = take(np * p.d * vsz);
  p.off_xref = take(np * p.d * 8);
  for (int b = 0; b < 2; b++) p.off_disp[b] = take(np * p.d * 8);
  p.off_ycell = take(need_ycell ? np * p.dy * 4 : 0);
  p.off_qc = take(need_qc ? np * 16 : 0);
  p.off_qc16 = take(np * 32);
  p.off_cell_of = take(np * 4);
  p.off_rank = take(np * 4);
  p.off_cell_count = take((size_t)cells_alloc * 4);
  p.off_cell_flat = take((size_t)(cells_alloc + 1) * 4);
  p.off_cell_local = take((size_t)cells_alloc * 4);
  p.off_chunk_sum = take((size_t)chunks_alloc * 4);
  p.off_chunk_off = take((size_t)chunks_alloc * 4);
  p.off_key = take(np * 4);
  p.off_src = take(np * 4);
  p.off_nl = take((size_t)p.width * np * 4);
  p.off_nlen = take(np * 4);
  p.off_part = take((size_t)p.nwaves * kPart * 8);
  p.off_swap = take(kSwapScratchBytes);
  p.bytes = o;
  return HDMD_OK;
}

template <typename T>
static T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

static SysDev make_desc(const hdmd_system* s, const Plan& p, void* ws) {
  SysDev h;
  std::memset(&h, 0, sizeof(h));
  h.d = p.d;
  h.potential = s->potential;
  h.morse_a = s->potential == HDMD_MORSE ? s->morse_a : 0.0;
  h.tau_t = s->thermostat_tau;
  h.temp_t = s->target_temp;
  h.vscale = 1.0;
  h.precision = s->precision;
  h.n = p.n;
  h.npad = p.npad;
  h.ncell = p.ncell;
  h.reach = p.reach;
  h.lpa = p.lpa;
  h.radix = p.radix;
  h.ncells = p.ncells;
  h.nstencil = p.nstencil;
  h.width = p.width;
  h.nchunks = p.nchunks;
  h.ntiles = p.ntiles;
  h.mode = MODE_STATIC;
  h.wrap = p.wrap;
  h.nwaves = p.nwaves;
  h.L = s->box_l;
  h.hL = 0.5 * s->box_l;
  h.cutoff = s->cutoff;
  h.skin = s->skin;
  h.eps = s->epsilon;
  h.sigma_max = s->sigma_max;
  h.rlmax = p.rlmax;
  h.lsc = s->box_l / (double)p.ncell;
  h.inv_lsc = (double)p.ncell / s->box_l;
  h.halfskin2 = 0.25 * s->skin * s->skin;
  h.fxscale = 4294967296.0 / s->box_l;
  h.fxinv = s->box_l / 4294967296.0;
  h.qinv = (double)kQScale / h.lsc;
  h.qmarg = 0.5 * std::sqrt((double)p.d) * (1.0 + 1e-6);
  h.ysort = p.n < (1 << 23) ? 1 : 0;
  if (p.wrap) {
    // n_cell <= 2: prefilter on 16-bit wrapped coordinates, unit Delta = L/2^16;
    // |u_j - u_i|^2 < tq keeps every pair within r_l,max (each axis is off by
    // at most one unit), and a row is skipped when the gaps to its subcells,
    // one unit short per axis, reach r_l,max
    const double delta = s->box_l / 65536.0;
    const double thr = p.rlmax / delta + std::sqrt((double)p.d) * (1.0 + 1e-6);
    h.tq = (int32_t)std::min(std::floor(thr * thr) + 1.0, 2147483000.0);
    const double rc = p.rlmax / delta;
    h.tcull = (int32_t)std::min(std::ceil(rc * rc), 2147483000.0);
  } else {
    // int8 prefilter threshold: ((r_l,max + Delta sqrt(d)) / Delta)^2, Delta =
    // L_sc / 250, rounded down and made strict (+1), with slack on sqrt(d)
    const double delta = h.lsc / (double)kQScale;
    const double thr = (p.rlmax + delta * std::sqrt((double)p.d) * (1.0 + 1e-6)) / delta;
    h.tq = (int32_t)std::floor(thr * thr) + 1;
    // a home atom skips a row of linked subcells when its gap to the row,
    // taken one unit short per axis, is at least r_l,max: S >= (r_l,max/Delta)^2
    const double rc = p.rlmax / delta;
    h.tcull = (int32_t)std::ceil(rc * rc);
  }
  // FP32 prefilter radius: the largest list radius enlarged by a relative
  // 1e-4 plus 1e-5 L, far above the FP32 rounding of offsets from subcell
  // centres (|y| <= L_sc) and of the box length.
  const double rf = p.rlmax * (1.0 + 1.0e-4) + 1.0e-5 * s->box_l;
  h.rl2f = std::nextafter((float)(rf * rf), INFINITY);
  h.lscf = (float)h.lsc;
  h.Lf = (float)s->box_l;
  for (int b = 0; b < 2; b++) {
    h.x[b] = at<double>(ws, p.off_x[b]);
    h.q[b] = p.mix ? at<int32_t>(ws, p.off_q[b]) : nullptr;
    h.v[b] = at<void>(ws, p.off_v[b]);
    h.oid[b] = at<int32_t>(ws, p.off_oid[b]);
  }
  h.f = at<void>(ws, p.off_f);
  h.xref = at<double>(ws, p.off_xref);
  for (int b = 0; b < 2; b++) h.disp[b] = at<double>(ws, p.off_disp[b]);
  h.ycell = p.wrap ? at<float>(ws, p.off_ycell) : nullptr;
  h.qc = p.wrap ? nullptr : at<int32_t>(ws, p.off_qc);
  h.qc16 = at<int32_t>(ws, p.off_qc16);  // int16 offsets, or wrapped 16-bit coordinates
  h.cell_of = at<int32_t>(ws, p.off_cell_of);
  h.rank = at<int32_t>(ws, p.off_rank);
  h.cell_count = at<int32_t>(ws, p.off_cell_count);
  h.cell_flat = at<int32_t>(ws, p.off_cell_flat);
  h.cell_local = at<int32_t>(ws, p.off_cell_local);
  h.chunk_sum = at<int32_t>(ws, p.off_chunk_sum);
  h.chunk_off = at<int32_t>(ws, p.off_chunk_off);
  h.key = at<int32_t>(ws, p.off_key);
  h.src = at<int32_t>(ws, p.off_src);
  h.nl = at<int32_t>(ws, p.off_nl);
  h.nlen = at<int32_t>(ws, p.off_nlen);
  h.part = at<double>(ws, p.off_part);
  h.force_rebuild = 1;
  h.status = SLOT_RUNNING;
  return h;
}

// ---------------------------------------------------------------------------
// build-tile autotuner: workgroup size of the list build per (d, wrap,
// occupancy bucket), chosen by timing every variant on the first build that
// meets the key.  All variants produce identical lists.
// ---------------------------------------------------------------------------
// Per key: the grid an autotuned system takes (reach 1 or 2; 0: not decided)
// and the best build variant on each grid (0: not timed).
struct Tuned {
  int reach = 0, blk[3] = {0, 0, 0};
};
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, Tuned> g_tune;
// lanes per atom of the force kernels per (d, precision form, row bucket)
static std::map<std::tuple<int, int, int>, int> g_lanes;

static bool tuning_enabled() {
  const char* e = std::getenv("HDMD_AUTOTUNE");
  return !(e && e[0] == '0');
}

static int tuned_reach(int d, int wrap, int occ) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find({d, wrap, occ});
  return it == g_tune.end() ? 0 : it->second.reach;
}

static int default_blk(const Plan& p) {
  const char* e = std::getenv("HDMD_BUILD_BLK");
  if (e) return std::atoi(e);
  (void)p;
  return 1;
}

static int lookup_blk(const Plan& p, bool* known) {
  if (std::getenv("HDMD_BUILD_BLK")) {  // explicit choice wins over the tuned one
    *known = true;
    return default_blk(p);
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find({p.d, p.key_wrap, p.key_occ});
  // an autotuned system's key is known once its grid is decided
  const bool need_grid = p.nh_auto > 0;
  if (it == g_tune.end() || !it->second.blk[p.reach] || (need_grid && !it->second.reach)) {
    *known = false;
    return default_blk(p);
  }
  *known = true;
  return it->second.blk[p.reach];
}



// Lanes per atom of the force kernels (1, 2 or 4 lanes share an atom's row;
// their partial sums meet in a tree that depends on the count, so the choice
// fixes the rounding of the forces): chosen by the autotuner per (d,
// precision form, row bucket) and kept for every later system with that key,
// alone or in a batch.  Morse systems take one lane.  HDMD_LPA overrides.
static int lpa_env() {
  const char* e = std::getenv("HDMD_LPA");
  if (!e) return 0;
  const int v = std::atoi(e);
  return v >= 4 ? 4 : (v >= 2 ? 2 : 1);
}

// Systems below this size take one lane per atom without timing: their force
// kernels are short, and in a batch every other lane count costs a launch of
// its own per class, on every iteration.
constexpr int64_t kLanesMinAtoms = 16384;

static int lanes_for(const hdmd_system* s, int d, int rowkey) {
  if (s->potential == HDMD_MORSE) return 1;
  if (const int e = lpa_env()) return e;
  if (s->n < kLanesMinAtoms) return 1;
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_lanes.find({d, s->precision == HDMD_MIXED ? 1 : 0, rowkey});
  return it == g_lanes.end() ? 1 : it->second;
}

static int lpa_index(int lpa) { return lpa >= 4 ? 2 : (lpa == 2 ? 1 : 0); }
static int lpa_of_index(int k) { return 1 << k; }

// ---------------------------------------------------------------------------
// launch sequences
// ---------------------------------------------------------------------------
static inline hipStream_t S(void* st) { return reinterpret_cast<hipStream_t>(st); }

static KArgs single_args(SysDev* dev, int d) {
  KArgs a;
  a.single = dev;
  a.tab = nullptr;
  a.cls = d;
  a.part = 0;
  return a;
}

// bin -> scan -> scatter -> per-subcell sort/permute (chain_sort), then the
// list build; every kernel exits at once for systems that need no rebuild.
// The binning, placement and subcell-sort grids stride over their tiles:
// at most 1024 workgroups, so that the launches of steps without a rebuild
// (which exit at once) dispatch few of them.
static void chain_sort(const Plan& p, SysDev* dev, hipStream_t st) {
  const DKernels* K = dkernels(p.d);
  KArgs a = single_args(dev, p.d);
  const int gt = std::min(p.ntiles, 1024), gc = std::min(p.ncells, 1024);
  K->bin(a, gt, st);
  launch_scan1(a, p.nchunks, st);
  launch_scan2(a, 1, st);
  launch_scatter(a, gt, st);
  K->cellsort(p.mix, a, gc, st);
}

static void build_single(const Plan& p, SysDev* dev, hipStream_t st, int blk) {
  dkernels(p.d)->build(p.reach, p.wrap, blk, single_args(dev, p.d), p.ncells, st);
}

static void chain_single(const Plan& p, SysDev* dev, hipStream_t st, int blk) {
  chain_sort(p, dev, st);
  build_single(p, dev, st, blk);
}

// HIP events of the profiling mode, created once (with the system fence
// disabled, so that recording them neither writes back nor invalidates the
// caches) and reused by later calls.
static std::mutex g_ev_mu;
static std::vector<hipEvent_t> g_events;

static int event_pool(size_t n, std::vector<hipEvent_t>& out) {
  std::lock_guard<std::mutex> g(g_ev_mu);
  while (g_events.size() < n) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    g_events.push_back(e);
  }
  out.assign(g_events.begin(), g_events.begin() + n);
  return HDMD_OK;
}

static int read_desc(const SysDev* dev, SysDev* host, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(host, dev, sizeof(SysDev), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return HDMD_OK;
}

static int err_to_status(int32_t err, const char* where) {
  if (err & ERR_NONFINITE) return fail(HDMD_ERR_NONFINITE, std::string(where) + ": non-finite input");
  if (err & ERR_ARG) return fail(HDMD_ERR_ARG, std::string(where) + ": position outside [-3L/2, 3L/2) or diameter outside (0, sigma_max]");
  if (err & ERR_OVERFLOW) return fail(HDMD_ERR_NLIST_OVERFLOW, std::string(where) + ": Verlet row longer than max_neighbors");
  if (err & ERR_RUN_NAN) return fail(HDMD_ERR_NONFINITE, std::string(where) + ": non-finite energy during the run");
  return HDMD_OK;
}

// one int32 field of a device descriptor
static void set_i32(SysDev* dev, size_t off, int32_t v, hipStream_t st) {
  launch_fill_i32(reinterpret_cast<int32_t*>(reinterpret_cast<char*>(dev) + off), 1, v, st);
}

// Writes the descriptor of plan p and loads the caller's arrays into ws.
static void load_system(const hdmd_system* sys, const Plan& p, const double* pos,
                        const double* diam, const double* vel, void* ws, hipStream_t st) {
  SysDev* dev = at<SysDev>(ws, p.off_desc);
  SysDev h = make_desc(sys, p, ws);
  launch_setdesc(dev, h, st);
  launch_fill_i32(h.cell_count, p.ncells, 0, st);
  // displacements start at zero (both buffers; the first build permutes them)
  launch_fill_i32(reinterpret_cast<int32_t*>(h.disp[0]), (int64_t)p.npad * p.d * 2, 0, st);
  launch_fill_i32(reinterpret_cast<int32_t*>(h.disp[1]), (int64_t)p.npad * p.d * 2, 0, st);
  dkernels(p.d)->load(p.mix, dev, p.ntiles, st, pos, diam, vel);
}

// The autotuner, on the first build of a key: for each grid the system may
// take (an autotuned system whose half-size grid applies: both; otherwise its
// own), loads the system, times the binning and subcell sort, then each
// list-build variant (every variant gives the same list), and records the
// best variant of each grid timed and, for an autotuned system, the grid of
// the lower sum.  Half-size subcells are timed with the candidate-lane
// variants only: the home-lane build stages each of the 5^d linked subcells,
// most of them nearly empty.
static int tune_build(const hdmd_system* sys, const Plan& pf, const double* pos,
                      const double* diam, const double* vel, void* ws, hipStream_t st) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto elapsed = [&](float* ms) -> int {
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(ms, e0, e1));
    return HDMD_OK;
  };
  Tuned t;
  float total[3] = {0.f, 1e30f, 1e30f};
  const int r0 = pf.nh_auto ? 1 : pf.reach, r1 = pf.nh_auto ? 2 : pf.reach;
  for (int reach = r0; reach <= r1; reach++) {
    Plan p = pf;
    if (reach == 2) {
      // the same layout with the half-size grid
      p.reach = 2;
      p.ncell = pf.nh_auto ? pf.nh_auto : pf.ncell;
      p.radix = 5;
      p.ncells = (int)ipow(p.ncell, p.d);
      p.nstencil = (int)ipow(5, p.d);
      p.nchunks = (p.ncells + kChunk - 1) / kChunk;
      p.wrap = false;
    } else {
      p.reach = 1;
      p.ncell = choose_ncell(*sys, pf.rlmax);
      p.radix = p.ncell < 3 ? p.ncell : 3;
      p.ncells = (int)ipow(p.ncell, p.d);
      p.nstencil = (int)ipow(p.radix, p.d);
      p.nchunks = (p.ncells + kChunk - 1) / kChunk;
      p.wrap = p.ncell <= 2;
    }
    SysDev* dev = at<SysDev>(ws, p.off_desc);
    float sort_ms = 0.f;
    for (int rep = 0; rep < 2; rep++) {  // the second load and sort are timed
      load_system(sys, p, pos, diam, vel, ws, st);
      HIPCHK(hipEventRecord(e0, st));
      chain_sort(p, dev, st);
      HIPCHK(hipEventRecord(e1, st));
      int rc = elapsed(&sort_ms);
      if (rc) return rc;
    }
    float best = 1e30f;
    for (int cand : {1, 2, 4, 1 | kBuildMF, 2 | kBuildMF, 4 | kBuildMF, 8, 16, 64, 128, 256}) {
      if (reach == 2 && (cand & ~kBuildMF) > 4) break;
      if (!p.wrap && (cand == 8 || cand == 16)) continue;  // 8 and 16 waves: crowded subcells only
      if (p.wrap && (cand & kBuildMF)) continue;  // matrix-core tests: n_cell >= 3 only
      build_single(p, dev, st, cand);  // warm-up
      HIPCHK(hipEventRecord(e0, st));
      build_single(p, dev, st, cand);
      HIPCHK(hipEventRecord(e1, st));
      float ms = 0;
      int rc = elapsed(&ms);
      if (rc) return rc;
      if (ms < best) {
        best = ms;
        t.blk[reach] = cand;
      }
      // the half grid's other variants only while it stays within twice the
      // full grid's time (they are slower than its one-wave build)
      if (reach == 2 && r0 == 1 && sort_ms + best > 2.f * total[1]) break;
    }
    total[reach] = sort_ms + best;
  }
  HIPCHK(hipEventDestroy(e0));
  HIPCHK(hipEventDestroy(e1));
  std::lock_guard<std::mutex> g(g_tune_mu);
  Tuned& e = g_tune[std::make_tuple(pf.d, pf.key_wrap, pf.key_occ)];
  for (int r = r0; r <= r1; r++)
    if (!e.blk[r]) e.blk[r] = t.blk[r];
  // the grid of an autotuned system: decided once per key (one whose half
  // grid does not apply takes the full grid)
  if (!e.reach && (pf.nh_auto || pf.reach == 1) && sys->subcells == HDMD_SUBCELLS_AUTO)
    e.reach = total[2] < total[1] ? 2 : 1;
  return HDMD_OK;
}

// Loads a system into ws and builds its list (the descriptor ends in
// MODE_STATIC, running, with current buffers holding the sorted state).  A
// system whose key the autotuner has not met yet is tuned first, and p
// becomes the plan of the grid it chose (the layout stays the same).
static int init_system(const hdmd_system* sys, Plan& p, const double* pos,
                       const double* diam, const double* vel, void* ws, size_t ws_bytes,
                       hipStream_t st, int* blk_out, bool allow_tune = true) {
  if (!pos || !diam || !ws) return fail(HDMD_ERR_ARG, "null device pointer");
  if (ws_bytes < p.bytes)
    return fail(HDMD_ERR_WORKSPACE, "workspace too small: need " + std::to_string(p.bytes) + " bytes");
  bool known = false;
  int blk = lookup_blk(p, &known);
  if (!known && tuning_enabled() && allow_tune) {
    int rc = tune_build(sys, p, pos, diam, vel, ws, st);
    if (rc) return rc;
    Plan q;
    rc = make_plan(sys, q);
    if (rc) return rc;
    p = q;
    blk = lookup_blk(p, &known);
  }
  load_system(sys, p, pos, diam, vel, ws, st);
  SysDev* dev = at<SysDev>(ws, p.off_desc);
  chain_single(p, dev, st, blk);
  launch_finalize(single_args(dev, p.d), 1, st);
  HIPCHK(hipGetLastError());
  if (!p.morse && !lpa_env() && p.n >= kLanesMinAtoms && tuning_enabled() && allow_tune) {
    const int mix = p.mix ? 1 : 0;
    bool timed = false;
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      timed = g_lanes.count({p.d, mix, p.row_key}) > 0;
    }
    if (!timed) {
      // the force kernel with 1, 2 and 4 lanes per atom on the list just built;
      // more lanes only where one lane takes at least 20 us and they save 10 %
      // (below that, launch overheads and the batches' one all-class launch
      // for one-lane systems count for more)
      hipEvent_t e0, e1;
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      const DKernels* K = dkernels(p.d);
      KArgs a = single_args(dev, p.d);
      float best = 1e30f, one = 0.f;
      int best_lpa = 1;
      for (int cand : {1, 2, 4}) {
        set_i32(dev, offsetof(SysDev, lpa), cand, st);
        K->force(p.mix, cand, p.morse, a, p.ntiles, 0, st);  // warm-up
        HIPCHK(hipEventRecord(e0, st));
        K->force(p.mix, cand, p.morse, a, p.ntiles, 0, st);
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        if (cand == 1) one = ms;
        if (ms < best) {
          best = ms;
          best_lpa = cand;
        }
      }
      HIPCHK(hipEventDestroy(e0));
      HIPCHK(hipEventDestroy(e1));
      if (one < 0.020f || best > 0.9f * one) best_lpa = 1;
      {
        std::lock_guard<std::mutex> g(g_tune_mu);
        p.lpa = g_lanes.emplace(std::make_tuple(p.d, mix, p.row_key), best_lpa).first->second;
      }
      set_i32(dev, offsetof(SysDev, lpa), p.lpa, st);
    }
  }
  if (blk_out) *blk_out = blk;
  return HDMD_OK;
}

// ---------------------------------------------------------------------------
// graph cache (chunks of steps / iterations captured once per workspace)
// ---------------------------------------------------------------------------
// A captured chunk is valid for every system with the same key: the key holds
// each input that selects a kernel or a grid (the workspace address fixes the
// device descriptor the kernels read).
struct GraphKey {
  void* ws;
  int kind, chunk, d, mix, morse, wrap, blk, ntiles, ncells, nchunks;
  bool operator<(const GraphKey& o) const {
    return std::tie(ws, kind, chunk, d, mix, morse, wrap, blk, ntiles, ncells, nchunks) <
           std::tie(o.ws, o.kind, o.chunk, o.d, o.mix, o.morse, o.wrap, o.blk, o.ntiles, o.ncells,
                    o.nchunks);
  }
};
static std::mutex g_graph_mu;
static std::map<GraphKey, hipGraphExec_t> g_graphs;
static hipStream_t g_capture_stream = nullptr;

static bool graphs_enabled() {
  const char* e = std::getenv("HDMD_GRAPH");
  return !(e && e[0] == '0');
}

typedef void (*EnqueueFn)(const Plan& p, SysDev* dev, hipStream_t st, int blk);

static void enqueue_md_step(const Plan& p, SysDev* dev, hipStream_t st, int blk) {
  const DKernels* K = dkernels(p.d);
  KArgs a = single_args(dev, p.d);
  K->step(p.mix, p.lpa, p.morse, a, p.ntiles, st);
  chain_single(p, dev, st, blk);
  launch_finalize(a, 1, st);
}

static void enqueue_fire_iter(const Plan& p, SysDev* dev, hipStream_t st, int blk) {
  const DKernels* K = dkernels(p.d);
  KArgs a = single_args(dev, p.d);
  launch_fire_ctrl(a, 1, st);
  K->fire_update(p.mix, a, p.ntiles, st);
  chain_single(p, dev, st, blk);
  launch_finalize(a, 1, st);
  K->force(p.mix, p.lpa, p.morse, a, p.ntiles, 1, st);
}

static int run_chunk(void* ws, int kind, EnqueueFn fn, int chunk, const Plan& p, SysDev* dev,
                     hipStream_t st, int blk) {
  if (!graphs_enabled()) {
    for (int k = 0; k < chunk; k++) fn(p, dev, st, blk);
    HIPCHK(hipGetLastError());
    return HDMD_OK;
  }
  GraphKey key{ws,      kind,  chunk, p.d,     (int)p.mix + 2 * p.lpa, (int)p.morse, (int)p.wrap + 2 * p.reach,
               blk,     p.ntiles, p.ncells, p.nchunks};
  hipGraphExec_t exec = nullptr;
  {
    std::lock_guard<std::mutex> g(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) exec = it->second;
    if (!exec) {
      if (!g_capture_stream) HIPCHK(hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking));
      HIPCHK(hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < chunk; k++) fn(p, dev, g_capture_stream, blk);
      hipGraph_t graph;
      HIPCHK(hipStreamEndCapture(g_capture_stream, &graph));
      HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      HIPCHK(hipGraphDestroy(graph));
      g_graphs[key] = exec;
    }
  }
  HIPCHK(hipGraphLaunch(exec, st));
  return HDMD_OK;
}


}  // namespace hdmd

using namespace hdmd;

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* hdmd_last_error(void) { return g_err.c_str(); }

void hdmd_fire_defaults(hdmd_fire_params* p, double dt0, double f_tol, int64_t max_iter) {
  p->dt0 = dt0;
  p->dt_max = 10.0 * dt0;
  p->dt_min = 0.02 * dt0;
  p->f_inc = 1.1;
  p->f_dec = 0.5;
  p->alpha0 = 0.25;
  p->f_alpha = 0.99;
  p->n_delay = 20;
  p->n_neg_max = 2000;
  p->max_iter = max_iter;
  p->initial_delay = 1;
  p->f_tol = f_tol;
  p->e_tol = 0.0;
}

size_t hdmd_workspace_bytes(const hdmd_system* sys) {
  Plan p;
  if (make_plan(sys, p) != HDMD_OK) return 0;
  return p.bytes;
}

int hdmd_cells_per_axis(const hdmd_system* sys) {
  Plan p;
  int rc = make_plan(sys, p);
  if (rc) return rc;
  return sys->subcells == HDMD_SUBCELLS_HALF ? p.ncell : choose_ncell(*sys, p.rlmax);
}

int hdmd_build_config(const hdmd_system* sys, int32_t* reach, int32_t* cells_per_axis,
                      int32_t* variant, int32_t* lanes_per_atom) {
  Plan p;
  int rc = make_plan(sys, p);
  if (rc) return rc;
  bool known = false;
  const int blk = lookup_blk(p, &known);
  if (reach) *reach = p.reach;
  if (cells_per_axis) *cells_per_axis = p.ncell;
  if (variant) *variant = blk;
  if (lanes_per_atom) *lanes_per_atom = p.lpa;
  return known ? 1 : 0;
}

int hdmd_build_nlist(const hdmd_system* sys, const double* pos, const double* diam, void* ws,
                     size_t ws_bytes, int32_t* required_width, void* stream) {
  Plan p;
  int rc = make_plan(sys, p);
  if (rc) return rc;
  hipStream_t st = S(stream);
  rc = init_system(sys, p, pos, diam, nullptr, ws, ws_bytes, st, nullptr);
  if (rc) return rc;
  SysDev h;
  rc = read_desc(at<SysDev>(ws, p.off_desc), &h, st);
  if (rc) return rc;
  if (required_width) *required_width = h.max_row;
  return err_to_status(h.err, "hdmd_build_nlist");
}

int hdmd_nlist_export(const hdmd_system* sys, void* ws, int64_t* row_ptr, int32_t* cols,
                      int64_t cols_cap, int64_t* nnz, void* stream) {
  Plan p;
  int rc = make_plan(sys, p);
  if (rc) return rc;
  if (!ws || !row_ptr || !nnz) return fail(HDMD_ERR_ARG, "null pointer");
  hipStream_t st = S(stream);
  SysDev* dev = at<SysDev>(ws, p.off_desc);
  SysDev h;
  rc = read_desc(dev, &h, st);
  if (rc) return rc;
  if (h.n != p.n || h.d != p.d) return fail(HDMD_ERR_STATE, "workspace holds another system");
  launch_export(dev, p.n, row_ptr, cols, st, 0);
  launch_export(dev, p.n, row_ptr, cols, st, 1);
  int64_t total = 0;
  HIPCHK(hipMemcpyAsync(&total, row_ptr + p.n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *nnz = total;
  if (total > cols_cap || (total > 0 && !cols))
    return fail(HDMD_ERR_WORKSPACE, "cols_cap smaller than the entry count");
  launch_export(dev, p.n, row_ptr, cols, st, 2);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return HDMD_OK;
}

}  // extern "C"

namespace hdmd {

static int forces_run(const hdmd_system* sys, Plan& p, const double* pos, const double* diam,
                      void* ws, size_t ws_bytes, double* force, double* energy, void* stream,
                      bool allow_tune) {
  if (!force || !energy) return fail(HDMD_ERR_ARG, "null output pointer");
  hipStream_t st = S(stream);
  int rc = init_system(sys, p, pos, diam, nullptr, ws, ws_bytes, st, nullptr, allow_tune);
  if (rc) return rc;
  SysDev* dev = at<SysDev>(ws, p.off_desc);
  const DKernels* K = dkernels(p.d);
  K->force(p.mix, p.lpa, p.morse, single_args(dev, p.d), p.ntiles, 0, st);
  launch_reduce_pe(dev, energy, st);
  K->unload(p.mix, dev, p.ntiles, st, nullptr, nullptr, force);
  HIPCHK(hipGetLastError());
  SysDev h;
  rc = read_desc(dev, &h, st);
  if (rc) return rc;
  return err_to_status(h.err, "hdmd_forces");
}


// Device memory of hdmd_forces_noalloc: a scratch array the library holds on
// every device it runs on (until the process ends) in place of a caller's
// workspace.  Host code never passes the array's name to a kernel or a copy
// (on the host it is only a stand-in for the symbol): it uses the device
// address hipGetSymbolAddress returns, taken once per device with that
// device current.
constexpr size_t kNoAllocBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {nullptr};

static int scratch_ptr(void** out) {
  int devid = -1;
  HIPCHK(hipGetDevice(&devid));
  if (devid < 0 || devid >= kMaxDevices) return fail(HDMD_ERR_HIP, "device id out of range");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[devid]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(HDMD_ERR_HIP, "no device address for the scratch array");
    g_scratch_ptr[devid] = ptr;
  }
  *out = g_scratch_ptr[devid];
  return HDMD_OK;
}

}  // namespace hdmd

extern "C" {

int hdmd_forces(const hdmd_system* sys, const double* pos, const double* diam, void* ws,
                size_t ws_bytes, double* force, double* energy, void* stream) {
  Plan p;
  int rc = make_plan(sys, p);
  if (rc) return rc;
  return forces_run(sys, p, pos, diam, ws, ws_bytes, force, energy, stream, true);
}

size_t hdmd_forces_noalloc_bytes(void) { return kNoAllocBytes; }

int hdmd_forces_noalloc(const hdmd_system* sys, const double* pos, const double* diam,
                        double* force, double* energy, void* stream) {
  Plan p;
  int rc = make_plan(sys, p);
  if (rc) return rc;
  if (p.bytes > kNoAllocBytes)
    return fail(HDMD_ERR_WORKSPACE, "hdmd_forces_noalloc: the system needs " +
                                        std::to_string(p.bytes) + " bytes of workspace, more "
                                        "than the library's scratch array of " +
                                        std::to_string(kNoAllocBytes));
  void* ws = nullptr;
  rc = scratch_ptr(&ws);
  if (rc) return rc;
  // the build variant the autotuner chose for this key, or the default: no
  // timing runs (they would create events)
  return forces_run(sys, p, pos, diam, ws, kNoAllocBytes, force, energy, stream, false);
}

static int step_chunk_len() {
  const char* e = std::getenv("HDMD_CHUNK");
  int c = e ? std::atoi(e) : 50;
  return c < 1 ? 1 : c;
}

}  // extern "C"

namespace hdmd {

// Whether the descriptor h (read from ws) is a completed MD run of exactly
// this system (same plan and parameters, laid out in this workspace), as the
// last hdmd_step / hdmd_step_resume on ws left it.
static bool holds_run_of(const SysDev& h, const hdmd_system* sys, const Plan& p, void* ws) {
  return h.d == p.d && h.n == p.n && h.npad == p.npad && h.ncell == p.ncell && h.reach == p.reach &&
         h.lpa == p.lpa &&
         h.width == p.width && h.precision == sys->precision && h.potential == sys->potential &&
         h.L == sys->box_l && h.cutoff == sys->cutoff && h.skin == sys->skin &&
         h.eps == sys->epsilon && h.sigma_max == sys->sigma_max &&
         (sys->potential != HDMD_MORSE || h.morse_a == sys->morse_a) && h.mode == MODE_MD &&
         h.status == SLOT_DONE && h.err == 0 && h.step > 0 &&
         h.x[0] == at<double>(ws, p.off_x[0]) && h.nl == at<int32_t>(ws, p.off_nl);
}

// The MD run behind hdmd_step and hdmd_step_resume: a fresh call loads the
// caller's state and builds the list; a resumed one checks on the device that
// the caller's arrays are the state ws holds and continues from it.
static int md_run(const hdmd_system* sys, double* pos, double* vel, const double* diam, void* ws,
                  size_t ws_bytes, int64_t nsteps, double dt, int64_t thermo_every, double* thermo,
                  hdmd_step_stats* stats, void* stream, bool resume) {
  Plan p;
  int rc = make_plan(sys, p);
  if (rc) return rc;
  if (!vel || !pos || !diam || !ws) return fail(HDMD_ERR_ARG, "null pointer");
  if (nsteps < 0 || !(dt > 0) || !std::isfinite(dt)) return fail(HDMD_ERR_ARG, "need nsteps >= 0 and dt > 0");
  if (sys->thermostat_tau > 0 && sys->thermostat_tau < dt)
    return fail(HDMD_ERR_ARG, "thermostat_tau must be >= dt");
  hipStream_t st = S(stream);
  SysDev* dev = at<SysDev>(ws, p.off_desc);
  SysDev h;
  int blk = 0;
  const DKernels* K = dkernels(p.d);
  if (resume) {
    if (ws_bytes < p.bytes)
      return fail(HDMD_ERR_WORKSPACE, "workspace too small: need " + std::to_string(p.bytes) + " bytes");
    rc = read_desc(dev, &h, st);
    if (rc) return rc;
    if (!holds_run_of(h, sys, p, ws))
      return fail(HDMD_ERR_STATE, "hdmd_step_resume: the workspace holds no completed run of this system");
    set_i32(dev, offsetof(SysDev, differ), 0, st);
    K->same_state(p.mix, dev, p.ntiles, st, pos, vel, diam);
    HIPCHK(hipGetLastError());
    rc = read_desc(dev, &h, st);
    if (rc) return rc;
    if (h.differ)
      return fail(HDMD_ERR_STATE,
                  "hdmd_step_resume: pos, vel or diam differ from the state the last call returned");
    K->disp_restart(dev, p.ntiles, st);
    bool known = false;
    blk = lookup_blk(p, &known);
    h.tau_t = sys->thermostat_tau;
    h.temp_t = sys->target_temp;
    h.vscale = 1.0;
    h.force_rebuild = 0;
    h.status = SLOT_RUNNING;
  } else {
    rc = init_system(sys, p, pos, diam, vel, ws, ws_bytes, st, &blk);
    if (rc) return rc;
    rc = read_desc(dev, &h, st);
    if (rc) return rc;
    rc = err_to_status(h.err, "hdmd_step");
    if (rc) {
      if (stats) stats->max_row = h.max_row;
      return rc;
    }
  }
  const int64_t builds0 = h.builds;
  // switch the descriptor to MD mode
  h.mode = MODE_MD;
  h.dt = dt;
  h.nsteps = nsteps;
  h.thermo = thermo;
  h.thermo_every = thermo_every > 0 ? thermo_every : 0;
  h.step = 0;
  launch_setdesc(dev, h, st);
  // steps 0..nsteps (nsteps+1 force evaluations), in captured chunks
  const char* prof_env = std::getenv("HDMD_PROFILE");
  const bool profile = prof_env && prof_env[0] == '1';
  std::vector<hipEvent_t> ev;
  if (profile) {
    // one launch at a time (the launches of the captured chunks), fused-step
    // and list-build kernels bracketed by events
    KArgs a = single_args(dev, p.d);
    rc = event_pool(4 * (size_t)(nsteps + 1), ev);
    if (rc) return rc;
    for (int64_t k = 0; k <= nsteps; k++) {
      HIPCHK(hipEventRecord(ev[4 * k], st));
      K->step(p.mix, p.lpa, p.morse, a, p.ntiles, st);
      HIPCHK(hipEventRecord(ev[4 * k + 1], st));
      chain_sort(p, dev, st);
      HIPCHK(hipEventRecord(ev[4 * k + 2], st));
      build_single(p, dev, st, blk);
      HIPCHK(hipEventRecord(ev[4 * k + 3], st));
      launch_finalize(a, 1, st);
    }
    HIPCHK(hipGetLastError());
  } else {
    const int chunk = step_chunk_len();
    int64_t todo = nsteps + 1;
    while (todo > 0) {
      int c = (int)std::min<int64_t>(chunk, todo);
      if (c < chunk && graphs_enabled()) c = chunk;  // surplus steps are no-ops once done
      rc = run_chunk(ws, 1, enqueue_md_step, c, p, dev, st, blk);
      if (rc) return rc;
      todo -= c;
    }
  }
  rc = read_desc(dev, &h, st);
  if (rc) return rc;
  if (stats) {
    stats->steps_done = h.step > 0 ? h.step - 1 : 0;
    stats->builds = h.builds - builds0;
    stats->ke = h.ke;
    stats->pe = h.pe;
    stats->max_row = h.max_row;
    stats->step_kernel_ms = 0;
    stats->step_kernels = 0;
    stats->build_kernel_ms = 0;
    stats->build_kernels = 0;
    if (profile) {
      std::vector<float> bt;
      for (int64_t k = 0; k <= nsteps; k++) {
        float a = 0, b = 0;
        HIPCHK(hipEventElapsedTime(&a, ev[4 * k], ev[4 * k + 1]));
        HIPCHK(hipEventElapsedTime(&b, ev[4 * k + 2], ev[4 * k + 3]));
        stats->step_kernel_ms += a;
        stats->step_kernels++;
        bt.push_back(b);
      }
      // the launches that built are the longest ones (the others exit at once)
      std::sort(bt.begin(), bt.end());
      const int64_t nb = std::min<int64_t>(stats->builds, (int64_t)bt.size());
      for (int64_t k = 0; k < nb; k++) stats->build_kernel_ms += bt[bt.size() - 1 - k];
      stats->build_kernels = nb;
    }
  }
  rc = err_to_status(h.err, "hdmd_step");
  if (rc) return rc;  // caller arrays untouched
  K->unload(p.mix, dev, p.ntiles, st, pos, vel, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return HDMD_OK;
}

}  // namespace hdmd

extern "C" {

int hdmd_step(const hdmd_system* sys, double* pos, double* vel, const double* diam, void* ws,
              size_t ws_bytes, int64_t nsteps, double dt, int64_t thermo_every, double* thermo,
              hdmd_step_stats* stats, void* stream) {
  return md_run(sys, pos, vel, diam, ws, ws_bytes, nsteps, dt, thermo_every, thermo, stats, stream,
                false);
}

int hdmd_step_resume(const hdmd_system* sys, double* pos, double* vel, const double* diam,
                     void* ws, size_t ws_bytes, int64_t nsteps, double dt, int64_t thermo_every,
                     double* thermo, hdmd_step_stats* stats, void* stream) {
  return md_run(sys, pos, vel, diam, ws, ws_bytes, nsteps, dt, thermo_every, thermo, stats, stream,
                true);
}

int hdmd_van_hove(const hdmd_system* sys, void* ws, size_t ws_bytes, int32_t nbins,
                  double bin_width, int64_t* hist, double* disp, void* stream) {
  Plan p;
  int rc = make_plan(sys, p);
  if (rc) return rc;
  if (!ws) return fail(HDMD_ERR_ARG, "null workspace");
  if (ws_bytes < p.bytes) return fail(HDMD_ERR_WORKSPACE, "workspace too small");
  if (!hist && !disp) return fail(HDMD_ERR_ARG, "neither hist nor disp given");
  if (hist && (nbins < 1 || !(bin_width > 0) || !std::isfinite(bin_width)))
    return fail(HDMD_ERR_ARG, "need nbins >= 1 and bin_width > 0");
  hipStream_t st = S(stream);
  SysDev* dev = at<SysDev>(ws, p.off_desc);
  SysDev h;
  rc = read_desc(dev, &h, st);
  if (rc) return rc;
  if (h.n != p.n || h.d != p.d) return fail(HDMD_ERR_STATE, "workspace holds another system");
  if (h.mode != MODE_MD || h.err != 0)
    return fail(HDMD_ERR_STATE, "the workspace holds no completed hdmd_step run");
  if (hist) launch_fill_i32(reinterpret_cast<int32_t*>(hist), 2 * ((int64_t)nbins + 1), 0, st);
  dkernels(p.d)->vanhove(dev, p.ntiles, st, nbins, bin_width,
                         reinterpret_cast<unsigned long long*>(hist), disp);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return HDMD_OK;
}

}  // extern "C"

namespace hdmd {

// SWAP Monte Carlo with its scratch at `scr` (kSwapScratchBytes of device
// memory): one rounds of a batch each (dE of every attempt, then the
// settlement in order), enqueued in runs of as many rounds as the attempts
// left need at least, the counters read back after each run.
static int swap_run(const hdmd_system* sys, const double* pos, double* diam, void* ws,
                    size_t ws_bytes, int64_t n_att, const int32_t* pairs, const double* u,
                    double temperature, int32_t* accepted, int64_t* n_accepted, void* stream,
                    void* scr) {
  Plan p;
  int rc = make_plan(sys, p);
  if (rc) return rc;
  if (!pos || !diam || !n_accepted) return fail(HDMD_ERR_ARG, "null pointer");
  if (n_att < 0 || n_att > INT32_MAX) return fail(HDMD_ERR_ARG, "n_att out of range");
  if (n_att > 0 && (!pairs || !u)) return fail(HDMD_ERR_ARG, "null pairs or uniforms");
  if (!(temperature > 0) || !std::isfinite(temperature))
    return fail(HDMD_ERR_ARG, "temperature must be > 0");
  hipStream_t st = S(stream);
  SwapScratch w = swap_scratch(scr);
  long long hc[4] = {0, 0, 0, 0};
  // every attempt names two atoms of the system (checked before any change)
  launch_fill_i32(reinterpret_cast<int32_t*>(w.ctl), 8, 0, st);
  launch_swap_init(n_att, pairs, p.n, w.ctl, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(hc, w.ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hc[3]) return fail(HDMD_ERR_ARG, "swap pair names an atom outside [0, n)");
  rc = init_system(sys, p, pos, diam, nullptr, ws, ws_bytes, st, nullptr);
  if (rc) return rc;
  SysDev* dev = at<SysDev>(ws, p.off_desc);
  SysDev h;
  rc = read_desc(dev, &h, st);
  if (rc) return rc;
  rc = err_to_status(h.err, "hdmd_swap");
  if (rc) return rc;
  *n_accepted = 0;
  if (n_att == 0) return HDMD_OK;
  int32_t* slot_of = at<int32_t>(ws, p.off_src);  // free outside a rebuild
  launch_slot_of(dev, p.n, slot_of, st);
  const DKernels* K = dkernels(p.d);
  int64_t left = n_att, rounds = 0;
  int cur = 0;
  while (left > 0) {
    // the first attempt of a batch always settles, so every round makes progress
    const int64_t run = std::max<int64_t>(1, (left + kSwapBatch - 1) / kSwapBatch);
    if (rounds + run > n_att + 1) return fail(HDMD_ERR_STATE, "hdmd_swap: no progress");
    for (int64_t r = 0; r < run; r++) {
      K->swap_de(dev, st, w.ctl, w.off[cur], n_att, pairs, slot_of, w.de, w.conf);
      K->swap_settle(dev, st, w.ctl, w.off[cur], w.off[cur ^ 1], n_att, pairs, u, temperature,
                     slot_of, w.de, w.conf, accepted, diam);
      cur ^= 1;
    }
    rounds += run;
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hc, w.ctl, sizeof(hc), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    left = hc[0] + (n_att - hc[2]);
  }
  *n_accepted = hc[1];
  return HDMD_OK;
}

}  // namespace hdmd

extern "C" {

int hdmd_swap(const hdmd_system* sys, const double* pos, double* diam, void* ws, size_t ws_bytes,
              int64_t n_att, const int32_t* pairs, const double* u, double temperature,
              int32_t* accepted, int64_t* n_accepted, void* stream) {
  Plan p;
  int rc = make_plan(sys, p);
  if (rc) return rc;
  if (!ws) return fail(HDMD_ERR_ARG, "null workspace");
  if (ws_bytes < p.bytes)
    return fail(HDMD_ERR_WORKSPACE, "workspace too small: need " + std::to_string(p.bytes) + " bytes");
  return swap_run(sys, pos, diam, ws, ws_bytes, n_att, pairs, u, temperature, accepted, n_accepted,
                  stream, at<char>(ws, p.off_swap));
}

static void set_fire(SysDev& h, const hdmd_fire_params* fp) {
  h.mode = MODE_FIRE;
  h.fc.dt0 = fp->dt0;
  h.fc.dtmax = fp->dt_max;
  h.fc.dtmin = fp->dt_min;
  h.fc.finc = fp->f_inc;
  h.fc.fdec = fp->f_dec;
  h.fc.alpha0 = fp->alpha0;
  h.fc.falpha = fp->f_alpha;
  h.fc.ftol = fp->f_tol;
  h.fc.etol = fp->e_tol;
  h.fc.ndelay = fp->n_delay;
  h.fc.nnegmax = fp->n_neg_max;
  h.fc.maxiter = fp->max_iter;
  h.fc.initdelay = fp->initial_delay;
  h.fdt = fp->dt0;
  h.falpha = fp->alpha0;
  h.npos = 0;
  h.nneg = 0;
  h.iters = 0;
  h.fstatus = 0;
}

static int check_fire_params(const hdmd_fire_params* fp) {
  if (!fp) return fail(HDMD_ERR_ARG, "null FIRE parameters");
  if (!(fp->dt0 > 0) || !(fp->dt_max >= fp->dt0) || !(fp->dt_min > 0) || !(fp->f_tol >= 0) ||
      fp->max_iter < 0)
    return fail(HDMD_ERR_ARG, "bad FIRE parameters");
  return HDMD_OK;
}

// load + build, switch to FIRE mode, first forces (velocities start at zero)
static int fire_start(const hdmd_system* sys, Plan& p, const double* pos, const double* diam,
                      void* ws, size_t ws_bytes, const hdmd_fire_params* fp, hipStream_t st,
                      int* blk) {
  int rc = check_fire_params(fp);
  if (rc) return rc;
  rc = init_system(sys, p, pos, diam, nullptr, ws, ws_bytes, st, blk);
  if (rc) return rc;
  SysDev* dev = at<SysDev>(ws, p.off_desc);
  SysDev h;
  rc = read_desc(dev, &h, st);
  if (rc) return rc;
  rc = err_to_status(h.err, "FIRE setup");
  if (rc) return rc;
  set_fire(h, fp);
  launch_setdesc(dev, h, st);
  dkernels(p.d)->force(p.mix, p.lpa, p.morse, single_args(dev, p.d), p.ntiles, 1, st);
  HIPCHK(hipGetLastError());
  return HDMD_OK;
}

static void fill_result(const SysDev& h, int64_t builds0, hdmd_fire_result* r) {
  r->iterations = h.iters;
  r->builds = h.builds - builds0;
  r->fmax = h.fmax;
  r->energy = h.pe;
  r->status = h.fstatus;
  r->pad = 0;
}

int hdmd_fire_minimize(const hdmd_system* sys, double* pos, const double* diam, void* ws,
                       size_t ws_bytes, const hdmd_fire_params* params, hdmd_fire_result* result,
                       void* stream) {
  Plan p;
  int rc = make_plan(sys, p);
  if (rc) return rc;
  hipStream_t st = S(stream);
  int blk = 0;
  rc = fire_start(sys, p, pos, diam, ws, ws_bytes, params, st, &blk);
  if (rc) return rc;
  SysDev* dev = at<SysDev>(ws, p.off_desc);
  const int chunk = step_chunk_len();
  SysDev h;
  for (;;) {
    rc = run_chunk(ws, 2, enqueue_fire_iter, chunk, p, dev, st, blk);
    if (rc) return rc;
    rc = read_desc(dev, &h, st);
    if (rc) return rc;
    if (h.status != SLOT_RUNNING) break;
  }
  if (result) fill_result(h, 0, result);
  rc = err_to_status(h.err, "hdmd_fire_minimize");
  if (rc) return rc;
  dkernels(p.d)->unload(p.mix, dev, p.ntiles, st, pos, nullptr, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return h.fstatus == 0 ? HDMD_OK : HDMD_NOT_CONVERGED;
}

}  // extern "C"

// ===========================================================================
// batches of uneven replicas
// ===========================================================================
namespace hdmd {

struct SlotInfo {
  bool used = false;
  Plan p;
  SysDev* dev = nullptr;
  void* ws = nullptr;
  int mode = 0;
  int blk = 64;
};

struct HostBatch {
  int max_slots = 0;
  int64_t cap_atom = 0, cap_cell = 0, cap_chunk = 0;
  Table* dtab = nullptr;
  int2* d_atom = nullptr;
  int2* d_cell = nullptr;
  int2* d_cell_all = nullptr;  // every class: all n_cell >= 3 subcells, then all wrap ones
  int2* d_chunk = nullptr;
  int32_t* d_syslist = nullptr;
  int32_t* d_state = nullptr;
  int64_t* d_iters = nullptr;
  std::vector<SlotInfo> slots;
  bool dirty = true;
  // current composition
  int n_atom[kMaxD + 1] = {0}, n_cell[kMaxD + 1] = {0}, n_nowrap[kMaxD + 1] = {0};
  int n_chunk = 0, n_sys = 0, blk[kMaxD + 1] = {0};  // wrap-variant build tile per d
  int n_atom_all = 0, n_cell_all = 0, n_nowrap_all = 0;
  bool has_fire = false, has_md = false, has_wrap[kMaxD + 1] = {false},
       has_nowrap[kMaxD + 1] = {false}, mix[kMaxD + 1] = {false},
       has_half[kMaxD + 1] = {false};  // systems on half-size subcells
  // kernel kinds present per class, bit (mix | 2 morse | 4 lanes index): MD
  // systems, FIRE systems (lanes index 0, 1, 2: 1, 2, 4 lanes per atom)
  int kinds_md[kMaxD + 1] = {0}, kinds_fire[kMaxD + 1] = {0};
  std::map<std::vector<int>, hipGraphExec_t> graphs;
};

static std::mutex g_batch_mu;
static std::unordered_map<void*, HostBatch*> g_batches;

struct BatchLayout {
  size_t off_tab, off_atom, off_cell, off_cell_all, off_chunk, off_sys, off_state, off_iters, bytes;
};

static BatchLayout batch_layout(int max_slots, int64_t cap_atom, int64_t cap_cell,
                                int64_t cap_chunk) {
  BatchLayout L;
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t r = o;
    o = align256(o + b);
    return r;
  };
  L.off_tab = take(sizeof(Table));
  L.off_atom = take((size_t)cap_atom * sizeof(int2));
  L.off_cell = take((size_t)cap_cell * sizeof(int2));
  L.off_cell_all = take((size_t)cap_cell * sizeof(int2));
  L.off_chunk = take((size_t)cap_chunk * sizeof(int2));
  L.off_sys = take((size_t)max_slots * 4);
  L.off_state = take((size_t)max_slots * 4);
  L.off_iters = take((size_t)max_slots * 8);
  L.bytes = o;
  return L;
}

static void caps(int max_slots, int64_t max_atoms, int64_t max_cells, int64_t& ca, int64_t& cc,
                 int64_t& ch) {
  ca = max_atoms / kTile + max_slots;
  cc = max_cells + max_slots;
  ch = max_cells / kChunk + max_slots;
}

static HostBatch* find_batch(void* table_ws) {
  std::lock_guard<std::mutex> g(g_batch_mu);
  auto it = g_batches.find(table_ws);
  return it == g_batches.end() ? nullptr : it->second;
}

// Rebuilds and uploads the tile tables for the current set of slots.
static int upload_tables(HostBatch* B, hipStream_t st) {
  std::vector<int2> atom, cell, chunk;
  std::vector<int32_t> sys;
  Table t;
  std::memset(&t, 0, sizeof(t));
  t.max_slots = B->max_slots;
  std::memset(B->n_atom, 0, sizeof(B->n_atom));
  std::memset(B->n_cell, 0, sizeof(B->n_cell));
  std::memset(B->n_nowrap, 0, sizeof(B->n_nowrap));
  B->has_fire = B->has_md = false;
  for (int d = 0; d <= kMaxD; d++) {
    B->has_wrap[d] = B->has_nowrap[d] = B->mix[d] = B->has_half[d] = false;
    B->kinds_md[d] = B->kinds_fire[d] = 0;
  }
  int64_t atom_base = 0, cell_base = 0;
  int64_t a_off[kMaxD + 1], c_off[kMaxD + 1];
  for (int d = kMinD; d <= kMaxD; d++) {
    a_off[d] = atom_base;
    c_off[d] = cell_base;
    int occ_tot = 0, occ_n = 0;
    for (int s = 0; s < B->max_slots; s++) {
      const SlotInfo& S = B->slots[s];
      if (!S.used || S.p.d != d) continue;
      for (int k = 0; k < S.p.ntiles; k++) atom.push_back(make_int2(s, k));
      B->n_atom[d] += S.p.ntiles;
      if (S.p.mix) B->mix[d] = true;
      if (S.p.reach == 2) B->has_half[d] = true;
      const int kind = 1 << ((S.p.mix ? 1 : 0) | (S.p.morse ? 2 : 0) | (lpa_index(S.p.lpa) << 2));
      if (S.mode == MODE_MD) B->kinds_md[d] |= kind;
      else B->kinds_fire[d] |= kind;
      occ_tot += S.p.n;
      occ_n += S.p.ncells;
    }
    // cell tiles: systems with n_cell >= 3 first, then the wrap systems
    for (int pass = 0; pass < 2; pass++) {
      for (int s = 0; s < B->max_slots; s++) {
        const SlotInfo& S = B->slots[s];
        if (!S.used || S.p.d != d || (int)S.p.wrap != pass) continue;
        for (int k = 0; k < S.p.ncells; k++) cell.push_back(make_int2(s, k));
        B->n_cell[d] += S.p.ncells;
        if (pass == 0) B->n_nowrap[d] += S.p.ncells, B->has_nowrap[d] = true;
        else B->has_wrap[d] = true;
      }
    }
    atom_base += B->n_atom[d];
    cell_base += B->n_cell[d];
    double occ = occ_n ? (double)occ_tot / occ_n : 1.0;
    // candidate-lane build for the n_cell <= 2 systems too, four waves per
    // subcell (few, crowded subcells per system; HDMD_WRAP_G overrides)
    {
      const char* e = std::getenv("HDMD_WRAP_G");
      const int g = e ? std::atoi(e) : 4;
      B->blk[d] = (g == 1 || g == 2 || g == 4) ? g : 4;
    }
    (void)occ;
  }
  for (int s = 0; s < B->max_slots; s++) {
    const SlotInfo& S = B->slots[s];
    if (!S.used) continue;
    for (int k = 0; k < S.p.nchunks; k++) chunk.push_back(make_int2(s, k));
    sys.push_back(s);
    t.sys[s] = S.dev;
    if (S.mode == MODE_FIRE) B->has_fire = true;
    if (S.mode == MODE_MD) B->has_md = true;
  }
  if ((int64_t)atom.size() > B->cap_atom || (int64_t)cell.size() > B->cap_cell ||
      (int64_t)chunk.size() > B->cap_chunk)
    return fail(HDMD_ERR_WORKSPACE, "batch table capacity exceeded (max_atoms / max_cells)");
  B->n_chunk = (int)chunk.size();
  B->n_sys = (int)sys.size();
  for (int d = kMinD; d <= kMaxD; d++) {
    t.n_atom[d] = B->n_atom[d];
    t.n_cell[d] = B->n_cell[d];
    t.n_cell_nowrap[d] = B->n_nowrap[d];
    t.atom_tiles[d] = B->d_atom + a_off[d];
    t.cell_tiles[d] = B->d_cell + c_off[d];
  }
  t.n_atom[0] = (int32_t)atom_base;  // class 0: every class
  // class 0 lists its cell tiles in an array of its own, the n_cell >= 3
  // subcells of every class before the wrap ones (the list build of a batch
  // gives the former one wave each and the latter a workgroup each)
  std::vector<int2> cell_all;
  cell_all.reserve(cell.size());
  for (int pass = 0; pass < 2; pass++)
    for (int d = kMinD; d <= kMaxD; d++) {
      const int64_t lo = c_off[d] + (pass ? B->n_nowrap[d] : 0);
      const int64_t hi = c_off[d] + (pass ? B->n_cell[d] : B->n_nowrap[d]);
      cell_all.insert(cell_all.end(), cell.begin() + lo, cell.begin() + hi);
    }
  B->n_nowrap_all = 0;
  for (int d = kMinD; d <= kMaxD; d++) B->n_nowrap_all += B->n_nowrap[d];
  t.n_cell[0] = (int32_t)cell_base;
  t.n_cell_nowrap[0] = B->n_nowrap_all;
  t.atom_tiles[0] = B->d_atom;
  t.cell_tiles[0] = B->d_cell_all;
  B->n_atom_all = (int)atom_base;
  B->n_cell_all = (int)cell_base;
  t.n_chunk = B->n_chunk;
  t.n_sys = B->n_sys;
  t.chunk_tiles = B->d_chunk;
  t.sys_list = B->d_syslist;
  if (!atom.empty()) HIPCHK(hipMemcpyAsync(B->d_atom, atom.data(), atom.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  if (!cell.empty()) HIPCHK(hipMemcpyAsync(B->d_cell, cell.data(), cell.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  if (!cell_all.empty())
    HIPCHK(hipMemcpyAsync(B->d_cell_all, cell_all.data(), cell_all.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  if (!chunk.empty()) HIPCHK(hipMemcpyAsync(B->d_chunk, chunk.data(), chunk.size() * sizeof(int2), hipMemcpyHostToDevice, st));
  if (!sys.empty()) HIPCHK(hipMemcpyAsync(B->d_syslist, sys.data(), sys.size() * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(B->dtab, &t, sizeof(Table), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));  // host vectors die here
  B->dirty = false;
  return HDMD_OK;
}

static inline int pow2_grid(int n, int cap) {
  int g = 1;
  while (g < n && g < cap) g <<= 1;
  return g;
}

static KArgs batch_args(HostBatch* B, int d, int part = 0) {
  KArgs a;
  a.single = nullptr;
  a.tab = B->dtab;
  a.cls = d;
  a.part = part;
  return a;
}

// One iteration over every running slot: FIRE control and update, MD steps,
// the shared rebuild chain, finalisation, then the FIRE forces.
static void enqueue_batch_iter(HostBatch* B, const std::vector<int>& grids, hipStream_t st) {
  const int gsys = grids[0], gchunk = grids[1];
  auto ga = [&](int d) { return grids[2 + 3 * (d - kMinD)]; };
  auto gc = [&](int d) { return grids[3 + 3 * (d - kMinD)]; };
  KArgs a0 = batch_args(B, 0);  // class 0: the tiles of every class
  const int ga_all = grids[grids.size() - 4], gc_all = grids[grids.size() - 3];
  const int gb_all = grids[grids.size() - 2];
  if (B->has_fire) {
    launch_fire_ctrl(a0, gsys, st);
    launch_fire_update_all(a0, ga_all, st);
  }
  if (B->has_md)
    for (int d = kMinD; d <= kMaxD; d++)
      for (int k = 0; k < 12; k++)
        if (B->kinds_md[d] >> k & 1)
          dkernels(d)->step(k & 1, lpa_of_index(k >> 2), k & 2, batch_args(B, d), ga(d), st);
  launch_bin_all(a0, ga_all, st);
  launch_scan1(a0, gchunk, st);
  launch_scan2(a0, gsys, st);
  launch_scatter(a0, ga_all, st);
  launch_cellsort_all(a0, gc_all, st);
  // list builds: one launch per stencil radius present (a launch serves the
  // systems of its own radius and passes over the others' subcells)
  auto class_builds = [&](int d) {
    if (B->has_nowrap[d]) dkernels(d)->build(1, false, 1, batch_args(B, d, 1), gc(d), st);
    if (B->has_half[d]) dkernels(d)->build(2, false, 1, batch_args(B, d, 1), gc(d), st);
    if (B->has_wrap[d]) dkernels(d)->build(1, true, B->blk[d], batch_args(B, d, 2), gc(d), st);
  };
  if (gb_all > 0) {
    bool half = false;
    for (int d = kMinD; d <= kBuildAllMaxD; d++) half |= B->has_half[d];
    launch_build_all(a0, gb_all, 1, st);
    if (half) launch_build_all(a0, gb_all, 2, st);
    for (int d = kBuildAllMaxD + 1; d <= kMaxD; d++) class_builds(d);
  } else {
    for (int d = kMinD; d <= kMaxD; d++) class_builds(d);
  }
  launch_finalize(a0, gsys, st);
  if (B->has_fire) {
    // systems with one lane per atom in classes d <= kBuildAllMaxD: one launch
    // over every class (Morse systems in a launch of their own); the others:
    // a launch per class and kind
    int kinds = 0;
    for (int d = kMinD; d <= kBuildAllMaxD; d++) kinds |= B->kinds_fire[d];
    if (kinds & 0x3) launch_force_all(a0, ga_all, 1, false, st);
    if (kinds & 0xc) launch_force_all(a0, ga_all, 1, true, st);
    for (int d = kMinD; d <= kMaxD; d++)
      for (int k = d <= kBuildAllMaxD ? 4 : 0; k < 12; k++)
        if (B->kinds_fire[d] >> k & 1)
          dkernels(d)->force(k & 1, lpa_of_index(k >> 2), k & 2, batch_args(B, d), ga(d), 1, st);
  }
}

}  // namespace hdmd

extern "C" {

size_t hdmd_batch_bytes(int32_t max_slots, int64_t max_atoms, int64_t max_cells) {
  if (max_slots < 1 || max_slots > kMaxSlots || max_atoms < 0 || max_cells < 0) return 0;
  int64_t ca, cc, ch;
  caps(max_slots, max_atoms, max_cells, ca, cc, ch);
  return batch_layout(max_slots, ca, cc, ch).bytes;
}

int hdmd_batch_init(void* table_ws, size_t table_bytes, int32_t max_slots, int64_t max_atoms,
                    int64_t max_cells, void* stream) {
  if (!table_ws) return fail(HDMD_ERR_ARG, "null table workspace");
  if (max_slots < 1 || max_slots > kMaxSlots) return fail(HDMD_ERR_ARG, "max_slots must be in [1, 1024]");
  int64_t ca, cc, ch;
  caps(max_slots, max_atoms, max_cells, ca, cc, ch);
  BatchLayout L = batch_layout(max_slots, ca, cc, ch);
  if (table_bytes < L.bytes) return fail(HDMD_ERR_WORKSPACE, "table workspace too small");
  HostBatch* B = new HostBatch();
  B->max_slots = max_slots;
  B->cap_atom = ca;
  B->cap_cell = cc;
  B->cap_chunk = ch;
  B->dtab = at<Table>(table_ws, L.off_tab);
  B->d_atom = at<int2>(table_ws, L.off_atom);
  B->d_cell = at<int2>(table_ws, L.off_cell);
  B->d_cell_all = at<int2>(table_ws, L.off_cell_all);
  B->d_chunk = at<int2>(table_ws, L.off_chunk);
  B->d_syslist = at<int32_t>(table_ws, L.off_sys);
  B->d_state = at<int32_t>(table_ws, L.off_state);
  B->d_iters = at<int64_t>(table_ws, L.off_iters);
  B->slots.resize(max_slots);
  {
    std::lock_guard<std::mutex> g(g_batch_mu);
    auto it = g_batches.find(table_ws);
    if (it != g_batches.end()) {
      for (auto& kv : it->second->graphs) hipGraphExecDestroy(kv.second);
      delete it->second;
    }
    g_batches[table_ws] = B;
  }
  return upload_tables(B, S(stream));
}

static int batch_add(void* table_ws, int32_t slot, const hdmd_system* sys, const double* pos,
                     const double* vel, const double* diam, void* ws, size_t ws_bytes,
                     const hdmd_fire_params* fp, int64_t nsteps, double dt, void* stream) {
  HostBatch* B = find_batch(table_ws);
  if (!B) return fail(HDMD_ERR_STATE, "batch table not initialised");
  if (slot < 0 || slot >= B->max_slots) return fail(HDMD_ERR_ARG, "slot out of range");
  if (B->slots[slot].used) return fail(HDMD_ERR_STATE, "slot is occupied");
  Plan p;
  int rc = make_plan(sys, p);
  if (rc) return rc;
  hipStream_t st = S(stream);
  int blk = 64;
  SysDev* dev = at<SysDev>(ws, p.off_desc);
  SysDev h;
  if (fp) {
    rc = fire_start(sys, p, pos, diam, ws, ws_bytes, fp, st, &blk);
    if (rc) return rc;
    rc = read_desc(dev, &h, st);
    if (rc) return rc;
  } else {
    if (nsteps < 0 || !(dt > 0)) return fail(HDMD_ERR_ARG, "need nsteps >= 0 and dt > 0");
    if (sys->thermostat_tau > 0 && sys->thermostat_tau < dt)
      return fail(HDMD_ERR_ARG, "thermostat_tau must be >= dt");
    if (!vel) return fail(HDMD_ERR_ARG, "null velocity pointer");
    rc = init_system(sys, p, pos, diam, vel, ws, ws_bytes, st, &blk);
    if (rc) return rc;
    rc = read_desc(dev, &h, st);
    if (rc) return rc;
    rc = err_to_status(h.err, "hdmd_batch_add_md");
    if (rc) return rc;
    h.mode = MODE_MD;
    h.dt = dt;
    h.nsteps = nsteps;
    h.thermo = nullptr;
    h.thermo_every = 0;
    h.step = 0;
    launch_setdesc(dev, h, st);
    HIPCHK(hipStreamSynchronize(st));
  }
  SlotInfo& S_ = B->slots[slot];
  S_.used = true;
  S_.p = p;
  S_.dev = dev;
  S_.ws = ws;
  S_.mode = fp ? MODE_FIRE : MODE_MD;
  S_.blk = blk;
  B->dirty = true;
  return HDMD_OK;
}

int hdmd_batch_add_fire(void* table_ws, int32_t slot, const hdmd_system* sys, const double* pos,
                        const double* diam, void* ws, size_t ws_bytes,
                        const hdmd_fire_params* params, void* stream) {
  if (!params) return fail(HDMD_ERR_ARG, "null FIRE parameters");
  return batch_add(table_ws, slot, sys, pos, nullptr, diam, ws, ws_bytes, params, 0, 0.0, stream);
}

int hdmd_batch_add_md(void* table_ws, int32_t slot, const hdmd_system* sys, const double* pos,
                      const double* vel, const double* diam, void* ws, size_t ws_bytes,
                      int64_t nsteps, double dt, void* stream) {
  return batch_add(table_ws, slot, sys, pos, vel, diam, ws, ws_bytes, nullptr, nsteps, dt, stream);
}

int hdmd_batch_run(void* table_ws, int32_t iterations, void* stream) {
  HostBatch* B = find_batch(table_ws);
  if (!B) return fail(HDMD_ERR_STATE, "batch table not initialised");
  if (iterations < 1) return fail(HDMD_ERR_ARG, "iterations must be >= 1");
  hipStream_t st = S(stream);
  if (B->dirty) {
    int rc = upload_tables(B, st);
    if (rc) return rc;
  }
  if (B->n_sys == 0) return HDMD_OK;
  // persistent grids rounded up to powers of two so that a captured graph
  // stays valid while the composition changes within the same sizes
  std::vector<int> grids;
  grids.push_back(pow2_grid(B->n_sys, 1024));
  grids.push_back(pow2_grid(B->n_chunk, 2048));
  for (int d = kMinD; d <= kMaxD; d++) {
    grids.push_back(B->n_atom[d] ? pow2_grid(B->n_atom[d], 4096) : 0);
    grids.push_back(B->n_cell[d] ? pow2_grid(B->n_cell[d], 8192) : 0);
    grids.push_back(B->blk[d] * 4 + (B->has_wrap[d] ? 2 : 0) + (B->has_nowrap[d] ? 1 : 0) +
                    (B->mix[d] ? 1024 : 0) + (B->has_half[d] ? 2048 : 0));
  }
  for (int d = kMinD; d <= kMaxD; d++) grids.push_back(B->kinds_md[d] | (B->kinds_fire[d] << 12));
  grids.push_back(B->has_fire ? 1 : 0);
  grids.push_back(B->has_md ? 1 : 0);
  grids.push_back(pow2_grid(B->n_atom_all, 4096));  // all-class launches
  grids.push_back(pow2_grid(B->n_cell_all, 8192));
  // one list-build launch over every class (0: one launch per class and variant)
  grids.push_back(std::getenv("HDMD_BUILD_PER_CLASS")
                      ? 0
                      : pow2_grid((B->n_nowrap_all + 3) / 4 + (B->n_cell_all - B->n_nowrap_all), 8192));
  grids.push_back(iterations);
  if (!graphs_enabled()) {
    for (int k = 0; k < iterations; k++) enqueue_batch_iter(B, grids, st);
    HIPCHK(hipGetLastError());
    return HDMD_OK;
  }
  hipGraphExec_t exec = nullptr;
  auto it = B->graphs.find(grids);
  if (it != B->graphs.end()) exec = it->second;
  if (!exec) {
    std::lock_guard<std::mutex> g(g_graph_mu);
    if (!g_capture_stream) HIPCHK(hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < iterations; k++) enqueue_batch_iter(B, grids, g_capture_stream);
    hipGraph_t graph;
    HIPCHK(hipStreamEndCapture(g_capture_stream, &graph));
    HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    HIPCHK(hipGraphDestroy(graph));
    B->graphs[grids] = exec;
  }
  HIPCHK(hipGraphLaunch(exec, st));
  return HDMD_OK;
}

int hdmd_batch_poll(void* table_ws, int32_t* state, int64_t* iters, void* stream) {
  HostBatch* B = find_batch(table_ws);
  if (!B) return fail(HDMD_ERR_STATE, "batch table not initialised");
  if (!state) return fail(HDMD_ERR_ARG, "null state array");
  hipStream_t st = S(stream);
  if (B->dirty) {
    int rc = upload_tables(B, st);
    if (rc) return rc;
  }
  launch_poll(B->dtab, B->max_slots, B->d_state, B->d_iters, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(state, B->d_state, (size_t)B->max_slots * 4, hipMemcpyDeviceToHost, st));
  if (iters) HIPCHK(hipMemcpyAsync(iters, B->d_iters, (size_t)B->max_slots * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return HDMD_OK;
}

int hdmd_batch_take(void* table_ws, int32_t slot, double* pos, double* vel,
                    hdmd_fire_result* result, void* stream) {
  HostBatch* B = find_batch(table_ws);
  if (!B) return fail(HDMD_ERR_STATE, "batch table not initialised");
  if (slot < 0 || slot >= B->max_slots || !B->slots[slot].used)
    return fail(HDMD_ERR_STATE, "slot is empty");
  hipStream_t st = S(stream);
  SlotInfo& S_ = B->slots[slot];
  SysDev h;
  int rc = read_desc(S_.dev, &h, st);
  if (rc) return rc;
  if (result) {
    if (S_.mode == MODE_FIRE) {
      fill_result(h, 0, result);
    } else {
      result->iterations = h.step > 0 ? h.step - 1 : 0;
      result->builds = h.builds;
      result->fmax = 0.0;
      result->energy = h.pe + h.ke;
      result->status = 0;
      result->pad = 0;
    }
  }
  int status = err_to_status(h.err, "batch slot");
  if (status == HDMD_OK && (pos || vel)) {
    dkernels(S_.p.d)->unload(S_.p.mix, S_.dev, S_.p.ntiles, st, pos, vel, nullptr);
    HIPCHK(hipGetLastError());
  }
  S_.used = false;
  S_.dev = nullptr;
  B->dirty = true;
  rc = upload_tables(B, st);  // the slot's workspace may be released after this call
  if (rc) return rc;
  if (status) return status;
  if (S_.mode == MODE_FIRE && h.fstatus != 0) return HDMD_NOT_CONVERGED;
  return HDMD_OK;
}

}  // extern "C"
