// kernels.h -- the gfx950 kernels of the hot path, templated on the dimension D.
//
//  k_load        caller [n][d] arrays -> internal buffers (wrap, validate)
//  k_bin         subcell of every atom + occupancy counts      (Sec. II.C)
//  k_scatter     counting-sort placement by subcell            (common.hip)
//  k_cellsort    per-subcell sort by caller id, permutation of every per-atom
//                array, reference positions, prefilter offsets
//  k_build       Verlet rows over the 3^d linked subcells      (Sec. II.C, Fig. 1)
//  k_force       pair forces and energy (+ FIRE reductions)    (Sec. II.B)
//  k_step        fused velocity-Verlet step + rebuild trigger (Sec. II.B/II.C)
//  k_fire_update semi-implicit Euler FIRE update
//  k_unload      internal -> caller order
//  k_vanhove     unwrapped displacements and the self van Hove histogram
//  k_swap_de, k_swap_settle  SWAP Monte Carlo in batches (Sec. II.D)
#pragma once
#include <type_traits>

#include "hdmd_dev.h"

namespace hdmd {

// ---------------------------------------------------------------------------
// load / unload
// ---------------------------------------------------------------------------
template <int D, typename VT>
__global__ __launch_bounds__(kTile) void k_load(SysDev* s, const double* __restrict__ pos,
                                                const double* __restrict__ diam,
                                                const double* __restrict__ vel) {
  int i = blockIdx.x * kTile + threadIdx.x;
  if (i >= s->npad) return;
  const int cur = s->xcur, pc = s->pcur, npad = s->npad;
  double* xo = s->x[cur ^ 1];
  VT* vo = reinterpret_cast<VT*>(s->v[pc]);
  double x[D];
  if (i >= s->n) {
#pragma unroll
    for (int k = 0; k < D; k++) {
      x[k] = 0.0;
      vo[(size_t)k * npad + i] = VT(0);
    }
    store_rec<D>(xo, i, x, 0.0);
    s->oid[pc][i] = -1;
    return;
  }
  const double L = s->L, h = s->hL;
  int err = 0;
#pragma unroll
  for (int k = 0; k < D; k++) {
    double t = pos[(size_t)i * D + k];
    if (!isfinite(t)) {
      err |= ERR_NONFINITE;
      t = 0.0;
    } else if (t < -3.0 * h || t >= 3.0 * h) {
      err |= ERR_ARG;
      t = 0.0;
    }
    x[k] = wrap1(t, L, h);
    double u = vel ? vel[(size_t)i * D + k] : 0.0;
    if (!isfinite(u)) {
      err |= ERR_NONFINITE;
      u = 0.0;
    }
    vo[(size_t)k * npad + i] = VT(u);
  }
  double sg = diam[i];
  if (!isfinite(sg)) {
    err |= ERR_NONFINITE;
    sg = 0.0;
  } else if (!(sg > 0.0) || sg > s->sigma_max) {
    err |= ERR_ARG;
  }
  store_rec<D>(xo, i, x, sg);
  s->oid[pc][i] = i;
  if (err) atomicOr(&s->err, err);
}

template <int D, typename VT>
__global__ __launch_bounds__(kTile) void k_unload(const SysDev* s, double* __restrict__ pos,
                                                  double* __restrict__ vel,
                                                  double* __restrict__ force) {
  int p = blockIdx.x * kTile + threadIdx.x;
  if (p >= s->n) return;
  const int cur = s->xcur, pc = s->pcur, npad = s->npad;
  int a = s->oid[pc][p];
  if (pos) {
    double x[D];
    load_x<D>(s->x[cur], p, x);
#pragma unroll
    for (int k = 0; k < D; k++) pos[(size_t)a * D + k] = x[k];
  }
  if (vel) {
    const VT* v = reinterpret_cast<const VT*>(s->v[pc]);
#pragma unroll
    for (int k = 0; k < D; k++) vel[(size_t)a * D + k] = double(v[(size_t)k * npad + p]);
  }
  if (force) {
    const VT* f = reinterpret_cast<const VT*>(s->f);
#pragma unroll
    for (int k = 0; k < D; k++) force[(size_t)a * D + k] = double(f[(size_t)k * npad + p]);
  }
}

// Whether the caller's arrays (positions, velocities, diameters in caller
// order) are bit for bit the state the workspace holds, as the last unload
// wrote them; any difference sets s->differ.
template <int D, typename VT>
__global__ __launch_bounds__(kTile) void k_same_state(SysDev* s, const double* __restrict__ pos,
                                                      const double* __restrict__ vel,
                                                      const double* __restrict__ diam) {
  const int p = blockIdx.x * kTile + threadIdx.x;
  if (p >= s->n) return;
  const int pc = s->pcur, npad = s->npad;
  const int a = s->oid[pc][p];
  double x[D], sg;
  load_rec<D>(s->x[s->xcur], p, x, sg);
  const VT* v = reinterpret_cast<const VT*>(s->v[pc]);
  bool same = diam[a] == sg;
#pragma unroll
  for (int k = 0; k < D; k++) {
    same = same && pos[(size_t)a * D + k] == x[k];
    same = same && vel[(size_t)a * D + k] == double(v[(size_t)k * npad + p]);
  }
  if (!same) atomicOr(&s->differ, 1);
}

// The displacement observables of a continued run start from zero: the
// displacement up to the last build is set to minus the part since it.
template <int D>
__global__ __launch_bounds__(kTile) void k_disp_restart(SysDev* s) {
  const int p = blockIdx.x * kTile + threadIdx.x;
  if (p >= s->npad) return;
  const int pc = s->pcur, npad = s->npad;
  double x[D];
  load_x<D>(s->x[s->xcur], p, x);
#pragma unroll
  for (int k = 0; k < D; k++) {
    const size_t o = (size_t)k * npad + p;
    s->disp[pc][o] = p < s->n ? -min_image(x[k] - s->xref[o], s->L, s->hL) : 0.0;
  }
}

// Unwrapped displacement of every atom since the MD call's step 0 (the
// displacement up to the last build plus the minimum image of x - x_ref),
// written in caller order to disp ([n][d], optional), and the histogram of
// |dr| behind the self part of the van Hove function (eq. VGC, Sec. II.E):
// hist[b] counts b w <= |dr| < (b+1) w, hist[nbins] the atoms beyond.
template <int D>
__global__ __launch_bounds__(kTile) void k_vanhove(const SysDev* s, int nbins, double w,
                                                   unsigned long long* __restrict__ hist,
                                                   double* __restrict__ disp) {
  const int p = blockIdx.x * kTile + threadIdx.x;
  if (p >= s->n) return;
  const int pc = s->pcur, npad = s->npad;
  const double L = s->L, h = s->hL;
  double x[D];
  load_x<D>(s->x[s->xcur], p, x);
  const int a = s->oid[pc][p];
  double r2 = 0.0;
#pragma unroll
  for (int k = 0; k < D; k++) {
    const size_t o = (size_t)k * npad + p;
    const double dk = s->disp[pc][o] + min_image(x[k] - s->xref[o], L, h);
    if (disp) disp[(size_t)a * D + k] = dk;
    r2 = __builtin_fma(dk, dk, r2);
  }
  if (hist) {
    const double q = floor(sqrt(r2) / w);
    const int b = q < (double)nbins ? (int)q : nbins;
    atomicAdd(hist + b, 1ull);
  }
}

// ---------------------------------------------------------------------------
// subcell binning: C_k = floor((x_k + L/2) n/L) clamped, I = sum C_k n^(d-1-k)
// ---------------------------------------------------------------------------
template <int D>
__device__ inline int flat_cell(const SysDev* s, const double (&x)[D]) {
  const int nc = s->ncell;
  const double h = s->hL, inv = s->inv_lsc;
  int I = 0;
#pragma unroll
  for (int k = 0; k < D; k++) {
    int c = (int)floor((x[k] + h) * inv);
    c = c < 0 ? 0 : (c > nc - 1 ? nc - 1 : c);
    I = I * nc + c;
  }
  return I;
}

// One atom tile of a system that rebuilds: subcell index and arrival rank.
template <int D>
__device__ inline void bin_tile(SysDev* s, int tile) {
  if (tile == 0 && threadIdx.x == 0) s->max_cell = 0;
  int i = tile * kTile + threadIdx.x;
  if (i >= s->n) return;
  double x[D];
  load_x<D>(s->x[s->xcur ^ 1], i, x);
  if (s->mode == MODE_MD) {
    // fold the displacement since the last build into the unwrapped
    // displacement (it stays below L/2 between builds, so the minimum image
    // is the true one)
    double* dp = s->disp[s->pcur];
    const size_t np = s->npad;
#pragma unroll
    for (int k = 0; k < D; k++)
      dp[k * np + i] += min_image(x[k] - s->xref[k * np + i], s->L, s->hL);
  }
  int c = flat_cell<D>(s, x);
  s->cell_of[i] = c;
  s->rank[i] = atomicAdd(&s->cell_count[c], 1);
}

template <int D>
__global__ __launch_bounds__(kTile) void k_bin(KArgs a) {
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int tile;
    if (!fetch_atom_tile(a, t, s, tile)) break;
    if (!running(s) || !need_rebuild(s)) {
      if (a.single) break;  // one system: the same for every tile
      continue;
    }
    bin_tile<D>(s, tile);
  }
}

// ---------------------------------------------------------------------------
// per-subcell sort (all-ascending bitonic network; entries at index >= cnt
// act as +infinity so any occupancy works) and permutation of the atom arrays
// ---------------------------------------------------------------------------
template <bool KV>
__device__ inline void bitonic_sort(int* keys, int* vals, int cnt) {
  int p2 = 1;
  while (p2 < cnt) p2 <<= 1;
  const int half = p2 >> 1;
  auto cas = [&](int i, int p) {
    if (p < cnt && keys[i] > keys[p]) {
      int k = keys[i]; keys[i] = keys[p]; keys[p] = k;
      if (KV) { int v = vals[i]; vals[i] = vals[p]; vals[p] = v; }
    }
  };
  for (int size = 2; size <= p2; size <<= 1) {
    const int hs = size >> 1;
    for (int t = threadIdx.x; t < half; t += blockDim.x) {
      int blk = t / hs, off = t % hs;
      cas(blk * size + off, blk * size + size - 1 - off);
    }
    __syncthreads();
    for (int st = size >> 2; st > 0; st >>= 1) {
      for (int t = threadIdx.x; t < half; t += blockDim.x) {
        int blk = t / st, off = t % st;
        int i = blk * 2 * st + off;
        cas(i, i + st);
      }
      __syncthreads();
    }
  }
}

__device__ inline int sext8(int w, int k) { return (int)(signed char)((w >> (8 * k)) & 0xff); }

// One subcell of a system that rebuilds (a block of 256 threads): its atoms
// sorted by their keys (caller id, or, with ysort, the quantised offset along
// the last axis and then caller id), then every per-atom array permuted into
// subcell order.
template <int D, typename VT>
__device__ inline void cellsort_tile(SysDev* s, int c, int* sk, int* sv) {
  constexpr int DY = Dims<D>::DY, QW = Dims<D>::QW;
  constexpr bool MIX = sizeof(VT) == 4;
  const int s0 = cell_start(s, c), cnt = cell_start(s, c + 1) - s0;
  if (threadIdx.x == 0) {
    s->cell_count[c] = 0;  // ready for the next build
    s->cell_flat[c] = s0;
    if (c == s->ncells - 1) s->cell_flat[s->ncells] = s->n;
  }
  if (cnt == 0) return;
  int* keys;
  int* vals;
  if (cnt <= kSortCap) {
    for (int q = threadIdx.x; q < cnt; q += blockDim.x) {
      sk[q] = s->key[s0 + q];
      sv[q] = s->src[s0 + q];
    }
    keys = sk;
    vals = sv;
  } else {
    keys = s->key + s0;
    vals = s->src + s0;
  }
  __syncthreads();
  bitonic_sort<true>(keys, vals, cnt);
  // subcell centre
  const int nc = s->ncell;
  double cen[D];
  {
    int u = c;
#pragma unroll
    for (int k = D - 1; k >= 0; k--) {
      cen[k] = k == D - 1 ? last_centre(s, c) : ((double)(u % nc) + 0.5) * s->lsc - s->hL;
      u /= nc;
    }
  }
  const int cur = s->xcur, pc = s->pcur, pn = pc ^ 1, npad = s->npad;
  const bool wrap = s->wrap != 0;
  const VT* vin = reinterpret_cast<const VT*>(s->v[pc]);
  VT* vout = reinterpret_cast<VT*>(s->v[pn]);
  const bool md = s->mode == MODE_MD;
  const double* din = s->disp[pc];
  double* dout = s->disp[pn];
  for (int q = threadIdx.x; q < cnt; q += blockDim.x) {
    const int src = vals[q], dst = s0 + q;
    double x[D], sg;
    load_rec<D>(s->x[cur ^ 1], src, x, sg);
    store_rec<D>(s->x[cur], dst, x, sg);
    if (MIX) store_q<D>(s->q[cur], dst, x, sg, s->hL, s->fxscale);
#pragma unroll
    for (int k = 0; k < D; k++) {
      s->xref[(size_t)k * npad + dst] = x[k];
      vout[(size_t)k * npad + dst] = vin[(size_t)k * npad + src];
      if (md) dout[(size_t)k * npad + dst] = din[(size_t)k * npad + src];
    }
    if (wrap) {
      float y[DY];
#pragma unroll
      for (int k = 0; k < DY; k++) y[k] = k < D ? (float)(x[k] - cen[k]) : 0.0f;
      float4* yp = reinterpret_cast<float4*>(s->ycell + (size_t)dst * DY);
#pragma unroll
      for (int k = 0; k < DY / 4; k++) yp[k] = make_float4(y[4 * k], y[4 * k + 1], y[4 * k + 2], y[4 * k + 3]);
      // 16-bit coordinates u = (x + L/2) 2^16 / L, wrapping at L: the 16-bit
      // difference u_j - u_i is the minimum-image displacement in L/2^16
      // units (candidate-lane build with n_cell <= 2)
      const double ws16 = 65536.0 / s->L;
      int p16[8];
#pragma unroll
      for (int k = 0; k < 8; k++) p16[k] = 0;
#pragma unroll
      for (int k = 0; k < D; k++) {
        const int u = (int)((long long)rint((x[k] + s->hL) * ws16) & 0xffff);
        p16[k / 2] |= u << (16 * (k % 2));
      }
      int4* pp = reinterpret_cast<int4*>(s->qc16 + (size_t)dst * 8);
      pp[0] = make_int4(p16[0], p16[1], p16[2], p16[3]);
      pp[1] = make_int4(p16[4], p16[5], p16[6], p16[7]);
    } else {
      int w[QW];
#pragma unroll
      for (int k = 0; k < QW; k++) w[k] = 0;
#pragma unroll
      for (int k = 0; k < D; k++)
        w[k / 4] |= (quant8(x[k] - cen[k], s->qinv) & 0xff) << (8 * (k % 4));
#pragma unroll
      for (int k = 0; k < QW; k++) s->qc[(size_t)dst * 4 + k] = w[k];
      // the same offsets as int16 pairs for the candidate-lane build, with
      // the atom's share of the pair threshold.  A pair is within its list
      // radius r_ij = a_i + a_j, a = (c sigma + s)/2, only if
      // |q_j - q_i| < alpha_i + alpha_j, alpha = a/Delta + sqrt(d)/2 (each
      // axis is off by at most one unit), and (alpha_i + alpha_j)^2 <=
      // 2 alpha_i^2 + 2 alpha_j^2 < T_i + T_j with T = floor(2 alpha^2) + 1:
      // one integer per atom, so the test stays one sum of products.  The
      // row cull takes the atom's reach a_i + r_l,max/2 instead of r_l,max.
      int p16[8], B = 0;
#pragma unroll
      for (int k = 0; k < 8; k++) p16[k] = 0;
#pragma unroll
      for (int k = 0; k < D; k++) {
        const int qv = sext8(w[k / 4], k % 4);
        p16[k / 2] |= (qv & 0xffff) << (16 * (k % 2));
        B += qv * qv;
      }
      const int T = thresh_share(s, sg);
      const double ai = 0.5 * (s->cutoff * sg + s->skin);
      const double reach = (ai + 0.5 * s->rlmax) * s->qinv;
      p16[(D + 1) / 2 < 4 ? 3 : 7] = B - T;
      p16[5] = (int)ceil(reach * reach);
      p16[6] = T;
      int4* pp = reinterpret_cast<int4*>(s->qc16 + (size_t)dst * 8);
      pp[0] = make_int4(p16[0], p16[1], p16[2], p16[3]);
      pp[1] = make_int4(p16[4], p16[5], p16[6], p16[7]);
    }
    s->oid[pn][dst] = s->ysort ? keys[q] & ((1 << 23) - 1) : keys[q];
  }
  __syncthreads();
}

template <int D, typename VT>
__global__ __launch_bounds__(256) void k_cellsort(KArgs a) {
  __shared__ int sk[kSortCap];
  __shared__ int sv[kSortCap];
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int c;
    if (!fetch_cell_tile(a, t, s, c)) break;
    if (!running(s) || !need_rebuild(s)) {
      if (a.single) break;  // one system: the same for every tile
      continue;
    }
    cellsort_tile<D, VT>(s, c, sk, sv);
  }
}

// ---------------------------------------------------------------------------
// Verlet-list build over the linked subcells (Sec. II.C, Fig. 1)
//
// One workgroup per home subcell; its atoms are the lanes (in chunks of BLK).
// The linked subcells are decoded on the fly from a mixed-radix counter
// (offsets -1/0/+1 per axis, -2..+2 on half-size subcells, or the
// deduplicated {0,+1} / {0} when n_cell is 2 / 1).  Each linked subcell's atoms are staged in LDS and every lane tests
// every staged atom with a conservative prefilter; survivors go to a per-lane
// LDS queue and are re-tested exactly in FP64 with the per-pair radius -- the
// operation sequence of the list definition -- before being appended to the
// row.  Row order: linked-subcell order, then slot order (deterministic).
//
// Prefilter, not wrapped (n_cell >= 3, or half-size subcells, at least 5 per
// axis): the image shift of a linked subcell is its offset times the subcell
// side for every pair within the list radius, so with
// offsets y from the subcell centres quantised to q = y/Delta (Delta =
// L_sc/250, shift D = 250 o exactly), |r - Delta |q_j + D - q_i|| <= Delta
// sqrt(d) and
//   |q_j + D - q_i|^2 = A_j + C_i - 2 q_i.q_j,  A_j = |q_j + D|^2,
//   C_i = |q_i|^2 - 2 q_i.D,
// where q_i.q_j is two or three packed int8 dot products (v_dot4_i32_i8);
// a pair survives when that is below ((r_l,max + Delta sqrt(d)) / Delta)^2.
// Prefilter, n_cell <= 2: FP32 offsets with the per-axis minimum image
// min(|u|, L - |u|), against the largest list radius enlarged by 1e-4.
// ---------------------------------------------------------------------------
template <int D>
__device__ inline void decode_linked(int q, int radix, int reach, int nc, const int (&ci)[D],
                                     int (&o)[D], int (&cj)[D]) {
  // radix 2 reach + 1: offsets -reach..+reach; fewer subcells per axis than
  // that: each of the n_cell subcells once (the deduplicated stencil)
  const bool dedup = radix < 2 * reach + 1;
#pragma unroll
  for (int k = D - 1; k >= 0; k--) {
    int dig = q % radix;
    q /= radix;
    int oo = dedup ? dig : dig - reach;
    int c2 = ci[k] + oo;
    c2 = c2 < 0 ? c2 + nc : (c2 >= nc ? c2 - nc : c2);
    cj[k] = c2;
    o[k] = dedup ? c2 - ci[k] : oo;
  }
}

template <int D, bool WRAP, int BLK>
__global__ __launch_bounds__(BLK) void k_build(KArgs a) {
  constexpr int DY = Dims<D>::DY, QW = Dims<D>::QW;
  constexpr int SW = WRAP ? DY : 4;  // staged words per candidate
  constexpr int UNR = WRAP ? 4 : 8;  // candidates tested per batch of LDS reads
  __shared__ float stage[BLK * SW];
  __shared__ int qbuf[kQCap * BLK];
  const int tid = threadIdx.x;
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int hc;
    if (!fetch_cell_tile(a, t, s, hc)) break;
    if (!running(s) || !need_rebuild(s)) {
      if (a.single) break;  // one system: the same for every tile
      continue;
    }
    const int h0 = cell_start(s, hc), h1 = cell_start(s, hc + 1);
    if (h0 == h1) continue;
    const int nc = s->ncell, radix = s->radix, nst = s->nstencil, npad = s->npad;
    const int reach = s->reach;
    const int W = s->width;
    const double* __restrict__ xb = s->x[s->xcur];
    int* __restrict__ nl = s->nl;
    const double L = s->L, hL = s->hL, cut = s->cutoff, skin = s->skin;
    const float lscf = s->lscf, Lf = s->Lf, rl2f = s->rl2f;
    const int tq = s->tq;
    int ci[D];
    {
      int u = hc;
#pragma unroll
      for (int k = D - 1; k >= 0; k--) {
        ci[k] = u % nc;
        u /= nc;
      }
    }
    int rowmax = 0;
    for (int hb = h0; hb < h1; hb += BLK) {
      const int i = hb + tid;
      const bool vi = i < h1;
      const int ii = vi ? i : h0;
      double xi[D], si;
      load_rec<D>(xb, ii, xi, si);
      float yi[D];
      int qi[QW], qik[D], qn2 = 0;
      if (WRAP) {
#pragma unroll
        for (int k = 0; k < D; k++) yi[k] = s->ycell[(size_t)ii * DY + k];
      } else {
#pragma unroll
        for (int k = 0; k < QW; k++) qi[k] = s->qc[(size_t)ii * 4 + k];
#pragma unroll
        for (int k = 0; k < D; k++) {
          qik[k] = sext8(qi[k / 4], k % 4);
          qn2 += qik[k] * qik[k];
        }
      }
      int len = 0, qn = 0;

      auto flush = [&]() {
        for (int m = 0; m < qn; m++) {
          const int j = qbuf[m * BLK + tid];
          double xj[D], sj;
          load_rec<D>(xb, j, xj, sj);
          const double r2 = dist2_exact<D>(xi, xj, L, hL);
          if (r2 < list_r2(si, sj, cut, skin)) {
            if (len < W) nl[(size_t)len * npad + i] = j;
            len++;
          }
        }
        qn = 0;
      };

      for (int q = 0; q < nst; q++) {
        int o[D], cj[D];
        decode_linked<D>(q, radix, reach, nc, ci, o, cj);
        int J = 0;
#pragma unroll
        for (int k = 0; k < D; k++) J = J * nc + cj[k];
        float tk[D];
        int Ci = 0;
        if (WRAP) {
#pragma unroll
          for (int k = 0; k < D; k++) tk[k] = (float)o[k] * lscf - yi[k];
        } else {
          Ci = qn2;
#pragma unroll
          for (int k = 0; k < D; k++) Ci -= 2 * kQScale * o[k] * qik[k];
        }
        const int j0 = __builtin_amdgcn_readfirstlane(cell_start(s, J));
        const int j1 = __builtin_amdgcn_readfirstlane(cell_start(s, J + 1));
        for (int jb = j0; jb < j1; jb += BLK) {
          const int m = min(BLK, j1 - jb);
          const int mp = (m + UNR - 1) / UNR * UNR;  // staged entries padded with sentinels
          __syncthreads();
          if (tid < mp) {
            if (WRAP) {
              float4* dst = reinterpret_cast<float4*>(stage + tid * SW);
              if (tid < m) {
                const float4* src = reinterpret_cast<const float4*>(s->ycell + (size_t)(jb + tid) * DY);
#pragma unroll
                for (int k = 0; k < DY / 4; k++) dst[k] = src[k];
              } else {
#pragma unroll
                for (int k = 0; k < DY / 4; k++) dst[k] = make_float4(1e30f, 1e30f, 1e30f, 1e30f);
              }
            } else {
              int w[4] = {0, 0, 0, 0x3fffffff};  // sentinel: A_j far above any threshold
              if (tid < m) {
#pragma unroll
                for (int k = 0; k < QW; k++) w[k] = s->qc[(size_t)(jb + tid) * 4 + k];
                int A = 0;
#pragma unroll
                for (int k = 0; k < D; k++) {
                  const int c = sext8(w[k / 4], k % 4) + kQScale * o[k];
                  A += c * c;
                }
                w[3] = A;  // QW <= 3 words of coordinates, then A_j
              }
              reinterpret_cast<int4*>(stage)[tid] = make_int4(w[0], w[1], w[2], w[3]);
            }
          }
          __syncthreads();
          for (int u0 = 0; u0 < mp; u0 += UNR) {
            unsigned mask = 0;
            if (WRAP) {
              float yj[UNR][DY];
#pragma unroll
              for (int uu = 0; uu < UNR; uu++) {
                const float4* src = reinterpret_cast<const float4*>(stage + (u0 + uu) * SW);
#pragma unroll
                for (int k = 0; k < DY / 4; k++) {
                  const float4 v = src[k];
                  yj[uu][4 * k] = v.x;
                  yj[uu][4 * k + 1] = v.y;
                  yj[uu][4 * k + 2] = v.z;
                  yj[uu][4 * k + 3] = v.w;
                }
              }
#pragma unroll
              for (int uu = 0; uu < UNR; uu++) {
                float r2 = 0.0f;
#pragma unroll
                for (int k = 0; k < D; k++) {
                  float dx = fabsf(yj[uu][k] + tk[k]);
                  dx = fminf(dx, Lf - dx);
                  r2 = __builtin_fmaf(dx, dx, r2);
                }
                mask |= (r2 < rl2f ? 1u : 0u) << uu;
              }
            } else {
              int4 w[UNR];
#pragma unroll
              for (int uu = 0; uu < UNR; uu++) w[uu] = reinterpret_cast<const int4*>(stage)[u0 + uu];
#pragma unroll
              for (int uu = 0; uu < UNR; uu++) {
                int dot = __builtin_amdgcn_sdot4(qi[0], w[uu].x, 0, false);
                if (QW > 1) dot = __builtin_amdgcn_sdot4(qi[QW > 1 ? 1 : 0], w[uu].y, dot, false);
                if (QW > 2) dot = __builtin_amdgcn_sdot4(qi[QW > 2 ? 2 : 0], w[uu].z, dot, false);
                mask |= (w[uu].w + Ci - 2 * dot < tq ? 1u : 0u) << uu;
              }
            }
            if (vi && mask) {
              while (mask) {
                const int b = __builtin_ctz(mask);
                mask &= mask - 1;
                const int j = jb + u0 + b;
                if (j != i) {
                  qbuf[qn * BLK + tid] = j;
                  qn++;
                }
              }
            }
            if (__any(qn > kQCap - UNR)) flush();
          }
        }
      }
      flush();
      if (vi) {
        s->nlen[i] = len;
        rowmax = max(rowmax, len);
      }
    }
    rowmax = wave_max_i(rowmax);
    if ((tid & (kWave - 1)) == 0 && rowmax > 0) {
      atomicMax(&s->max_row, rowmax);
      if (rowmax > W) atomicOr(&s->err, ERR_OVERFLOW);
    }
  }
}

// ---------------------------------------------------------------------------
// Verlet-list build, candidate-lane form
//
// Same list, same row order and the same exact FP64 test as k_build; the
// work is laid out the other way round.  The linked subcells come in rows
// along the last axis (offsets -1, 0, +1; -2..+2 on half-size subcells, RAD
// = 2), whose atoms are packed into 64-lane chunks: every lane takes one
// candidate j, shifts its quantised offsets by the subcell offset (q'_j = q_j
// + 250 o as int16, |q'| <= 125 + 250 RAD) and forms A_j = |q'_j|^2.  The home atoms i kept for the row are then
// walked uniformly, their records (q_i as int16 pairs and B_i = |q_i|^2 - T_i)
// coming through the scalar cache, each test being
//   |q'_j - q_i|^2 < T_i + T_j  <=>  (T_j - A_j) + q_i.(2 q'_j) > B_i
// (v_dot2_i32_i16 on int16 pairs), with per-atom threshold shares T that
// follow the pair's own list radius (set where the records are written).
// Wrapped systems (n_cell <= 2) test |u_j - u_i|^2 < tq on 16-bit wrapped
// coordinates against the largest list radius.
// The ballot of each test is written into lane i of a mask register, so
// after a chunk lane i holds the 64-bit mask of its surviving candidates.
// Every NB chunks the lanes turn back into home atoms and run the exact
// test on their survivors in chunk and lane order, appending to their own
// rows.
//
// A workgroup of G waves takes one home subcell; wave w takes the w-th of G
// contiguous shares of its atoms (more waves in flight per subcell at the
// price of repeating the candidate set-up), with no barrier between waves.
// ---------------------------------------------------------------------------
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef _Float16 hv4 __attribute__((ext_vector_type(4)));
typedef float fv4 __attribute__((ext_vector_type(4)));
typedef unsigned uv2 __attribute__((ext_vector_type(2)));
typedef unsigned uv4 __attribute__((ext_vector_type(4)));

// Operands of the matrix-core form of the pair test.  A pair test
//   S_ij = q_i.(2 q'_j) + C_j - B_i > 0   (C_j = T_j - A_j, B_i = |q_i|^2 - T_i)
// is read off one entry of the product of a candidate matrix (rows) and a
// home matrix (columns) over 16 slots:
//   candidate [2q'_j,0 .. 2q'_j,d-1, 2048, 1, 1, floor(C_j/2048), C_j mod 2048, 0 ..]
//   home      [-q_i,0 .. -q_i,d-1, floor(B_i/2048), B_i mod 2048, 1/2, -2048, -1, 0 ..]
// gives 1/2 - S_ij, negative exactly when the test passes.  Every slot is an
// integer of magnitude <= 2048 or 1/2 (exact in f16: |q| <= 127, |2q'| <=
// 1254, -3.93e6 <= C < 2^22, |B| < 2^18) and every partial sum is a multiple
// of 1/2 below 2^23 in magnitude, so the f32 accumulation is exact in any
// order.
__device__ inline unsigned pack_h2(_Float16 lo, _Float16 hi) {
  return (unsigned)__builtin_bit_cast(unsigned short, lo) |
         ((unsigned)__builtin_bit_cast(unsigned short, hi) << 16);
}
// f16 value of int16 half k of a packed word (converted from 16 bits: one
// instruction, where a conversion from 32 bits goes through f32)
__device__ inline _Float16 i16_half(int w, int k) {
  return (_Float16)(short)(k ? (w >> 16) : w);
}
// f16 value of a small integer (|v| <= 2048)
__device__ inline _Float16 small_h(int v) { return (_Float16)(short)v; }
// the 16 slots as 8 words (word t: slots 2t, 2t + 1)
__device__ inline void slot_words(const _Float16 (&sl)[16], unsigned (&w)[8]) {
#pragma unroll
  for (int t = 0; t < 8; t++) w[t] = pack_h2(sl[2 * t], sl[2 * t + 1]);
}
// home slots from the atom's int16 offset words and its term B
template <int D>
__device__ inline void home_slots(const int* ow, int B, unsigned (&w)[8]) {
  _Float16 sl[16];
#pragma unroll
  for (int k = 0; k < 16; k++) sl[k] = (_Float16)0;
#pragma unroll
  for (int k = 0; k < D; k++) sl[k] = -i16_half(ow[k / 2], k % 2);
  sl[D] = small_h(B >> 11);
  sl[D + 1] = small_h(B & 2047);
  sl[D + 2] = (_Float16)0.5f;
  sl[D + 3] = (_Float16)(-2048);
  sl[D + 4] = (_Float16)(-1);
  slot_words(sl, w);
}
// candidate slots from its shifted, doubled offset words and C (an empty
// lane's C, below -2^22, becomes -2^22: its entries stay negative)
template <int D>
__device__ inline void cand_slots(const int* cw, int C, unsigned (&w)[8]) {
  C = max(C, -4194304);
  _Float16 sl[16];
#pragma unroll
  for (int k = 0; k < 16; k++) sl[k] = (_Float16)0;
#pragma unroll
  for (int k = 0; k < D; k++) sl[k] = i16_half(cw[k / 2], k % 2);
  sl[D] = (_Float16)2048;
  sl[D + 1] = (_Float16)1;
  sl[D + 2] = (_Float16)1;
  sl[D + 3] = small_h(C >> 11);
  sl[D + 4] = small_h(C & 2047);
  slot_words(sl, w);
}

// Uniform loads of the home records go through the scalar cache: read
// through the constant address space, which tells the compiler that the
// kernel does not write them (they come from an earlier kernel).
typedef __attribute__((address_space(4))) const v4i cv4i;
typedef __attribute__((address_space(4))) const v8i cv8i;

// A pointer that is the same in every lane, moved into scalar registers (a
// pointer read from device memory lands in vector registers otherwise).
template <typename T>
__device__ inline T* uniform_ptr(T* p) {
  const unsigned long long u = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return reinterpret_cast<T*>(((unsigned long long)hi << 32) | lo);
}

__device__ inline int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline double uniform_dbl(double v) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The lane-write intrinsic (v_writelane_b32): returns `old` with lane `ln`
// replaced by the uniform `val`.
__device__ int amdgcn_writelane(int val, int ln, int old) __asm("llvm.amdgcn.writelane");

// Wave priority 3, 2, 1, 0 over the four quarters of done/total (uniform).
__device__ inline void set_prio_by_progress(int done, int total) {
  const int q = (4 * done) / total;
  if (q == 0) __builtin_amdgcn_s_setprio(3);
  else if (q == 1) __builtin_amdgcn_s_setprio(2);
  else if (q == 2) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}

// Orders this wave's LDS writes before its later LDS reads (other lanes).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// One home subcell of a system that rebuilds, split over G waves: gw (< G)
// selects this wave's share of the home atoms; msk/cand are the wave's LDS
// arrays.
template <int D, int G, bool WR, int RAD = 1, bool MF = false>
__device__ inline void build_t_tile(SysDev* s, int hc, int gw, unsigned long long* msk, int* cand) {
  static_assert(RAD == 1 || (RAD == 2 && !WR), "wrapped systems take the 3^d stencil");
  static_assert(!(MF && WR), "the matrix-core test is for subcells of n_cell >= 3");
  constexpr int HW = (D + 1) / 2;        // int16 pair words of q
  // subcell slots of a row along the last axis: offsets -RAD..+RAD (wrapped:
  // the subcell itself and, for n_cell = 2, the other one; the third slot empty)
  constexpr int NRS = WR ? 3 : 2 * RAD + 1;
  constexpr int RW = HW < 4 ? 4 : 8;     // record words read per home atom
  constexpr int BW = RW - 1;             // word of B = |q|^2
  constexpr int CB = 4;                  // chunks of a row tested per home-record load
  constexpr int NB = 8;                  // chunks per exact pass (a multiple of CB)
  typedef typename std::conditional<RW == 4, v4i, v8i>::type Rec;
  typedef typename std::conditional<RW == 4, cv4i, cv8i>::type CRec;
  typedef __attribute__((address_space(4))) const int cint;
  typedef short short2v __attribute__((ext_vector_type(2)));
  const int lane = threadIdx.x & 63;
  // the position in a chunk of the candidate a lane takes: its lane, or for
  // the matrix-core test (MF) the position whose sign bit lands in bit order
  // (row 4g + v of candidate block cb = lane / 16: position 16g + 15 - 4cb - v)
  const int cpos = MF ? 16 * ((lane >> 2) & 3) + 15 - 4 * (lane >> 4) - (lane & 3) : lane;
  // subcell starts come through the scalar cache (written by an earlier kernel)
  cint* flat = (cint*)uniform_ptr(s->cell_flat);
  const int c0h = flat[hc];
  const int c1h = flat[hc + 1];
  // this wave's share of the home atoms
  const int per = (c1h - c0h + G - 1) / G;
  const int h0 = c0h + gw * per;
  const int h1 = min(c1h, h0 + per);
  if (h0 >= h1) return;
  const int nc = uniform_int(s->ncell), npad = uniform_int(s->npad);
  const int W = uniform_int(s->width), tq = uniform_int(s->tq), tcull = uniform_int(s->tcull);
  // sparse subcells (not wrapped): a row's NRS subcells hold 48 atoms or fewer on average
  const bool sparse = !WR && NRS * uniform_int(s->n) <= 48 * uniform_int(s->ncells);
  const double* __restrict__ xb = uniform_ptr(s->x[s->xcur]);
  const int* __restrict__ qc16 = uniform_ptr(s->qc16);
  HDMD_GLOBAL int* __restrict__ nl = gbl(uniform_ptr(s->nl));
  const double L = uniform_dbl(s->L), invL = 1.0 / L, hL = uniform_dbl(s->hL);
  const double cut = uniform_dbl(s->cutoff), skin = uniform_dbl(s->skin);
  int ci[D - 1], stride[D - 1];
  int cl;
  {
    int u = hc, st = 1;
    cl = u % nc;
    u /= nc;
    st = nc;
#pragma unroll
    for (int k = D - 2; k >= 0; k--) {
      ci[k] = u % nc;
      u /= nc;
      stride[k] = st;
      st *= nc;
    }
  }
  // rows of linked subcells: radix 2 RAD + 1 (offsets -RAD..+RAD; 3 for
  // subcells of side >= r_l,max, 5 for half-size subcells) or, for n_cell <=
  // 2, radix n_cell (offsets 0, +1: the deduplicated stencil)
  const int R = WR ? nc : NRS;
  int nrow = 1;
#pragma unroll
  for (int k = 0; k < D - 1; k++) nrow *= R;
  // the subcells of a row along the last axis and their offsets in the int16
  // half of the last axis (n_cell >= 2 RAD + 1 when not wrapped: all distinct)
  constexpr int lsh = 16 * ((D - 1) % 2);
  auto lcell = [&](int r) -> int {
    if (WR) return r == 0 ? cl : (cl == nc - 1 ? 0 : cl + 1);
    const int c2 = cl + r - RAD;
    return c2 < 0 ? c2 + nc : (c2 >= nc ? c2 - nc : c2);
  };
  auto lvalid = [&](int r) -> bool { return !WR || r == 0 || (r == 1 && R >= 2); };
  auto lshift = [&](int r) -> int {
    return WR ? 0 : (int)((unsigned)((kQScale * (r - RAD)) & 0xffff) << lsh);
  };
  // base subcell index of a row of linked subcells (offset digits of `row`
  // in base R over the first d-1 axes, last digit fastest)
  auto row_base = [&](int row, int (&Dp)[HW], int (&og)[D - 1]) -> int {
    int P = 0, r = row;
#pragma unroll
    for (int k = 0; k < HW; k++) Dp[k] = 0;
#pragma unroll
    for (int k = D - 2; k >= 0; k--) {
      const int o = WR ? r % R : r % R - RAD;
      r /= R;
      og[k] = o;
      int c2 = ci[k] + o;
      c2 = c2 < 0 ? c2 + nc : (c2 >= nc ? c2 - nc : c2);
      P += c2 * stride[k];
      Dp[k / 2] |= ((kQScale * o) & 0xffff) << (16 * (k % 2));
    }
    return P;
  };
  int rowmax = 0;
  // home atoms in passes of up to 128: lane l holds atoms hb + l and hb + 64 + l
  for (int hb = h0; hb < h1; hb += 128) {
    const int hcnt = uniform_int(min(128, h1 - hb));
    const bool two = hcnt > 64;
    const int i0 = hb + lane, i1 = hb + 64 + lane;
    const bool v0 = lane < hcnt, v1 = lane + 64 < hcnt;
    const int ii0 = v0 ? i0 : hb, ii1 = v1 ? i1 : hb;
    int qh0[D], qh1[D];
    // the row-cull threshold of each home atom (n_cell >= 3: its own reach;
    // wrapped: r_l,max)
    const int tc0 = WR ? tcull : qc16[(size_t)ii0 * 8 + 5];
    const int tc1 = WR ? tcull : qc16[(size_t)ii1 * 8 + 5];
    auto own_q = [&](int ii, int (&qh)[D]) {
      const v4i w0 = *reinterpret_cast<const v4i*>(qc16 + (size_t)ii * 8);
      int w[5] = {w0.x, w0.y, w0.z, w0.w, 0};
      if (HW > 4) w[4] = qc16[(size_t)ii * 8 + 4];
#pragma unroll
      for (int k = 0; k < D; k++) {
        const int word = w[k / 2];
        if (WR) {
          // gap to the other subcell along axis k (n_cell = 2: it touches both
          // faces), one unit short: L_sc/2 - |u - centre| - 1 in 2^16/L units
          const int u = (k % 2) ? ((word >> 16) & 0xffff) : (word & 0xffff);
          const int cc = (k < D - 1 ? ci[k < D - 1 ? k : 0] : cl) * 32768 + 16384;
          const int y = (int)(short)((u - cc) & 0xffff);
          qh[k] = max(16384 - abs(y) - 1, 0);
        } else {
          qh[k] = (k % 2) ? (word >> 16) : (int)(short)(word & 0xffff);
        }
      }
    };
    if constexpr (WR) {  // (n_cell >= 3: the offsets come from the record words)
      own_q(ii0, qh0);
      own_q(ii1, qh1);
    }
    // the lane's own home record (offset words and the home term), from
    // which the pair tests of n_cell >= 3 systems take each home atom's words
    // with v_readlane: the records of every wave of a CU (one subcell each)
    // do not fit the scalar cache.  Wrapped systems, whose waves walk long
    // runs of one crowded subcell, read them with scalar loads.
    int ow0[HW + 1], ow1[HW + 1];
#pragma unroll
    for (int k = 0; k < HW; k++) {
      ow0[k] = qc16[(size_t)ii0 * 8 + k];
      ow1[k] = qc16[(size_t)ii1 * 8 + k];
    }
    ow0[HW] = qc16[(size_t)ii0 * 8 + BW];
    ow1[HW] = qc16[(size_t)ii1 * 8 + BW];
    int len0 = 0, len1 = 0, nb = 0;

    // exact test of the survivors, spread over the lanes.  The survivors of
    // the pass are listed home atom by home atom (set 0, then set 1; each
    // atom's in chunk and bit order, the row order) as 16-bit codes (home
    // atom, chunk, bit) in the free chunk slots after the pass's masks (at
    // least one: chunks are tested only while nb + CB <= NB - 1), and taken
    // 64 at a time, one per lane.  In a batch the survivors of one home atom are a
    // run of consecutive lanes; a passing one goes to the atom's row at its
    // length so far plus the passing survivors of its run on lower lanes, so
    // every row takes its pairs in the row order.  (Walking each atom's own
    // survivors in its lane instead leaves most lanes idle: in a pass only
    // the atoms near its rows have survivors.)
    // The nearest image is taken with rint: with n_cell >= 3 the list radius
    // is at most L/3 (on half-size subcells, at least 5 per axis: 2L/5), so
    // every pair it can admit has all |dx_k| clear of L/2, where rint and
    // the definition's shift give the same value bit for bit; pairs with
    // some |dx_k| near L/2 are beyond the radius either way.
    static_assert(NB <= 8, "the chunk index fits three bits of a code");
    auto exact_pass = [&]() {
      wave_lds_sync();
      // survivor counts of the lane's two home atoms, and the chunks that
      // hold any (bit set * NB + b)
      int c0 = 0, c1 = 0;
      unsigned ne = 0;
      for (int b = 0; b < nb; b++) {
        const int n0 = __builtin_popcountll(msk[b * 128 + lane]);
        const int n1 = two ? __builtin_popcountll(msk[b * 128 + 64 + lane]) : 0;
        c0 += n0;
        c1 += n1;
        ne |= (n0 ? 1u << b : 0u) | (n1 ? 1u << (NB + b) : 0u);
      }
      int p0 = c0, p1 = c1;  // inclusive prefix sums over the lanes
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int u0 = __shfl_up(p0, o), u1 = __shfl_up(p1, o);
        if (lane >= o) {
          p0 += u0;
          p1 += u1;
        }
      }
      const int S0 = __shfl(p0, 63), S = S0 + __shfl(p1, 63);
      // first list index and count of each atom's survivors, packed
      // (index < 7 * 64 * 128 < 2^16, count <= 7 * 64)
      const unsigned r0 = ((unsigned)(p0 - c0) << 16) | (unsigned)c0;
      const unsigned r1 = ((unsigned)(S0 + p1 - c1) << 16) | (unsigned)c1;
      // Survivors spread evenly over the lanes (dense subcells and long rows
      // in d <= 4: the largest lane count within a few times the mean) are
      // walked lane by lane, each lane its own atoms' (set 0, then set 1;
      // chunk and bit order), which needs no listing.  (In higher d a pass's
      // rows are a small part of the stencil and its survivors crowd into
      // few atoms; the walk is not compiled there.)
      if (D <= 4 && 11 * wave_max_i(c0 + c1) <= S) {
        unsigned long long m = 0;
        int cb = 0, cur = -1, i = 0;
        double xi[D], si;  // own record, loaded when the walk reaches its set
        while (true) {
          if (m == 0) {
            if (ne == 0) break;
            cb = __builtin_ctz(ne);
            ne &= ne - 1;
            const int set = cb >= NB ? 1 : 0;
            m = msk[(cb % NB) * 128 + set * 64 + lane];
            if (set != cur) {
              cur = set;
              i = set ? i1 : i0;
              load_rec<D>(xb, set ? ii1 : ii0, xi, si);
            }
          }
          const int j = cand[(cb % NB) * 64 + __builtin_ctzll(m)];
          m &= m - 1;
          double xj[D], sj;
          load_rec<D>(xb, j, xj, sj);
          if (j != i) {
            double r2 = 0.0;
#pragma unroll
            for (int k = 0; k < D; k++) {
              const double dx = WR ? min_image(xj[k] - xi[k], L, hL)
                                   : near_image(xj[k] - xi[k], L, invL);
              r2 = __builtin_fma(dx, dx, r2);
              __builtin_amdgcn_sched_barrier(0);  // one axis at a time: few live registers
            }
            if (r2 < list_r2(si, sj, cut, skin)) {
              const int len = cur ? len1 : len0;
              if (len < W) nl[(size_t)len * npad + i] = j;
              if (cur) len1 = len + 1;
              else len0 = len + 1;
            }
          }
        }
        wave_lds_sync();
        nb = 0;
        return;
      }
      unsigned short* code = reinterpret_cast<unsigned short*>(msk + nb * 128);
      const int cap = 512 * (NB - nb);
      // each lane's walk over its survivors (set 0, then set 1; chunk and
      // bit order), resumed round after round: list index e, current chunk
      // cb and its remaining bits m
      int e = (int)(r0 >> 16), cb = 0;
      unsigned long long m = 0;
      for (int e0 = 0; e0 < S; e0 += cap) {
        const int e1 = min(S, e0 + cap);
        // the codes of list entries e0 .. e1 - 1
        while (e < e1) {
          if (m == 0) {
            if (ne == 0) break;
            const int nx = __builtin_ctz(ne);
            ne &= ne - 1;
            if (nx >= NB && cb < NB) e = (int)(r1 >> 16);  // on to set 1's list entries
            cb = nx;
            m = msk[(cb % NB) * 128 + (cb >= NB ? 64 : 0) + lane];
            if (e >= e1) break;
          }
          // up to two codes per trip (the trips are set by the lane with most)
          const int hc = (((cb >= NB ? 64 : 0) + lane) << 9) | ((cb % NB) << 6);
          code[e - e0] = (unsigned short)(hc | __builtin_ctzll(m));
          m &= m - 1;
          e++;
          if (m != 0 && e < e1) {
            code[e - e0] = (unsigned short)(hc | __builtin_ctzll(m));
            m &= m - 1;
            e++;
          }
        }
        wave_lds_sync();
        for (int t = e0; t < e1; t += 64) {
          const bool valid = t + lane < e1;
          const int cd = valid ? (int)code[t + lane - e0] : 0;
          const int h = cd >> 9;
          const int i = hb + h;
          const int j = valid ? cand[((cd >> 6) & 7) * 64 + (cd & 63)] : i;
          // the lanes below this one in its run (the run's head: the highest
          // lane at or below it whose home atom differs from the lane
          // below's), and the atom's row length so far
          const int hp = __shfl_up(h, 1);
          const unsigned long long H = __ballot(lane == 0 || hp != h);
          const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
          const int head = 63 - __builtin_clzll(H & (below | (1ull << lane)));
          const unsigned long long run = below & ~((1ull << head) - 1);
          const int la = __shfl(len0, h & 63), lb = __shfl(len1, h & 63);
          const int base = h >= 64 ? lb : la;
          __builtin_amdgcn_sched_barrier(0);
          double xi[D], si, xj[D], sj;
          load_rec<D>(xb, i, xi, si);
          load_rec<D>(xb, j, xj, sj);
          bool pass = false;
          if (j != i) {
            double r2 = 0.0;
#pragma unroll
            for (int k = 0; k < D; k++) {
              const double dx = WR ? min_image(xj[k] - xi[k], L, hL)
                                   : near_image(xj[k] - xi[k], L, invL);
              r2 = __builtin_fma(dx, dx, r2);
              __builtin_amdgcn_sched_barrier(0);  // one axis at a time: few live registers
            }
            pass = r2 < list_r2(si, sj, cut, skin);
          }
          const unsigned long long P = __ballot(pass);
          const int pos = base + __builtin_popcountll(P & run);
          if (pass && pos < W) nl[(size_t)pos * npad + i] = j;
          // the lane's own atoms take their passing survivors of the batch
          auto add = [&](unsigned rs, int& len) {
            const int st = (int)(rs >> 16), c = (int)(rs & 0xffff);
            const int lo = max(st - t, 0), hi = min(st + c - t, 64);
            if (lo < hi) {
              const unsigned long long mk =
                  (hi == 64 ? ~0ull : ((1ull << hi) - 1)) & ~((1ull << lo) - 1);
              len += __builtin_popcountll(P & mk);
            }
          };
          add(r0, len0);
          add(r1, len1);
        }
        wave_lds_sync();  // the codes are read before the next round lists over them
      }
      nb = 0;
    };

    // ballots of the kept home atoms of one set against `nch` chunks, four
    // home atoms per group of scalar loads (a short last group repeats its
    // last atom); lane h of m[c] receives home atom h's ballot for chunk c
    auto test_set = [&](unsigned long long km, const int (&ow)[HW + 1], int rb, int nch,
                        const int (&cw)[CB][HW], const int (&tA)[CB], unsigned (&mlo)[CB],
                        unsigned (&mhi)[CB]) {
      while (km) {
        int hh[4];
        hh[0] = __builtin_ctzll(km);
        km &= km - 1;
#pragma unroll
        for (int u = 1; u < 4; u++) {
          hh[u] = km ? __builtin_ctzll(km) : hh[u - 1];
          km &= km - 1;
        }
        int r[4][HW + 1];
#pragma unroll
        for (int u = 0; u < 4; u++) {
          if constexpr (WR) {
            const Rec w = *(CRec*)(qc16 + (size_t)(rb + hh[u]) * 8);
#pragma unroll
            for (int k = 0; k < HW; k++) r[u][k] = w[k];
          } else {
#pragma unroll
            for (int k = 0; k <= HW; k++) r[u][k] = __builtin_amdgcn_readlane(ow[k], hh[u]);
          }
        }
#pragma unroll
        for (int c = 0; c < CB; c++) {
          if (c >= nch) break;
          unsigned long long m[4];
          if (WR) {
#pragma unroll
            for (int u = 0; u < 4; u++) {
              // |u_j - u_i|^2 over 16-bit wrapped differences (saturating: far
              // pairs clamp at INT_MAX) against the lane's threshold
              int acc = 0;
#pragma unroll
              for (int k = 0; k < HW; k++) {
                const short2v dq = __builtin_bit_cast(short2v, cw[c][k]) -
                                   __builtin_bit_cast(short2v, (int)r[u][k]);
                acc = __builtin_amdgcn_sdot2(dq, dq, acc, true);
              }
              m[u] = __ballot(acc < tA[c]);
            }
          } else {
            // the four home atoms' products word by word, so that each dot
            // product's result is not needed by the next instruction; the
            // first in the three-operand form, so the lane's threshold needs
            // no copy into an accumulator register
            int acc[4];
#pragma unroll
            for (int u = 0; u < 4; u++)
              asm("v_dot2_i32_i16 %0, %1, %2, %3"
                  : "=v"(acc[u])
                  : "s"((int)r[u][0]), "v"(cw[c][0]), "v"(tA[c]));
#pragma unroll
            for (int k = 1; k < HW; k++)
#pragma unroll
              for (int u = 0; u < 4; u++)
                acc[u] = __builtin_amdgcn_sdot2(__builtin_bit_cast(short2v, (int)r[u][k]),
                                                __builtin_bit_cast(short2v, cw[c][k]), acc[u],
                                                false);
#pragma unroll
            for (int u = 0; u < 4; u++) m[u] = __ballot(acc[u] > r[u][HW]);
          }
#pragma unroll
          for (int u = 0; u < 4; u++) {
            mlo[c] = (unsigned)amdgcn_writelane((int)(unsigned)m[u], hh[u], (int)mlo[c]);
            mhi[c] = (unsigned)amdgcn_writelane((int)(unsigned)(m[u] >> 32), hh[u], (int)mhi[c]);
          }
        }
      }
    };

    // home atoms that can reach a row: gap to the neighbouring faces along
    // the first d-1 axes, one quantisation unit short per axis
    // the int16 offset of axis k from a home record's offset words (n_cell >= 3)
    auto oq = [](const int (&w)[HW + 1], int k) -> int {
      return (k % 2) ? (w[k / 2] >> 16) : (int)(short)(w[k / 2] & 0xffff);
    };
    auto row_keep = [&](const int (&og)[D - 1], unsigned long long& keep0,
                        unsigned long long& keep1) {
      int S0 = 0, S1 = 0;
#pragma unroll
      for (int k = 0; k < D - 1; k++) {
        const int o = og[k];
        int g0, g1;
        if (WR) {
          g0 = o ? qh0[k] : 0;
          g1 = o ? qh1[k] : 0;
        } else if (RAD == 1) {
          g0 = (kQScale / 2) - o * oq(ow0, k) - 1;
          g1 = (kQScale / 2) - o * oq(ow1, k) - 1;
          g0 = (o == 0 || g0 < 0) ? 0 : g0;
          g1 = (o == 0 || g1 < 0) ? 0 : g1;
        } else {
          // the near face of a subcell |o| away: (|o| - 1/2) sides from the centre
          const int ao = o < 0 ? -o : o;
          const int face = (kQScale / 2) * (2 * ao - 1);
          g0 = face - (o > 0 ? oq(ow0, k) : -oq(ow0, k)) - 1;
          g1 = face - (o > 0 ? oq(ow1, k) : -oq(ow1, k)) - 1;
          g0 = (o == 0 || g0 < 0) ? 0 : g0;
          g1 = (o == 0 || g1 < 0) ? 0 : g1;
        }
        S0 += g0 * g0;
        S1 += g1 * g1;
      }
      keep0 = __ballot(v0 && S0 < tc0);
      keep1 = two ? __ballot(v1 && S1 < tc1) : 0ull;
    };
    // candidate tt of a row of T atoms whose subcell slot r (stencil order)
    // holds the candidates from cum[r-1] on, atom tt + db[0] + ... + db[r]:
    // its record (an in-range atom for an empty lane) shifted by the subcell
    // offset as packed int16 adds; returns the atom, or -1 for an empty lane.
    // (The atom is a sum of increments rather than a pick among run bases:
    // the compiler turns such a pick into an indexed load from scratch.)
    auto cand_words = [&](int tt, int T, const int (&db)[NRS], const int (&cum)[NRS],
                          const int (&Dp)[HW], int (&cwc)[HW], int& tAc)
        __attribute__((always_inline)) -> int {
      const bool valid = tt < T;
      int j = tt + db[0], lastv = lshift(0);
#pragma unroll
      for (int r = 1; r < NRS; r++) {
        const bool past = tt >= cum[r - 1];
        j += past ? db[r] : 0;
        lastv = past ? lshift(r) : lastv;
      }
      const HDMD_GLOBAL int* src = gbl(qc16 + (size_t)(valid ? j : hb) * 8);
      if (WR) {
#pragma unroll
        for (int k = 0; k < HW; k++) cwc[k] = src[k];
        tAc = valid ? tq : -1;  // the lane's threshold; none for an empty lane
      } else {
        int A = 0;
#pragma unroll
        for (int k = 0; k < HW; k++) {
          const short2v q2 = __builtin_bit_cast(short2v, src[k]);
          const short2v o2 = __builtin_bit_cast(short2v, Dp[k] + (k == (D - 1) / 2 ? lastv : 0));
          const short2v r2 = q2 + o2;
          A = __builtin_amdgcn_sdot2(r2, r2, A, false);
          cwc[k] = __builtin_bit_cast(int, r2 + r2);
        }
        tAc = valid ? src[6] - A : -0x3fffffff;  // never passes for an empty lane
      }
      return valid ? j : -1;
    };
    // (T_j - A_j) + q_i.(2 q'_j) > |q_i|^2 - T_i  <=>  |q'_j - q_i|^2 < T_i + T_j
    // for the kept home atoms of both sets against nch chunks (LDS slots nb..)
    // The matrix-core form of the same tests (MF).  Per chunk and block of
    // 16 kept home atoms of a set (columns, compacted; their slots staged in
    // LDS in the chunk slots whose masks this call writes last), one
    // 16x16x16 product per block of 16 candidates (rows): entry 1/2 - S_ij,
    // whose sign bit is the test's outcome.  Lane l of the chunk holds the
    // candidate at position cpos(l), so that the sign bits of the four
    // result registers of the four candidate blocks, shifted in order into
    // one word per lane, come out in position order: lane 16g + j holds home
    // column j's bits of positions 16g .. 16g + 15.  A half swap per block,
    // and a select between the two blocks of a pair, join them into the two
    // 32-bit halves of each home atom's 64-bit mask (lane r: positions 0..31
    // of compacted home r of the pair, lane 32 + r: positions 32..63), which
    // are scattered at the end to the home atoms' slots (all others zero).
    auto test_chunks_mf = [&](unsigned long long keep0, unsigned long long keep1, int nch,
                              const int (&cw)[CB][HW], const int (&tA)[CB]) {
      constexpr int EW = 8;  // staged words per home atom: all 16 slots
      static_assert(CB * 128 * 8 >= 2 * 64 * 4 * EW, "two sets of staged home slots fit CB chunk slots");
      unsigned* stg = reinterpret_cast<unsigned*>(msk + nb * 128);  // free: nb + CB <= NB - 1
      const int nk0 = __builtin_popcountll(keep0), nk1 = __builtin_popcountll(keep1);
      // stage the kept atoms' slots at their rank; returns, in lanes j and
      // j + 32, the home lanes of compacted rows j (first) and 32 + j
      // (second): kept atoms go to their rank, the others after them, a
      // permutation of the lanes
      auto stage = [&](unsigned long long km, int nk, const int (&ow)[HW + 1], unsigned* st, int& s0,
                       int& s1) {
        const int rank = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(km >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((unsigned)km, 0u));
        const bool kept = (km >> lane) & 1ull;
        if (kept) {
          // (converted here, each time: hoisted out of the row loop, the
          // slots of both sets would hold 16 registers through it)
          int owl[HW + 1];
#pragma unroll
          for (int k = 0; k <= HW; k++) {
            owl[k] = ow[k];
            asm volatile("" : "+v"(owl[k]));
          }
          unsigned w[8];
          home_slots<D>(owl, owl[HW], w);
          uv4* e = reinterpret_cast<uv4*>(st + EW * rank);
          e[0] = uv4{w[0], w[1], w[2], w[3]};
          e[1] = uv4{w[4], w[5], w[6], w[7]};
        }
        const int dst = kept ? rank : nk + (lane - rank);
        const unsigned src = (unsigned)__builtin_amdgcn_ds_permute(dst * 4, lane);
        const auto sw = __builtin_amdgcn_permlane32_swap(src, src, false, false);
        s0 = (int)sw[0];
        s1 = (int)sw[1];
      };
      int sa0, sb0, sa1 = 0, sb1 = 0;
      stage(keep0, nk0, ow0, stg, sa0, sb0);
      if (nk1 > 0) stage(keep1, nk1, ow1, stg + 64 * EW, sa1, sb1);
      wave_lds_sync();
      const int q = lane >> 4;
      // one set's home blocks 2p and 2p + 1 (compacted homes 32p ..) against
      // the chunk's candidate blocks X: lane r < 32 receives positions 0..31
      // of home 32p + r, lane 32 + r its positions 32..63
      auto mf_pair = [&](const unsigned* st, int nk, int p, const hv4 (&X)[4])
          __attribute__((always_inline)) -> unsigned {
        unsigned R[2] = {0u, 0u};
#pragma unroll
        for (int h = 0; h < 2; h++) {
          const int b = 2 * p + h;
          if (16 * b >= nk) break;
          const uv2* e = reinterpret_cast<const uv2*>(st + EW * (16 * b + (lane & 15)));
          const hv4 Hb = __builtin_bit_cast(hv4, e[q]);
          unsigned P = 0u;
#pragma unroll
          for (int cb = 0; cb < 4; cb++) {
            const fv4 zero = {};
            const fv4 e4 = __builtin_amdgcn_mfma_f32_16x16x16f16(X[cb], Hb, zero, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; v++) P = __builtin_amdgcn_alignbit(P, __float_as_uint(e4[v]), 31u);
          }
          // lanes j, 16 + j: positions 0..31 of home j; lanes 32 + j, 48 + j: 32..63
          const auto sw = __builtin_amdgcn_permlane16_swap(P, P, false, false);
          R[h] = (unsigned)sw[0] | ((unsigned)sw[1] << 16);
        }
        return (lane & 16) ? R[1] : R[0];
      };
      unsigned r00[CB], r01[CB], r10[CB], r11[CB];  // set, pair of home blocks
#pragma unroll
      for (int c = 0; c < CB; c++) {
        r00[c] = r01[c] = r10[c] = r11[c] = 0u;
        if (c >= nch) continue;
        unsigned w[8];
        cand_slots<D>(cw[c], tA[c], w);
        // lane group g of block X[cb] takes slot words 2g, 2g + 1 of the
        // candidate in lane 16 cb + (lane mod 16): a 4x4 transpose of lane
        // groups and word pairs in two rounds of half swaps
        unsigned W[4][2];
#pragma unroll
        for (int t = 0; t < 2; t++) {
#pragma unroll
          for (int g = 0; g < 4; g++) W[g][t] = w[2 * g + t];
#pragma unroll
          for (int g = 0; g < 2; g++) {
            const auto sw = __builtin_amdgcn_permlane32_swap(W[g][t], W[g + 2][t], false, false);
            W[g][t] = sw[0];
            W[g + 2][t] = sw[1];
          }
#pragma unroll
          for (int g = 0; g < 4; g += 2) {
            const auto sw = __builtin_amdgcn_permlane16_swap(W[g][t], W[g + 1][t], false, false);
            W[g][t] = sw[0];
            W[g + 1][t] = sw[1];
          }
        }
        hv4 X[4];
#pragma unroll
        for (int g = 0; g < 4; g++) X[g] = __builtin_bit_cast(hv4, uv2{W[g][0], W[g][1]});
        if (nk0 > 0) r00[c] = mf_pair(stg, nk0, 0, X);
        if (nk0 > 32) r01[c] = mf_pair(stg, nk0, 1, X);
        if (nk1 > 0) r10[c] = mf_pair(stg + 64 * EW, nk1, 0, X);
        if (nk1 > 32) r11[c] = mf_pair(stg + 64 * EW, nk1, 1, X);
      }
      // (the stage has been read: one wave's LDS operations complete in order)
      unsigned* mw = reinterpret_cast<unsigned*>(msk);
      const int hf = lane >> 5, rj = lane & 31;
#pragma unroll
      for (int c = 0; c < CB; c++) {
        if (c >= nch) continue;
        const int base = (nb + c) * 128;
        msk[base + lane] = 0ull;
        if (two) msk[base + 64 + lane] = 0ull;
        if (rj < nk0) mw[2 * (base + sa0) + hf] = r00[c];
        if (32 + rj < nk0) mw[2 * (base + sb0) + hf] = r01[c];
        if (rj < nk1) mw[2 * (base + 64 + sa1) + hf] = r10[c];
        if (32 + rj < nk1) mw[2 * (base + 64 + sb1) + hf] = r11[c];
      }
      nb += nch;
    };
    auto test_chunks = [&](unsigned long long keep0, unsigned long long keep1, int nch,
                           const int (&cw)[CB][HW], const int (&tA)[CB]) {
      if constexpr (MF) {
        test_chunks_mf(keep0, keep1, nch, cw, tA);
        return;
      }
      unsigned m0lo[CB], m0hi[CB], m1lo[CB], m1hi[CB];
#pragma unroll
      for (int c = 0; c < CB; c++) m0lo[c] = m0hi[c] = m1lo[c] = m1hi[c] = 0u;
      test_set(keep0, ow0, hb, nch, cw, tA, m0lo, m0hi);
      test_set(keep1, ow1, hb + 64, nch, cw, tA, m1lo, m1hi);
#pragma unroll
      for (int c = 0; c < CB; c++) {
        if (c < nch) {
          msk[(nb + c) * 128 + lane] = ((unsigned long long)m0hi[c] << 32) | m0lo[c];
          msk[(nb + c) * 128 + 64 + lane] = ((unsigned long long)m1hi[c] << 32) | m1lo[c];
        }
      }
      nb += nch;
    };

    // one row of linked subcells, walked chunk by chunk
    auto do_row = [&](int row) __attribute__((always_inline)) {
      // A SIMD issues for its oldest waves first, so without this the waves
      // of a launch finish one by one and the last ones run alone, their
      // latencies exposed.  A wave's priority falls as it gets through its
      // rows: the waves that lag get the issue slots, and those of a SIMD
      // finish together.
      set_prio_by_progress(row, nrow);
      // The row's set-up is redone for each round of CB chunks, after any
      // pass of exact tests: nothing of it stays live across that pass.
      for (int k0 = 0;; k0 += CB * 64) {
        if (nb + CB > NB - 1) exact_pass();
        int Dp[HW], og[D - 1];
        const int P = row_base(row, Dp, og);
        unsigned long long keep0, keep1;
        row_keep(og, keep0, keep1);
        if ((keep0 | keep1) == 0) return;
        // the row's subcells in stencil order: (-RAD..+RAD) or, wrapped, (0, +1)
        // (all scalar loads issued before the first is used)
        int f[2 * NRS];
#pragma unroll
        for (int r = 0; r < NRS; r++) {
          f[2 * r] = lvalid(r) ? flat[P + lcell(r)] : 0;
          f[2 * r + 1] = lvalid(r) ? flat[P + lcell(r) + 1] : 0;
        }
        int db[NRS], cum[NRS], T = 0;
#pragma unroll
        for (int r = 0; r < NRS; r++) {
          // run r starts at atom f[2r] and takes candidates T.. (T before it)
          db[r] = r == 0 ? f[0] : (f[2 * r] - f[2 * r - 2]) - (cum[r - 1] - (r >= 2 ? cum[r - 2] : 0));
          T += f[2 * r + 1] - f[2 * r];
          cum[r] = T;
        }
        if (k0 >= T) return;
        const int nch = min(CB, (T - k0 + 63) / 64);
        int cw[CB][HW], tA[CB];
#pragma unroll
        for (int c = 0; c < CB; c++) {
          if (c >= nch) continue;
          cand[(nb + c) * 64 + cpos] = cand_words(k0 + c * 64 + cpos, T, db, cum, Dp, cw[c], tA[c]);
        }
        test_chunks(keep0, keep1, nch, cw, tA);
      }
    };

    if (sparse) {
      // CB consecutive rows that each fit one chunk share a round of
      // candidate loads and tests (the loads of all CB rows are in flight
      // together), tested against the home atoms kept by any of them; the
      // chunks stay in row order, so the lists and their order are those of
      // the row-by-row walk, which a group with a longer row takes instead
      for (int row = 0; row < nrow; row += CB) {
        set_prio_by_progress(row, nrow);
        if (nb + CB > NB - 1) exact_pass();
        // in phases, so that the scalar loads of all CB rows and then their
        // candidate loads are issued before any of them is waited for
        int P[CB], Dps[CB][HW];
        unsigned long long k0m = 0, k1m = 0;
#pragma unroll
        for (int c = 0; c < CB; c++) {
          const bool rv = row + c < nrow;
          int og[D - 1];
          P[c] = row_base(rv ? row + c : row, Dps[c], og);
          unsigned long long kp0, kp1;
          row_keep(og, kp0, kp1);
          k0m |= rv ? kp0 : 0ull;
          k1m |= rv ? kp1 : 0ull;
        }
        if ((k0m | k1m) == 0) continue;
        int fl[CB][2 * NRS];
#pragma unroll
        for (int c = 0; c < CB; c++) {
#pragma unroll
          for (int r = 0; r < NRS; r++) {
            fl[c][2 * r] = flat[P[c] + lcell(r)];
            fl[c][2 * r + 1] = flat[P[c] + lcell(r) + 1];
          }
        }
        int tmx = 0, Tr[CB];
#pragma unroll
        for (int c = 0; c < CB; c++) {
          Tr[c] = 0;
#pragma unroll
          for (int r = 0; r < NRS; r++) Tr[c] += fl[c][2 * r + 1] - fl[c][2 * r];
          tmx = max(tmx, Tr[c]);
        }
        if (tmx > 64) {
#pragma unroll 1
          for (int c = 0; c < CB && row + c < nrow; c++) do_row(row + c);
          continue;
        }
        int rw[CB][HW + 1];  // the candidate's offset words and its threshold share
        int jj[CB], lv[CB];
#pragma unroll
        for (int c = 0; c < CB; c++) {
          const int T = row + c < nrow ? Tr[c] : 0;
          int j = fl[c][0] + cpos, acc = fl[c][1] - fl[c][0];
          lv[c] = lshift(0);
#pragma unroll
          for (int r = 1; r < NRS; r++) {
            if (cpos >= acc) {
              j = fl[c][2 * r] - acc + cpos;
              lv[c] = lshift(r);
            }
            acc += fl[c][2 * r + 1] - fl[c][2 * r];
          }
          jj[c] = cpos < T ? j : -1;
          const HDMD_GLOBAL int* src = gbl(qc16 + (size_t)(cpos < T ? j : hb) * 8);
#pragma unroll
          for (int k = 0; k < HW; k++) rw[c][k] = src[k];
          rw[c][HW] = src[6];
        }
        int cw[CB][HW], tA[CB];
#pragma unroll
        for (int c = 0; c < CB; c++) {
          int A = 0;
#pragma unroll
          for (int k = 0; k < HW; k++) {
            const short2v q2 = __builtin_bit_cast(short2v, rw[c][k]);
            const short2v o2 =
                __builtin_bit_cast(short2v, Dps[c][k] + (k == (D - 1) / 2 ? lv[c] : 0));
            const short2v r2 = q2 + o2;
            A = __builtin_amdgcn_sdot2(r2, r2, A, false);
            cw[c][k] = __builtin_bit_cast(int, r2 + r2);
          }
          tA[c] = jj[c] >= 0 ? rw[c][HW] - A : -0x3fffffff;  // never passes for an empty lane
          cand[(nb + c) * 64 + cpos] = jj[c];
        }
        test_chunks(k0m, k1m, CB, cw, tA);
      }
    } else {
      for (int row = 0; row < nrow; row++) do_row(row);
    }
    exact_pass();
    if (v0) {
      s->nlen[i0] = len0;
      rowmax = max(rowmax, len0);
    }
    if (v1) {
      s->nlen[i1] = len1;
      rowmax = max(rowmax, len1);
    }
  }
  rowmax = wave_max_i(rowmax);
  if (lane == 0 && rowmax > 0) {
    atomicMax(&s->max_row, rowmax);
    if (rowmax > W) atomicOr(&s->err, ERR_OVERFLOW);
  }
}

template <int D, int G, bool WR, int RAD = 1, bool MF = false>
__global__ __launch_bounds__(64 * G, G >= 8 ? 16 / G : 8) void k_build_t(KArgs a) {
  // per wave: survivor masks of up to 128 home atoms and the candidates of 8 chunks
  __shared__ unsigned long long msk_all[G][8 * 128];
  __shared__ int cand_all[G][8 * 64];
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int t = xcd_tile(blockIdx.x, gridDim.x);; t += gridDim.x) {
    SysDev* s;
    int hc;
    if (!fetch_cell_tile(a, t, s, hc)) break;
    s = uniform_ptr(s);
    hc = uniform_int(hc);
    if (!running(s) || !need_rebuild(s) || uniform_int(s->reach) != RAD) {
      if (a.single) break;  // one system: the same for every tile
      continue;
    }
    build_t_tile<D, G, WR, RAD, MF>(s, hc, wv, msk_all[wv], cand_all[wv]);
  }
}

// ---------------------------------------------------------------------------
// pair forces over one Verlet row (Sec. II.B getforce)
// ---------------------------------------------------------------------------
// F_i = sum_j fc (x_i - x_j) with fc = -U'(r)/r for r < c sigma_ij;
// e_i = 1/2 sum_j U(r).
// 1/x from the hardware reciprocal estimate and two Newton-Raphson steps
// (each squares the relative error): within an ulp or two of 1/x.
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return r;
}

// 1/sqrt(x) from the hardware estimate and two Newton-Raphson steps
// y <- y (3/2 - x y^2 / 2).
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = __builtin_fma(y, __builtin_fma(-hx * y, y, 0.5), y);
  y = __builtin_fma(y, __builtin_fma(-hx * y, y, 0.5), y);
  return y;
}

// MORSE selects the truncated, shifted Morse form at compile time: its
// exponential needs registers that would otherwise count against every force
// loop (WCA and harmonic share the other instantiation, switched at run time).
template <bool MORSE>
__device__ inline void pair_f64(int pot, double eps, double ma, double r2, double sij, double& fc,
                                double& u) {
  if constexpr (MORSE) {  // truncated, shifted Morse (Sec. II.A, eq. morsepot)
    // with t = e^{-a(r - sigma)}: U = eps (t - 1)^2, -U'(r)/r = 2 a eps t (t - 1) / r
    const double ir = rsqrt_nr(r2);  // 1/r
    const double t = exp(-ma * (r2 * ir - sij));
    fc = 2.0 * ma * eps * t * (t - 1.0) * ir;
    u = eps * (t - 1.0) * (t - 1.0);
    (void)pot;
  } else if (pot == 0) {  // WCA
    const double inv = recip(r2);
    const double s2 = sij * sij * inv;
    const double s6 = s2 * s2 * s2;
    fc = 24.0 * eps * (2.0 * s6 * s6 - s6) * inv;
    u = 4.0 * eps * (s6 * s6 - s6) + eps;
  } else {         // harmonic soft spheres
    const double ir = rsqrt_nr(r2);  // 1/r
    const double is = recip(sij);
    const double g = 1.0 - (r2 * ir) * is;
    fc = eps * g * is * ir;
    u = 0.5 * eps * g * g;
  }
}

// SWAP Monte Carlo (Sec. II.D).  Attempt k exchanges the diameters of the
// atoms with caller ids pairs[2k] and pairs[2k+1]; the energies before and
// after (eq. ebefore) sum the pair terms of both atoms with every partner
// inside the cutoff; the pair of the two atoms keeps its diameter and
// cancels.  Kept on the Metropolis rule dE <= 0 or u_k < exp(-dE/T).
// The attempts keep their serial meaning (each sees the diameters the
// earlier ones left) but run in batches: every attempt of a batch gets its
// dE from the diameters at the batch's start (one workgroup each), then one
// workgroup walks the batch in order and settles an attempt unless an
// earlier attempt of the batch that was kept or put off involves an atom
// within the interaction range c sigma_max of one of its atoms (then its dE
// could differ: it is put off to the next batch, ahead of the unbatched
// ones).  Settled attempts commute with the put-off ones they do not touch,
// so the outcome is that of the serial walk.  Diameters live in the records
// (read past the L1, as a kept swap rewrites them) and in diam (caller
// order).
__device__ inline double sig_get(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void sig_put(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// dE of exchanging the diameters of the atoms in slots pi and pj, with the
// current diameters, by a whole workgroup of up to 16 waves: the linked
// subcells of each atom's subcell (all subcells when n_cell <= 2) in groups
// of 64 per wave (a group's bounds loaded by its lanes at once), the lanes
// striding over a subcell's atoms, the wave sums added in wave order.
// Every thread returns the same value.
template <int D>
__device__ inline double swap_de(const SysDev* s, int pi, int pj, double (*red)[16], double& si_out,
                                 double& sj_out) {
  constexpr int DR = Dims<D>::DR;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int nc = s->ncell;
  const double L = s->L, h = s->hL, cut = s->cutoff, eps = s->eps, ma = s->morse_a;
  const int pot = s->potential;
  const bool morse = pot == kPotMorse;
  double* xb = s->x[s->xcur];
  const int* flat = s->cell_flat;
  // the linked subcells: offsets -reach..+reach per axis, or every subcell
  // once where an axis has fewer than 2 reach + 1
  const int reach = s->reach, rx = nc < 2 * reach + 1 ? nc : 2 * reach + 1;
  const bool dedup = nc < 2 * reach + 1;
  int nst = 1;
  for (int k = 0; k < D; k++) nst *= rx;
  const double si = sig_get(xb + (size_t)pi * DR + D), sj = sig_get(xb + (size_t)pj * DR + D);
  si_out = si;
  sj_out = sj;
  double eb = 0.0, ea = 0.0;
  if (pi != pj) {
    for (int side = 0; side < 2; side++) {
      const int p = side ? pj : pi, o = side ? pi : pj;
      const double sa = side ? sj : si, sb = side ? si : sj;  // p's diameter before, after
      double xp[D];
      load_x<D>(xb, p, xp);
      int cd[D];
      {
        int r = flat_cell<D>(s, xp);
        for (int a = D - 1; a >= 0; a--) {
          cd[a] = r % nc;
          r /= nc;
        }
      }
      for (int t0 = wv * 64; t0 < nst; t0 += 64 * nwv) {
        int cs = 0, ce = 0;
        const int t = t0 + lane;
        if (t < nst) {
          int cell = 0, r = t, mult = 1;
          for (int a = D - 1; a >= 0; a--) {
            int ca;
            if (dedup) {
              ca = r % nc;
              r /= nc;
            } else {
              ca = cd[a] + r % rx - reach;
              r /= rx;
              ca = ca < 0 ? ca + nc : (ca >= nc ? ca - nc : ca);
            }
            cell += ca * mult;
            mult *= nc;
          }
          cs = flat[cell];
          ce = flat[cell + 1];
        }
        const int ng = min(64, nst - t0);
        for (int g = 0; g < ng; g++) {
          const int q1 = __builtin_amdgcn_readlane(ce, g);
          for (int q = __builtin_amdgcn_readlane(cs, g) + lane; q < q1; q += 64) {
            if (q == p) continue;
            double xq[D];
            load_x<D>(xb, q, xq);
            const double sq = sig_get(xb + (size_t)q * DR + D);
            double r2 = 0.0;
            for (int a = 0; a < D; a++) {
              const double dx = min_image(xq[a] - xp[a], L, h);
              r2 = __builtin_fma(dx, dx, r2);
            }
            double fc, uu;
            const double s_b = 0.5 * (sa + sq);
            if (r2 < (cut * s_b) * (cut * s_b)) {
              if (morse) pair_f64<true>(pot, eps, ma, r2, s_b, fc, uu);
              else pair_f64<false>(pot, eps, ma, r2, s_b, fc, uu);
              eb += uu;
            }
            // after the exchange the partner carries p's old diameter
            const double s_a = 0.5 * (sb + (q == o ? sa : sq));
            if (r2 < (cut * s_a) * (cut * s_a)) {
              if (morse) pair_f64<true>(pot, eps, ma, r2, s_a, fc, uu);
              else pair_f64<false>(pot, eps, ma, r2, s_a, fc, uu);
              ea += uu;
            }
          }
        }
      }
    }
  }
  eb = wave_sum(eb);
  ea = wave_sum(ea);
  if (lane == 0) {
    red[0][wv] = eb;
    red[1][wv] = ea;
  }
  __syncthreads();
  eb = 0.0;
  ea = 0.0;
  for (int w = 0; w < nwv; w++) {
    eb += red[0][w];
    ea += red[1][w];
  }
  __syncthreads();  // red[] is free again
  return pi == pj ? 0.0 : ea - eb;
}

// The batch of a round: the nput attempts put off by the previous round
// (off_in, in order) followed by the attempts cursor, cursor + 1, ... not yet
// begun; kSwapBatch of them at most.  ctl[0] = nput, ctl[2] = cursor.
__device__ inline int swap_batch_size(const long long* ctl, int64_t n_att) {
  const long long rest = (long long)n_att - ctl[2];
  const long long nb = ctl[0] + rest;
  return (int)(nb < kSwapBatch ? nb : kSwapBatch);
}
__device__ inline int swap_attempt(const long long* ctl, const int32_t* off_in, int b) {
  const int nput = (int)ctl[0];
  return b < nput ? off_in[b] : (int)(ctl[2] + (b - nput));
}

// dE of the round's attempts, one workgroup each, with the two diameters it
// was taken with: de[3b] = dE, de[3b+1], de[3b+2] = the diameters of the
// first and the second atom.  conf[b][w] bit c: attempt b' = 64 w + c < b
// has an atom within c sigma_max of an atom of attempt b.
template <int D>
__global__ __launch_bounds__(1024) void k_swap_de(const SysDev* s, const long long* __restrict__ ctl,
                                                  const int32_t* __restrict__ off_in, int64_t n_att,
                                                  const int32_t* __restrict__ pairs,
                                                  const int32_t* __restrict__ slot_of,
                                                  double* __restrict__ de,
                                                  unsigned long long* __restrict__ conf) {
  __shared__ double red[2][16];
  const int b = blockIdx.x;
  const int nb = swap_batch_size(ctl, n_att);
  if (b >= nb) return;
  const int k = swap_attempt(ctl, off_in, b);
  const int pi = slot_of[pairs[2 * k]], pj = slot_of[pairs[2 * k + 1]];
  {
    const double* xb = s->x[s->xcur];
    const double L = s->L, h = s->hL;
    const double rr = s->cutoff * s->sigma_max, r2max = rr * rr * (1.0 + 1e-12);
    const int t = threadIdx.x;
    bool near = false;
    if (t < b) {
      const int k2 = swap_attempt(ctl, off_in, t);
      const int q2[2] = {slot_of[pairs[2 * k2]], slot_of[pairs[2 * k2 + 1]]};
      for (int e = 0; e < 4; e++) {
        double xa[D], xc[D];
        load_x<D>(xb, (e >> 1) ? pj : pi, xa);
        load_x<D>(xb, q2[e & 1], xc);
        double r2 = 0.0;
        for (int a = 0; a < D; a++) {
          const double dx = min_image(xa[a] - xc[a], L, h);
          r2 += dx * dx;
        }
        near = near || r2 <= r2max;
      }
    }
    const unsigned long long m = __ballot(near);
    if (t < kSwapBatch && (t & 63) == 0) conf[(size_t)b * (kSwapBatch / 64) + (t >> 6)] = m;
  }
  double si, sj;
  const double d = swap_de<D>(s, pi, pj, red, si, sj);
  if (threadIdx.x == 0) {
    de[3 * b] = d;
    de[3 * b + 1] = si;
    de[3 * b + 2] = sj;
  }
}

// Settles the round's batch in order (see above), applies the kept exchanges,
// and writes the attempts put off to off_out; ctl[0] = their number, ctl[2]
// advances past the attempts begun, ctl[1] += exchanges kept.
template <int D>
__global__ __launch_bounds__(1024) void k_swap_settle(SysDev* s, long long* __restrict__ ctl,
                                                      const int32_t* __restrict__ off_in,
                                                      int32_t* __restrict__ off_out, int64_t n_att,
                                                      const int32_t* __restrict__ pairs,
                                                      const double* __restrict__ u, double T,
                                                      const int32_t* __restrict__ slot_of,
                                                      const double* __restrict__ de,
                                                      const unsigned long long* __restrict__ cfg,
                                                      int32_t* __restrict__ acc,
                                                      double* __restrict__ diam) {
  constexpr int DR = Dims<D>::DR, NW = kSwapBatch / 64;
  __shared__ unsigned long long conf[kSwapBatch][NW];
  __shared__ int put_off[kSwapBatch];
  __shared__ int att[kSwapBatch], cid[kSwapBatch][2], slot[kSwapBatch][2];
  __shared__ double thr[kSwapBatch];  // the Metropolis decision as 0 / 1
  const int tid = threadIdx.x;
  const int nb = swap_batch_size(ctl, n_att);
  if (nb <= 0) return;
  const int nput = (int)ctl[0];
  double* xb = s->x[s->xcur];
  for (int t = tid; t < nb * NW; t += blockDim.x) conf[t / NW][t % NW] = cfg[t];
  for (int t = tid; t < 2 * nb; t += blockDim.x) {
    const int b = t >> 1, e = t & 1, k = swap_attempt(ctl, off_in, b);
    const int c = pairs[2 * k + e], q = slot_of[c];
    cid[b][e] = c;
    slot[b][e] = q;
    if (e == 0) {
      att[b] = k;
      // the decision of an attempt that settles (its dE stands)
      const double d = de[3 * b];
      thr[b] = (d <= 0.0 || u[k] < exp(-d / T)) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long blk[NW];
    for (int w = 0; w < NW; w++) blk[w] = 0;
    int noff = 0;
    long long kept = 0;
    for (int b = 0; b < nb; b++) {
      bool hit = false;
      for (int w = 0; w < NW; w++) hit = hit || (conf[b][w] & blk[w]) != 0;
      const int k = att[b];
      if (hit) {
        put_off[noff++] = k;
        blk[b >> 6] |= 1ull << (b & 63);
        continue;
      }
      const bool ok = thr[b] != 0.0;
      if (acc) acc[k] = ok ? 1 : 0;
      if (ok) {
        // a settled attempt's atoms were not touched earlier in the batch, so
        // their diameters are the ones its dE was taken with
        const double si = de[3 * b + 1], sj = de[3 * b + 2];
        sig_put(xb + (size_t)slot[b][0] * DR + D, sj);
        sig_put(xb + (size_t)slot[b][1] * DR + D, si);
        diam[cid[b][0]] = sj;
        diam[cid[b][1]] = si;
        kept++;
        blk[b >> 6] |= 1ull << (b & 63);
      }
    }
    for (int b = 0; b < noff; b++) off_out[b] = put_off[b];
    ctl[2] += nb - nput;
    ctl[0] = noff;
    ctl[1] += kept;
  }
}

// Own atom's data as the force loop needs it.
template <int D, bool MIX>
struct Own {
  double x[D];  // FP64 coordinates
  double sg;
  int u[D];     // fixed-point coordinates (mixed)
};

// Partial force of lane `sub` of the LPA lanes that share slot i: entries
// k = sub, sub + LPA, ...; the next group's row indices are fetched before
// the current group's records are used.  The LPA partial sums are combined
// with the same butterfly on every lane of the group.
template <int D, bool MIX, int LPA, typename FT, bool MORSE>
__device__ inline void force_part(const SysDev* s, int i, int sub, const Own<D, MIX>& me,
                                  FT (&F)[D], double& e, double& w, double& z) {
  constexpr int U = MIX ? 4 : 2;
  const int npad = s->npad;
  const int len = min(gbl(s->nlen)[i], s->width);
  const HDMD_GLOBAL int* __restrict__ nl = gbl(s->nl);
  const double L = s->L, c = s->cutoff, eps = s->eps, invL = 1.0 / L, ma = s->morse_a;
  const int pot = s->potential;
  const double* __restrict__ xb = s->x[s->xcur];
  const int32_t* __restrict__ qb = MIX ? s->q[s->xcur] : nullptr;
  const double fxinv = s->fxinv;
  // forces are summed in FP64 in both forms (the precision form stores them
  // as FP32): summing ~10^2-10^3 terms of mixed sign in FP32 would lose more
  // than 1e-5 of F_rms at high overlap
  double Fs[D];
#pragma unroll
  for (int k = 0; k < D; k++) Fs[k] = 0.0;
  e = 0.0;
  w = 0.0;
  z = 0.0;
  // row entries are read unconditionally from a clamped (in-bounds) slot and
  // masked afterwards, so the loads issue without branches and the wait for
  // the current group does not also wait for the prefetched one
  const int wm1 = s->width - 1;
  int jn[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int kk = sub + u * LPA;
    const int raw = nl[(size_t)min(kk, wm1) * npad + i];
    jn[u] = kk < len ? raw : -1;
  }
  for (int k0 = sub; k0 < len; k0 += U * LPA) {
    int jj[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      jj[u] = jn[u];
      const int kk = k0 + (U + u) * LPA;
      const int raw = nl[(size_t)min(kk, wm1) * npad + i];
      jn[u] = kk < len ? raw : -1;
    }
    if (!MIX) {
      double xj[U][D], sj[U];
#pragma unroll
      for (int u = 0; u < U; u++) load_rec<D>(xb, jj[u] >= 0 ? jj[u] : i, xj[u], sj[u]);
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (jj[u] < 0) continue;
        const double sij = 0.5 * (me.sg + sj[u]);
        const double rc = c * sij;
        double dx[D];
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; k++) {
          dx[k] = near_image(xj[u][k] - me.x[k], L, invL);
          r2 = __builtin_fma(dx[k], dx[k], r2);
        }
        if (r2 < rc * rc) {
          double fc, uu;
          pair_f64<MORSE>(pot, eps, ma, r2, sij, fc, uu);
#pragma unroll
          for (int k = 0; k < D; k++) Fs[k] -= fc * dx[k];
          e += 0.5 * uu;
          w += 0.5 * fc * r2;
          z += 1.0;
        }
      }
    } else {
      // mixed: exact integer displacements; distance, pair coefficient and
      // force sum in FP64 (stored as FP32 by the caller)
      int uj[U][D];
      double sj[U];
#pragma unroll
      for (int u = 0; u < U; u++) load_q<D>(qb, jj[u] >= 0 ? jj[u] : i, uj[u], sj[u]);
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (jj[u] < 0) continue;
        const double sij = 0.5 * (me.sg + sj[u]);
        const double rc = c * sij;
        double dx[D];
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; k++) {
          dx[k] = (double)(int)(uj[u][k] - me.u[k]) * fxinv;  // two's complement = minimum image
          r2 = __builtin_fma(dx[k], dx[k], r2);
        }
        if (r2 < rc * rc) {
          double fc, uu;
          pair_f64<MORSE>(pot, eps, ma, r2, sij, fc, uu);
#pragma unroll
          for (int k = 0; k < D; k++) Fs[k] -= fc * dx[k];
          e += 0.5 * uu;
          w += 0.5 * fc * r2;
          z += 1.0;
        }
      }
    }
  }
#pragma unroll
  for (int o = 1; o < LPA; o <<= 1) {
#pragma unroll
    for (int k = 0; k < D; k++) Fs[k] += __shfl_xor(Fs[k], o, 64);
    e += __shfl_xor(e, o, 64);
    w += __shfl_xor(w, o, 64);
    z += __shfl_xor(z, o, 64);
  }
#pragma unroll
  for (int k = 0; k < D; k++) F[k] = FT(Fs[k]);
}

// Partial force of one lane per atom (the whole row), with the neighbour
// records staged through LDS.  A gather in which every lane loads its own
// neighbour's record touches as many cache lines per load instruction as
// there are lanes; here the wave loads the records of R row entries of all 64
// lanes cooperatively (RB/16 lanes share one record, one 16-byte piece each,
// so an instruction covers 16 / 32 / 64 whole records) straight into LDS
// (global_load_lds_dwordx4), then every lane reads its own records back.  The
// pairs are summed in row order, exactly as force_part does, so the results
// are the same bits.  The loop runs to the longest row of the wave; the
// pieces of record r sit rotated by r in its LDS slot so that the lanes'
// reads spread over the banks.  stage: kStage16 16-byte slots of LDS.
constexpr int kStage16 = 512;  // 8 KiB per wave

template <int D, bool MIX>
struct StageGeom {
  static constexpr int RB = MIX ? Dims<D>::DQ * 4 : Dims<D>::DR * 8;  // record bytes
  static constexpr int PR = RB / 16;                                  // pieces per record
  static constexpr int R = kStage16 / (64 * PR);                      // rows entries per pass
};

template <int D, bool MIX, typename FT, bool MORSE>
__device__ inline void force_part_lds(const SysDev* s, int i, bool vi, const Own<D, MIX>& me,
                                      FT (&F)[D], double& e, double& w, double& z, vd2* stage) {
  typedef StageGeom<D, MIX> G;
  constexpr int PR = G::PR, R = G::R, RPI = 64 / PR;  // records per load instruction
  static_assert(R >= 1 && R * 64 * PR <= kStage16, "stage size");
  const int lane = threadIdx.x & 63;
  const int npad = s->npad, W = s->width;
  const int len = vi ? min(gbl(s->nlen)[i], W) : 0;
  const int mx = uniform_int(wave_max_i(len));
  const HDMD_GLOBAL int* __restrict__ nl = gbl(s->nl);
  const double L = s->L, c = s->cutoff, eps = s->eps, invL = 1.0 / L, ma = s->morse_a;
  const int pot = s->potential;
  const char* __restrict__ base =
      MIX ? reinterpret_cast<const char*>(s->q[s->xcur]) : reinterpret_cast<const char*>(s->x[s->xcur]);
  const double fxinv = s->fxinv;
  double Fs[D];
#pragma unroll
  for (int k = 0; k < D; k++) Fs[k] = 0.0;
  e = 0.0;
  w = 0.0;
  z = 0.0;
  for (int k0 = 0; k0 < mx; k0 += R) {
    int j[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int kk = k0 + r;
      const int raw = nl[(size_t)min(kk, W - 1) * npad + i];
      j[r] = kk < len ? raw : -1;
    }
    wave_lds_sync();  // the previous pass's reads of the stage are done
#pragma unroll
    for (int r = 0; r < R; r++) {
#pragma unroll
      for (int q = 0; q < PR; q++) {
        // lane t loads piece ((t % PR) - rec) mod PR of record rec = q RPI + t / PR
        // of this round into slot t % PR: LDS byte 16 t of the instruction's 1 KiB
        const int rec = q * RPI + lane / PR;
        const int jr = PR == 1 ? j[r] : __shfl(j[r], rec, 64);
        const int piece = ((lane % PR) - rec) & (PR - 1);
        const char* src = base + (size_t)(jr >= 0 ? jr : 0) * G::RB + 16 * piece;
        __builtin_amdgcn_global_load_lds((const void*)src, (void*)(stage + (r * PR + q) * 64), 16, 0,
                                         0);
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < R; r++) {
      // own record of this round: pieces p at slots (p + lane) mod PR
      const vd2* rec = stage + r * PR * 64 + lane * PR;
      if (!MIX) {
        double xj[D], sj = 0.0;
        vd2 pc[PR];
#pragma unroll
        for (int p = 0; p < PR; p++) pc[p] = rec[(p + lane) & (PR - 1)];
#pragma unroll
        for (int k = 0; k < D; k++) xj[k] = (k & 1) ? pc[k >> 1].y : pc[k >> 1].x;
        sj = (D & 1) ? pc[D >> 1].y : pc[D >> 1].x;
        if (j[r] < 0) continue;
        const double sij = 0.5 * (me.sg + sj);
        const double rc = c * sij;
        double dx[D];
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; k++) {
          dx[k] = near_image(xj[k] - me.x[k], L, invL);
          r2 = __builtin_fma(dx[k], dx[k], r2);
        }
        if (r2 < rc * rc) {
          double fc, uu;
          pair_f64<MORSE>(pot, eps, ma, r2, sij, fc, uu);
#pragma unroll
          for (int k = 0; k < D; k++) Fs[k] -= fc * dx[k];
          e += 0.5 * uu;
          w += 0.5 * fc * r2;
          z += 1.0;
        }
      } else {
        constexpr int SQ = Dims<D>::SQ;
        int v[4 * PR];
#pragma unroll
        for (int p = 0; p < PR; p++) {
          const vi4 t = reinterpret_cast<const vi4*>(rec)[(p + lane) & (PR - 1)];
          v[4 * p] = t.x;
          v[4 * p + 1] = t.y;
          v[4 * p + 2] = t.z;
          v[4 * p + 3] = t.w;
        }
        const double sj = __longlong_as_double(
            (long long)(((unsigned long long)(unsigned)v[SQ + 1] << 32) | (unsigned)v[SQ]));
        if (j[r] < 0) continue;
        const double sij = 0.5 * (me.sg + sj);
        const double rc = c * sij;
        double dx[D];
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; k++) {
          dx[k] = (double)(int)(v[k] - me.u[k]) * fxinv;  // two's complement = minimum image
          r2 = __builtin_fma(dx[k], dx[k], r2);
        }
        if (r2 < rc * rc) {
          double fc, uu;
          pair_f64<MORSE>(pot, eps, ma, r2, sij, fc, uu);
#pragma unroll
          for (int k = 0; k < D; k++) Fs[k] -= fc * dx[k];
          e += 0.5 * uu;
          w += 0.5 * fc * r2;
          z += 1.0;
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < D; k++) F[k] = FT(Fs[k]);
}

template <int D, bool MIX>
__device__ inline void load_own(const SysDev* s, int i, Own<D, MIX>& me) {
  load_rec<D>(s->x[s->xcur], i, me.x, me.sg);
  if (MIX) {
    double sgq;
    load_q<D>(s->q[s->xcur], i, me.u, sgq);
  }
}

template <bool MIX>
struct VType {
  typedef double T;
};
template <>
struct VType<true> {
  typedef float T;
};

// Per-tile partial sums of the slots in `use` (a bit per Part; the others
// are left as they are and read by nobody): each wave reduces its lanes, then
// (LPA > 1) thread 0 adds the waves of the tile in order (deterministic for a
// given LPA).  `use` is uniform over the block.
constexpr unsigned kUseForce = (1u << P_PE) | (1u << P_FV) | (1u << P_FF) | (1u << P_VV) |
                               (1u << P_FMAX2);
constexpr unsigned kUseStep = (1u << P_PE) | (1u << P_KE) | (1u << P_FMAX2) | (1u << P_VIR) |
                              (1u << P_NC);
constexpr unsigned kUseDisp = (1u << P_M2) | (1u << P_M4) | (1u << P_OV);

template <int LPA>
__device__ inline void tile_partials(double* dst, double (&vals)[kPart], double& maxv,
                                     double* sh, unsigned use) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int p = 0; p < kPart; p++)
    if (p != P_FMAX2 && (use >> p & 1u)) vals[p] = wave_sum(vals[p]);
  maxv = wave_max(maxv);
  if (LPA == 1) {
    if (lane == 0) {
#pragma unroll
      for (int p = 0; p < kPart; p++)
        if (use >> p & 1u) dst[p] = p == P_FMAX2 ? maxv : vals[p];
    }
    return;
  }
  if (lane == 0) {
#pragma unroll
    for (int p = 0; p < kPart; p++)
      if (use >> p & 1u) sh[w * kPart + p] = p == P_FMAX2 ? maxv : vals[p];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int p = 0; p < kPart; p++) {
      if (!(use >> p & 1u)) continue;
      double acc = sh[p];
      for (int ww = 1; ww < LPA; ww++)
        acc = p == P_FMAX2 ? fmax(acc, sh[ww * kPart + p]) : acc + sh[ww * kPart + p];
      dst[p] = acc;
    }
  }
  __syncthreads();
}

// Forces (stored in s->f) with the tile's energy and, for FIRE, the power
// P = F.v, |F|^2, |v|^2 and max_i |F_i|^2 partial sums.
// One atom tile's forces (stored in s->f) with the tile's energy and, for
// FIRE, the power P = F.v, |F|^2, |v|^2 and max_i |F_i|^2 partial sums.
// The force kernels serve the systems of one potential class: MORSE, or WCA
// and harmonic (run-time switch); of one precision form; and of one number
// of lanes per atom.
__device__ inline bool kernel_serves(const SysDev* s, bool mix, bool morse, int lpa) {
  return (s->precision != 0) == mix && (s->potential == kPotMorse) == morse && s->lpa == lpa;
}

template <int D, bool MIX, int LPA, bool MORSE>
__device__ inline void force_tile(SysDev* s, int tile, int fire, double* sh, vd2* stage) {
  typedef typename VType<MIX>::T FT;
  const int sub = threadIdx.x % LPA, slot = threadIdx.x / LPA;
  const int i = tile * kTile + slot;
  const int n = s->n, npad = s->npad, pc = s->pcur;
  const bool vi = i < n;
  const int ii = vi ? i : 0;
  Own<D, MIX> me;
  load_own<D, MIX>(s, ii, me);
  FT F[D];
  double e, w, z;
  if constexpr (LPA == 1) force_part_lds<D, MIX, FT, MORSE>(s, ii, vi, me, F, e, w, z, stage);
  else force_part<D, MIX, LPA, FT, MORSE>(s, ii, sub, me, F, e, w, z);
  double vals[kPart], mx = 0.0;
#pragma unroll
  for (int p = 0; p < kPart; p++) vals[p] = 0.0;
  if (vi && sub == 0) {
    FT* fo = reinterpret_cast<FT*>(s->f);
    const FT* v = reinterpret_cast<const FT*>(s->v[pc]);
    double fv = 0.0, ff = 0.0, vv = 0.0;
#pragma unroll
    for (int k = 0; k < D; k++) {
      fo[(size_t)k * npad + i] = F[k];
      if (fire) {
        const double fk = (double)F[k], vk = (double)v[(size_t)k * npad + i];
        fv += fk * vk;
        ff += fk * fk;
        vv += vk * vk;
      }
    }
    vals[P_PE] = e;
    vals[P_FV] = fv;
    vals[P_FF] = ff;
    vals[P_VV] = vv;
    mx = ff;
  }
  tile_partials<LPA>(s->part + (size_t)tile * kPart, vals, mx, sh, kUseForce);
}

template <int D, bool MIX, int LPA, bool MORSE>
__global__ __launch_bounds__(kTile * LPA) void k_force(KArgs a, int fire) {
  __shared__ double sh[LPA * kPart];
  __shared__ vd2 stage[LPA == 1 ? kStage16 : 1];
  for (int t = xcd_tile(blockIdx.x, gridDim.x);; t += gridDim.x) {
    SysDev* s;
    int tile;
    if (!fetch_atom_tile(a, t, s, tile)) break;
    if (!running(s) || !kernel_serves(s, MIX, MORSE, LPA)) continue;
    if (fire && s->mode != MODE_FIRE) continue;
    force_tile<D, MIX, LPA, MORSE>(s, tile, fire, sh, stage);
  }
}

// Fused velocity-Verlet step (kick-drift-kick leapfrog, Sec. II.B):
//   F = F(x^n); v^n = lambda (v^(n-1/2) + dt/2 F) (skipped at step 0, where v
//   is the full-step velocity; lambda is the Berendsen factor from the
//   previous full step's temperature, 1 without a thermostat: the paper folds
//   the thermostat into this kick); record KE(v^n), PE(x^n); v^(n+1/2) = v^n + dt/2 F;
//   x^(n+1) = wrap(x^n + dt v^(n+1/2)) into the other record buffer;
//   max_i |x^(n+1)_i - x_ref,i|^2 for the rebuild trigger (skin/2).
// At the closing step (n == nsteps) only the second kick is applied.
// On steps that record a thermo row, the unwrapped displacement since the
// run's start, Delta_i = disp_i + (x^n_i - x_ref,i), gives |Delta|^2,
// |Delta|^4 and the overlap term Theta(0.1 d - |Delta|) (Sec. II.E, eqs. ngp
// and fov); disp_i is advanced at each rebuild, so other steps read nothing.
template <int D, bool MIX, int LPA, bool MORSE>
__global__ __launch_bounds__(kTile * LPA) void k_step(KArgs a) {
  typedef typename VType<MIX>::T VT;
  __shared__ double sh[LPA * kPart];
  __shared__ vd2 stage[LPA == 1 ? kStage16 : 1];
  const int sub = threadIdx.x % LPA, slot = threadIdx.x / LPA;
  for (int t = xcd_tile(blockIdx.x, gridDim.x);; t += gridDim.x) {
    SysDev* s;
    int tile;
    if (!fetch_atom_tile(a, t, s, tile)) break;
    if (!running(s) || s->mode != MODE_MD || !kernel_serves(s, MIX, MORSE, LPA)) continue;
    const int i = tile * kTile + slot;
    const int n = s->n, npad = s->npad, pc = s->pcur, cur = s->xcur;
    const bool vi = i < n;
    const int ii = vi ? i : 0;
    const bool first = s->step == 0, close = s->step >= s->nsteps;
    const bool rec = s->thermo && s->thermo_every > 0 && s->step % s->thermo_every == 0;
    const double dt = s->dt, hdt = 0.5 * dt;
    Own<D, MIX> me;
    load_own<D, MIX>(s, ii, me);
    VT F[D];
    double e, w, z;
    if constexpr (LPA == 1) force_part_lds<D, MIX, VT, MORSE>(s, ii, vi, me, F, e, w, z, stage);
    else force_part<D, MIX, LPA, VT, MORSE>(s, ii, sub, me, F, e, w, z);
    double vals[kPart], mx = 0.0;
#pragma unroll
    for (int p = 0; p < kPart; p++) vals[p] = 0.0;
    if (vi && sub == 0) {
      VT* v = reinterpret_cast<VT*>(s->v[pc]);
      const VT lam = VT(s->vscale);
      const double L = s->L, h = s->hL;
      double m2 = 0.0;
      if (rec) {
#pragma unroll
        for (int k = 0; k < D; k++) {
          const size_t o = (size_t)k * npad + i;
          const double dd = s->disp[pc][o] + min_image(me.x[k] - s->xref[o], L, h);
          m2 = __builtin_fma(dd, dd, m2);
        }
      }
      VT vk[D];
      double xn[D], ke = 0.0;
#pragma unroll
      for (int k = 0; k < D; k++) {
        vk[k] = v[(size_t)k * npad + i];
        if (!first) vk[k] = lam * (vk[k] + VT(hdt) * F[k]);
        ke += (double)vk[k] * (double)vk[k];
      }
      double r2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; k++) {
        if (!close) {
          vk[k] += VT(hdt) * F[k];
          xn[k] = wrap1(me.x[k] + dt * (double)vk[k], L, h);
        } else {
          xn[k] = me.x[k];
        }
        v[(size_t)k * npad + i] = vk[k];
        const double dx = min_image(xn[k] - s->xref[(size_t)k * npad + i], L, h);
        r2 = __builtin_fma(dx, dx, r2);
      }
      store_rec<D>(s->x[cur ^ 1], i, xn, me.sg);
      if (MIX) store_q<D>(s->q[cur ^ 1], i, xn, me.sg, h, s->fxscale);
      vals[P_PE] = e;
      vals[P_KE] = 0.5 * ke;
      vals[P_VIR] = w;
      vals[P_NC] = z;
      vals[P_M2] = m2;
      vals[P_M4] = m2 * m2;
      vals[P_OV] = rec && m2 < 0.01 * D * D ? 1.0 : 0.0;
      mx = r2;
    }
    // the displacement maximum of the tile is reduced like the partial sums
    double* pt = s->part + (size_t)tile * kPart;
    tile_partials<LPA>(pt, vals, mx, sh, kUseStep | kUseDisp);
    if (threadIdx.x == 0 && pt[P_FMAX2] > 0.0)
      atomicMax(&s->maxdisp2, (unsigned long long)__double_as_longlong(pt[P_FMAX2]));
  }
}

// FIRE 2.0 semi-implicit Euler update with the coefficients of this
// iteration (computed per system by k_fire_ctrl):
//   on P <= 0: x -= dt/2 v, v = 0;  v += dt F;  v = (1-a) v + a |v|/|F| F;
//   x += dt v (wrapped, into the other buffer); displacement for the trigger.
template <int D, bool MIX>
__device__ inline void fire_update_tile(SysDev* s, int tile) {
  typedef typename VType<MIX>::T VT;
  const int i = tile * kTile + threadIdx.x;
  const int n = s->n, npad = s->npad, pc = s->pcur, cur = s->xcur;
  double disp2 = 0.0;
  if (i < n) {
    const double dt = s->c_dt, keep = s->c_keep, mix = s->c_mix;
    const bool zero = s->c_zero != 0;
    const double L = s->L, h = s->hL;
    double x[D], sg;
    load_rec<D>(s->x[cur], i, x, sg);
    VT* v = reinterpret_cast<VT*>(s->v[pc]);
    const VT* f = reinterpret_cast<const VT*>(s->f);
    double r2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; k++) {
      double vk = (double)v[(size_t)k * npad + i];
      const double fk = (double)f[(size_t)k * npad + i];
      if (zero) {
        x[k] = x[k] - 0.5 * dt * vk;
        vk = 0.0;
      }
      vk = vk + dt * fk;
      vk = keep * vk + mix * fk;
      const VT vs = VT(vk);
      v[(size_t)k * npad + i] = vs;
      x[k] = wrap1(x[k] + dt * (double)vs, L, h);
      double dx = min_image(x[k] - s->xref[(size_t)k * npad + i], L, h);
      r2 = __builtin_fma(dx, dx, r2);
    }
    store_rec<D>(s->x[cur ^ 1], i, x, sg);
    if (MIX) store_q<D>(s->q[cur ^ 1], i, x, sg, h, s->fxscale);
    disp2 = r2;
  }
  const double dm = wave_max(disp2);
  if ((threadIdx.x & (kWave - 1)) == 0 && dm > 0.0)
    atomicMax(&s->maxdisp2, (unsigned long long)__double_as_longlong(dm));
}

template <int D, bool MIX>
__global__ __launch_bounds__(kTile) void k_fire_update(KArgs a) {
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int tile;
    if (!fetch_atom_tile(a, t, s, tile)) break;
    if (!running(s) || s->mode != MODE_FIRE) continue;
    fire_update_tile<D, MIX>(s, tile);
  }
}

}  // namespace hdmd
