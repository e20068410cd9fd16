// kernels.h -- the gfx950 kernels of the hot path, templated on the dimension D.
//
//  k_load        caller [n][d] arrays -> internal buffers (wrap, validate)
//  k_bin         subcell of every atom + occupancy counts      (Sec. II.C)
//  k_scatter     counting-sort placement by subcell
//  k_cellsort    per-subcell sort by caller id, permutation of every per-atom
//                array, reference positions, FP32 subcell offsets
//  k_build       Verlet rows over the 3^d linked subcells      (Sec. II.C, Fig. 1)
//  k_force       pair forces and energy                        (Sec. II.B)
//  k_step        fused velocity-Verlet step + rebuild trigger (Sec. II.B/II.C)
//  k_fire_force  forces + FIRE reductions                      (Sec. II.B, FIRE 2.0)
//  k_fire_update semi-implicit Euler FIRE update
//  k_unload      internal -> caller order
//  k_export_*    canonical CSR export of the list
#pragma once
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
    store_x<D>(xo, i, x);
    s->sig[pc][i] = 0.0;
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
  store_x<D>(xo, i, x);
  double sg = diam[i];
  if (!isfinite(sg)) err |= ERR_NONFINITE;
  else if (!(sg > 0.0) || sg > s->sigma_max) err |= ERR_ARG;
  s->sig[pc][i] = sg;
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

template <int D>
__global__ __launch_bounds__(kTile) void k_bin(KArgs a) {
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int tile;
    if (!fetch_atom_tile(a, t, s, tile)) break;
    if (!running(s) || !need_rebuild(s)) continue;
    if (tile == 0 && threadIdx.x == 0) s->max_cell = 0;
    int i = tile * kTile + threadIdx.x;
    if (i >= s->n) continue;
    double x[D];
    load_x<D>(s->x[s->xcur ^ 1], i, x);
    int c = flat_cell<D>(s, x);
    s->cell_of[i] = c;
    s->rank[i] = atomicAdd(&s->cell_count[c], 1);
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

template <int D, typename VT>
__global__ __launch_bounds__(kTile) void k_cellsort(KArgs a) {
  constexpr int DY = Dims<D>::DY;
  __shared__ int sk[kSortCap];
  __shared__ int sv[kSortCap];
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int c;
    if (!fetch_cell_tile(a, t, s, c)) break;
    if (!running(s) || !need_rebuild(s)) continue;
    const int s0 = cell_start(s, c), cnt = cell_start(s, c + 1) - s0;
    if (threadIdx.x == 0) s->cell_count[c] = 0;  // ready for the next build
    if (cnt == 0) continue;
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
        cen[k] = ((double)(u % nc) + 0.5) * s->lsc - s->hL;
        u /= nc;
      }
    }
    const int cur = s->xcur, pc = s->pcur, pn = pc ^ 1, npad = s->npad;
    const VT* vin = reinterpret_cast<const VT*>(s->v[pc]);
    VT* vout = reinterpret_cast<VT*>(s->v[pn]);
    for (int q = threadIdx.x; q < cnt; q += blockDim.x) {
      const int src = vals[q], dst = s0 + q;
      double x[D];
      load_x<D>(s->x[cur ^ 1], src, x);
      store_x<D>(s->x[cur], dst, x);
      float y[DY];
#pragma unroll
      for (int k = 0; k < DY; k++) y[k] = 0.0f;
#pragma unroll
      for (int k = 0; k < D; k++) {
        s->xref[(size_t)k * npad + dst] = x[k];
        y[k] = (float)(x[k] - cen[k]);
        vout[(size_t)k * npad + dst] = vin[(size_t)k * npad + src];
      }
      float4* yp = reinterpret_cast<float4*>(s->ycell + (size_t)dst * DY);
#pragma unroll
      for (int k = 0; k < DY / 4; k++) yp[k] = make_float4(y[4 * k], y[4 * k + 1], y[4 * k + 2], y[4 * k + 3]);
      s->sig[pn][dst] = s->sig[pc][src];
      s->oid[pn][dst] = keys[q];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Verlet-list build over the linked subcells (Sec. II.C, Fig. 1)
//
// One workgroup per home subcell; its atoms are the lanes.  The linked
// subcells are decoded on the fly from a mixed-radix counter (offsets -1/0/+1
// per axis, or the deduplicated {0,+1} / {0} when n_cell is 2 / 1).  Each
// linked subcell's FP32 offsets-from-centre are staged in LDS and every lane
// tests every staged atom with a conservative FP32 prefilter (r^2 against the
// largest list radius, enlarged far beyond FP32 rounding).  Survivors go to a
// per-lane LDS queue and are re-tested exactly in FP64 with the per-pair
// radius -- the same operation sequence as the list definition -- before
// being appended to the row.  Row order: linked-subcell order, then slot
// order, which makes the list deterministic.
// With n_cell >= 3 the image shift of a linked subcell is its offset times the
// subcell side (exact for every pair within the list radius); with n_cell <= 2
// the per-axis minimum image is taken in the prefilter instead (WRAP).
// ---------------------------------------------------------------------------
template <int D, bool WRAP, int BLK>
__global__ __launch_bounds__(BLK) void k_build(KArgs a) {
  constexpr int DY = Dims<D>::DY;
  __shared__ float ys[BLK * DY];
  __shared__ int qbuf[kQCap * BLK];
  const int tid = threadIdx.x;
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int hc;
    if (!fetch_cell_tile(a, t, s, hc)) break;
    if (!running(s) || !need_rebuild(s)) continue;
    const int h0 = cell_start(s, hc), h1 = cell_start(s, hc + 1);
    if (h0 == h1) continue;
    const int nc = s->ncell, radix = s->radix, nst = s->nstencil, npad = s->npad;
    const int W = s->width;
    const int pn = s->pcur ^ 1;
    const double* __restrict__ xb = s->x[s->xcur];
    const double* __restrict__ sg = s->sig[pn];
    const float* __restrict__ yc = s->ycell;
    int* __restrict__ nl = s->nl;
    const double L = s->L, hL = s->hL, cut = s->cutoff, skin = s->skin;
    const float lscf = s->lscf, Lf = s->Lf, rl2f = s->rl2f;
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
      double xi[D];
      load_x<D>(xb, ii, xi);
      float yi[D];
#pragma unroll
      for (int k = 0; k < D; k++) yi[k] = yc[(size_t)ii * DY + k];
      const double si = sg[ii];
      int len = 0, qn = 0;

      auto flush = [&]() {
        for (int m = 0; m < qn; m++) {
          const int j = qbuf[m * BLK + tid];
          double xj[D];
          load_x<D>(xb, j, xj);
          const double r2 = dist2_exact<D>(xi, xj, L, hL);
          if (r2 < list_r2(si, sg[j], cut, skin)) {
            if (len < W) nl[(size_t)len * npad + i] = j;
            len++;
          }
        }
        qn = 0;
      };

      for (int q = 0; q < nst; q++) {
        // decode the linked subcell (axis 0 most significant)
        float tk[D];
        int J = 0;
        {
          int u = q;
          int cj[D];
#pragma unroll
          for (int k = D - 1; k >= 0; k--) {
            int dig = u % radix;
            u /= radix;
            int o = (radix == 3) ? dig - 1 : dig;
            int c2 = ci[k] + o;
            c2 = c2 < 0 ? c2 + nc : (c2 >= nc ? c2 - nc : c2);
            cj[k] = c2;
            if (WRAP) tk[k] = (float)(c2 - ci[k]) * lscf - yi[k];
            else tk[k] = (float)o * lscf - yi[k];
          }
#pragma unroll
          for (int k = 0; k < D; k++) J = J * nc + cj[k];
        }
        const int j0 = cell_start(s, J), j1 = cell_start(s, J + 1);
        for (int jb = j0; jb < j1; jb += BLK) {
          const int m = min(BLK, j1 - jb);
          __syncthreads();
          if (tid < m) {
            const float4* src = reinterpret_cast<const float4*>(yc + (size_t)(jb + tid) * DY);
            float4* dst = reinterpret_cast<float4*>(ys + tid * DY);
#pragma unroll
            for (int k = 0; k < DY / 4; k++) dst[k] = src[k];
          }
          __syncthreads();
          for (int u0 = 0; u0 < m; u0 += 8) {
#pragma unroll
            for (int uu = 0; uu < 8; uu++) {
              const int idx = u0 + uu;
              if (idx < m) {
                const float* yj = ys + idx * DY;
                float r2 = 0.0f;
#pragma unroll
                for (int k = 0; k < D; k++) {
                  float dx = yj[k] + tk[k];
                  if (WRAP) {
                    dx = fabsf(dx);
                    dx = fminf(dx, Lf - dx);
                  }
                  r2 = __builtin_fmaf(dx, dx, r2);
                }
                const int j = jb + idx;
                if (vi && r2 < rl2f && j != i) {
                  qbuf[qn * BLK + tid] = j;
                  qn++;
                }
              }
            }
            if (__any(qn > kQCap - 8)) flush();
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
// pair forces over one Verlet row (Sec. II.B getforce)
// ---------------------------------------------------------------------------
// F_i = sum_j fc (x_i - x_j) with fc = -U'(r)/r for r < c sigma_ij;
// e_i = 1/2 sum_j U(r).  FP64 path.
template <int D>
__device__ inline void pair_f64(int pot, double eps, double c, double r2, double sij,
                                double& fc, double& u) {
  if (pot == 0) {  // WCA
    const double inv = 1.0 / r2;
    const double s2 = sij * sij * inv;
    const double s6 = s2 * s2 * s2;
    fc = 24.0 * eps * (2.0 * s6 * s6 - s6) * inv;
    u = 4.0 * eps * (s6 * s6 - s6) + eps;
  } else {         // harmonic soft spheres
    const double r = sqrt(r2);
    const double g = 1.0 - r / sij;
    fc = eps * g / (sij * r);
    u = 0.5 * eps * g * g;
  }
}

__device__ inline void pair_f32(int pot, float eps, float r2, float sij, float& fc, float& u) {
  if (pot == 0) {
    const float inv = 1.0f / r2;
    const float s2 = sij * sij * inv;
    const float s6 = s2 * s2 * s2;
    fc = 24.0f * eps * (2.0f * s6 * s6 - s6) * inv;
    u = 4.0f * eps * (s6 * s6 - s6) + eps;
  } else {
    const float r = sqrtf(r2);
    const float g = 1.0f - r / sij;
    fc = eps * g / (sij * r);
    u = 0.5f * eps * g * g;
  }
}

// Accumulates the force on slot i (F as FT = double or float) and its energy.
template <int D, bool MIX, typename FT>
__device__ inline void force_row(const SysDev* s, const double* __restrict__ xb,
                                 const double* __restrict__ sg, int i, const double (&xi)[D],
                                 double si, FT (&F)[D], double& e) {
  const int npad = s->npad;
  const int len = min(s->nlen[i], s->width);
  const int* __restrict__ nl = s->nl;
  const double L = s->L, h = s->hL, c = s->cutoff, eps = s->eps;
  const int pot = s->potential;
#pragma unroll
  for (int k = 0; k < D; k++) F[k] = FT(0);
  e = 0.0;
  constexpr int U = 4;
  for (int k0 = 0; k0 < len; k0 += U) {
    int jj[U];
#pragma unroll
    for (int u = 0; u < U; u++) jj[u] = (k0 + u < len) ? nl[(size_t)(k0 + u) * npad + i] : i;
    double xj[U][D];
    double sj[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      load_x<D>(xb, jj[u], xj[u]);
      sj[u] = sg[jj[u]];
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (jj[u] == i) continue;
      const double sij = 0.5 * (si + sj[u]);
      const double rc = c * sij;
      if (!MIX) {
        double dx[D];
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; k++) {
          dx[k] = min_image(xj[u][k] - xi[k], L, h);
          r2 = __builtin_fma(dx[k], dx[k], r2);
        }
        if (r2 < rc * rc) {
          double fc, uu;
          pair_f64<D>(pot, eps, c, r2, sij, fc, uu);
#pragma unroll
          for (int k = 0; k < D; k++) F[k] -= FT(fc * dx[k]);
          e += 0.5 * uu;
        }
      } else {
        float dx[D];
        float r2 = 0.0f;
#pragma unroll
        for (int k = 0; k < D; k++) {
          dx[k] = (float)min_image(xj[u][k] - xi[k], L, h);
          r2 = __builtin_fmaf(dx[k], dx[k], r2);
        }
        const float rcf = (float)rc;
        if (r2 < rcf * rcf) {
          float fc, uu;
          pair_f32(pot, (float)eps, r2, (float)sij, fc, uu);
#pragma unroll
          for (int k = 0; k < D; k++) F[k] -= FT(fc * dx[k]);
          e += 0.5 * (double)uu;
        }
      }
    }
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

// Forces (stored in s->f) with per-wave energy and, for FIRE, the power
// P = F.v, |F|^2, |v|^2 and max_i |F_i|^2 partial sums.
template <int D, bool MIX>
__global__ __launch_bounds__(kTile) void k_force(KArgs a, int fire) {
  typedef typename VType<MIX>::T FT;
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int tile;
    if (!fetch_atom_tile(a, t, s, tile)) break;
    if (!running(s)) continue;
    if (fire && s->mode != MODE_FIRE) continue;
    const int i = tile * kTile + threadIdx.x;
    const int n = s->n, npad = s->npad, pc = s->pcur;
    const bool vi = i < n;
    const int ii = vi ? i : 0;
    const double* xb = s->x[s->xcur];
    double xi[D];
    load_x<D>(xb, ii, xi);
    FT F[D];
    double e;
    force_row<D, MIX, FT>(s, xb, s->sig[pc], ii, xi, s->sig[pc][ii], F, e);
    FT* fo = reinterpret_cast<FT*>(s->f);
    double fv = 0.0, ff = 0.0, vv = 0.0;
    const FT* v = reinterpret_cast<const FT*>(s->v[pc]);
    if (vi) {
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
    } else {
      e = 0.0;
    }
    const double pe = wave_sum(e);
    double r_fv = 0, r_ff = 0, r_vv = 0, r_fm = 0;
    if (fire) {
      r_fv = wave_sum(fv);
      r_ff = wave_sum(ff);
      r_vv = wave_sum(vv);
      r_fm = wave_max(ff);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
      double* p = s->part + (size_t)(i / kWave) * kPart;
      p[P_PE] = pe;
      p[P_FV] = r_fv;
      p[P_FF] = r_ff;
      p[P_VV] = r_vv;
      p[P_FMAX2] = r_fm;
    }
  }
}

// Fused velocity-Verlet step (kick-drift-kick leapfrog, Sec. II.B):
//   F = F(x^n); v^n = v^(n-1/2) + dt/2 F (skipped at step 0, where v is the
//   full-step velocity); record KE(v^n), PE(x^n); v^(n+1/2) = v^n + dt/2 F;
//   x^(n+1) = wrap(x^n + dt v^(n+1/2)) into the other position buffer;
//   max_i |x^(n+1)_i - x_ref,i|^2 for the rebuild trigger (skin/2).
// At the closing step (n == nsteps) only the second kick is applied.
template <int D, bool MIX>
__global__ __launch_bounds__(kTile) void k_step(KArgs a) {
  typedef typename VType<MIX>::T VT;
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int tile;
    if (!fetch_atom_tile(a, t, s, tile)) break;
    if (!running(s) || s->mode != MODE_MD) continue;
    const int i = tile * kTile + threadIdx.x;
    const int n = s->n, npad = s->npad, pc = s->pcur, cur = s->xcur;
    const bool vi = i < n;
    const int ii = vi ? i : 0;
    const bool first = s->step == 0, close = s->step >= s->nsteps;
    const double dt = s->dt, hdt = 0.5 * dt;
    const double* xb = s->x[cur];
    double xi[D];
    load_x<D>(xb, ii, xi);
    VT F[D];
    double e;
    force_row<D, MIX, VT>(s, xb, s->sig[pc], ii, xi, s->sig[pc][ii], F, e);
    VT* v = reinterpret_cast<VT*>(s->v[pc]);
    double ke = 0.0, disp2 = 0.0;
    if (vi) {
      VT vk[D];
      double xn[D];
#pragma unroll
      for (int k = 0; k < D; k++) {
        vk[k] = v[(size_t)k * npad + i];
        if (!first) vk[k] += VT(hdt) * F[k];
        ke += (double)vk[k] * (double)vk[k];
      }
      ke *= 0.5;
      const double L = s->L, h = s->hL;
#pragma unroll
      for (int k = 0; k < D; k++) {
        if (!close) {
          vk[k] += VT(hdt) * F[k];
          xn[k] = wrap1(xi[k] + dt * (double)vk[k], L, h);
        } else {
          xn[k] = xi[k];
        }
        v[(size_t)k * npad + i] = vk[k];
      }
      store_x<D>(s->x[cur ^ 1], i, xn);
      double r2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; k++) {
        double dx = min_image(xn[k] - s->xref[(size_t)k * npad + i], L, h);
        r2 = __builtin_fma(dx, dx, r2);
      }
      disp2 = r2;
    } else {
      e = 0.0;
    }
    const double pe = wave_sum(e);
    const double kes = wave_sum(ke);
    const double dm = wave_max(disp2);
    if ((threadIdx.x & (kWave - 1)) == 0) {
      double* p = s->part + (size_t)(i / kWave) * kPart;
      p[P_PE] = pe;
      p[P_KE] = kes;
      if (dm > 0.0) atomicMax(&s->maxdisp2, (unsigned long long)__double_as_longlong(dm));
    }
  }
}

// FIRE 2.0 semi-implicit Euler update with the coefficients of this
// iteration (computed per system by k_fire_ctrl):
//   on P <= 0: x -= dt/2 v, v = 0;  v += dt F;  v = (1-a) v + a |v|/|F| F;
//   x += dt v (wrapped, into the other buffer); displacement for the trigger.
template <int D, bool MIX>
__global__ __launch_bounds__(kTile) void k_fire_update(KArgs a) {
  typedef typename VType<MIX>::T VT;
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int tile;
    if (!fetch_atom_tile(a, t, s, tile)) break;
    if (!running(s) || s->mode != MODE_FIRE) continue;
    const int i = tile * kTile + threadIdx.x;
    const int n = s->n, npad = s->npad, pc = s->pcur, cur = s->xcur;
    double disp2 = 0.0;
    if (i < n) {
      const double dt = s->c_dt, keep = s->c_keep, mix = s->c_mix;
      const bool zero = s->c_zero != 0;
      const double L = s->L, h = s->hL;
      double x[D];
      load_x<D>(s->x[cur], i, x);
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
      store_x<D>(s->x[cur ^ 1], i, x);
      disp2 = r2;
    }
    const double dm = wave_max(disp2);
    if ((threadIdx.x & (kWave - 1)) == 0 && dm > 0.0)
      atomicMax(&s->maxdisp2, (unsigned long long)__double_as_longlong(dm));
  }
}

}  // namespace hdmd
