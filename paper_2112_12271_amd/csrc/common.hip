// common.hip -- dimension-independent kernels: descriptor upload, prefix
// sums of the subcell occupancies, counting-sort placement, per-system
// finalisation of a step (reductions, thermo rows, buffer flips) and the
// per-system FIRE 2.0 control.
#include "kernels.h"
#include "dispatch.h"

namespace hdmd {

const DKernels* dkernels_d2();
const DKernels* dkernels_d3();
const DKernels* dkernels_d4();
const DKernels* dkernels_d5();
const DKernels* dkernels_d6();
const DKernels* dkernels_d7();
const DKernels* dkernels_d8();
const DKernels* dkernels_d9();
const DKernels* dkernels_d10();

const DKernels* dkernels(int d) {
  switch (d) {
    case 2: return dkernels_d2();
    case 3: return dkernels_d3();
    case 4: return dkernels_d4();
    case 5: return dkernels_d5();
    case 6: return dkernels_d6();
    case 7: return dkernels_d7();
    case 8: return dkernels_d8();
    case 9: return dkernels_d9();
    case 10: return dkernels_d10();
    default: return nullptr;
  }
}

__global__ void k_setdesc(SysDev* dst, SysDev val) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = val;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_set_status(SysDev* s, int32_t status) {
  if (threadIdx.x == 0) s->status = status;
}

// Snapshot of every slot's state and iteration / step count.
__global__ void k_poll(const Table* t, int32_t* state, int64_t* iters) {
  int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= t->max_slots) return;
  const SysDev* s = t->sys[slot];
  if (!s) {
    state[slot] = SLOT_EMPTY;
    iters[slot] = 0;
    return;
  }
  state[slot] = s->status;
  iters[slot] = s->mode == MODE_MD ? (s->step > 0 ? s->step - 1 : 0) : s->iters;
}

// Exclusive scan of the occupancies of one chunk of kChunk subcells.
__global__ __launch_bounds__(256) void k_scan1(KArgs a) {
  __shared__ int sh[256];
  const int tid = threadIdx.x;
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int ch;
    if (!fetch_chunk_tile(a, t, s, ch)) break;
    if (!running(s) || !need_rebuild(s)) {
      if (a.single) break;  // one system: the same for every tile
      continue;
    }
    const int nc = s->ncells;
    const int c0 = ch * kChunk + tid * 4;
    int v[4], local = 0, mx = 0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
      v[u] = (c0 + u < nc) ? s->cell_count[c0 + u] : 0;
      local += v[u];
      mx = max(mx, v[u]);
    }
    sh[tid] = local;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      int x = tid >= off ? sh[tid - off] : 0;
      __syncthreads();
      sh[tid] += x;
      __syncthreads();
    }
    int run = sh[tid] - local;
#pragma unroll
    for (int u = 0; u < 4; u++) {
      if (c0 + u < nc) s->cell_local[c0 + u] = run;
      run += v[u];
    }
    if (tid == 255) s->chunk_sum[ch] = sh[255];
    mx = wave_max_i(mx);
    if ((tid & 63) == 0 && mx > 0) atomicMax(&s->max_cell, mx);
    __syncthreads();
  }
}

// Exclusive scan of the chunk totals of one system.
__global__ __launch_bounds__(256) void k_scan2(KArgs a) {
  __shared__ int sh[256];
  const int tid = threadIdx.x;
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    if (!fetch_sys(a, t, s)) break;
    if (!running(s) || !need_rebuild(s)) {
      if (a.single) break;  // one system: the same for every tile
      continue;
    }
    int carry = 0;
    for (int b = 0; b < s->nchunks; b += 256) {
      const int c = b + tid;
      const int v = c < s->nchunks ? s->chunk_sum[c] : 0;
      sh[tid] = v;
      __syncthreads();
      for (int off = 1; off < 256; off <<= 1) {
        int x = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += x;
        __syncthreads();
      }
      if (c < s->nchunks) s->chunk_off[c] = carry + sh[tid] - v;
      carry += sh[255];
      __syncthreads();
    }
    if (tid == 0) s->max_row = 0;
    __syncthreads();
  }
}

// Counting-sort placement: slot = start(subcell) + arrival rank.
__global__ __launch_bounds__(kTile) void k_scatter(KArgs a) {
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    int tile;
    if (!fetch_atom_tile(a, t, s, tile)) break;
    if (!running(s) || !need_rebuild(s)) {
      if (a.single) break;  // one system: the same for every tile
      continue;
    }
    const int i = tile * kTile + threadIdx.x;
    if (i >= s->n) continue;
    const int c = s->cell_of[i];
    const int slot = cell_start(s, c) + s->rank[i];
    int key = s->oid[s->pcur][i];
    if (s->ysort) {
      // the offset along the last axis exactly as the subcell sort quantises
      // it (caller ids below 2^23)
      const double xl = s->x[s->xcur ^ 1][(size_t)i * rec_stride(s->d) + s->d - 1];
      key |= (quant8(xl - last_centre(s, c), s->qinv) + 128) << 23;
    }
    s->key[slot] = key;
    s->src[slot] = i;
  }
}

// End of a step / iteration for one system: energy reductions and thermo
// row (MD), buffer flips (the permuted buffers after a rebuild, otherwise the
// freshly written position buffer), trigger reset, step counter.
__global__ __launch_bounds__(256) void k_finalize(KArgs a) {
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    if (!fetch_sys(a, t, s)) break;
    if (!running(s)) continue;
    const bool rb = need_rebuild(s);
    if (s->mode == MODE_MD) {
      const int nw = s->nwaves, per = (nw + 255) / 256;
      const bool rec = s->thermo && s->thermo_every > 0 && s->step % s->thermo_every == 0;
      double pe = 0.0, ke = 0.0, vir = 0.0, nc = 0.0, m2 = 0.0, m4 = 0.0, ov = 0.0;
      for (int w = tid * per; w < min(nw, (tid + 1) * per); w++) {
        const double* pw = s->part + (size_t)w * kPart;
        pe += pw[P_PE];
        ke += pw[P_KE];
        if (rec) {
          vir += pw[P_VIR];
          nc += pw[P_NC];
          m2 += pw[P_M2];
          m4 += pw[P_M4];
          ov += pw[P_OV];
        }
      }
      pe = block_sum<256>(pe, sh);
      ke = block_sum<256>(ke, sh);
      if (rec) {
        vir = block_sum<256>(vir, sh);
        nc = block_sum<256>(nc, sh);
        m2 = block_sum<256>(m2, sh);
        m4 = block_sum<256>(m4, sh);
        ov = block_sum<256>(ov, sh);
      }
      if (tid == 0) {
        s->pe = pe;
        s->ke = ke;
        if (!isfinite(pe + ke)) s->err |= ERR_RUN_NAN;
        // Berendsen factor for the next full-step kick, from this step's T
        if (s->tau_t > 0.0 && ke > 0.0) {
          const double T = 2.0 * ke / ((double)s->d * (double)(s->n - 1));
          s->vscale = sqrt(1.0 + s->dt / s->tau_t * (s->temp_t / T - 1.0));
        } else {
          s->vscale = 1.0;
        }
        if (rec) {
          double* r = s->thermo + kThermoCols * (s->step / s->thermo_every);
          r[0] = (double)s->step;
          r[1] = ke;
          r[2] = pe;
          r[3] = ke + pe;
          r[4] = vir;                 // sum over pairs of r_ij . F_ij
          r[5] = nc / (double)s->n;   // mean neighbours inside the cutoff (Z)
          // displacement moments since the run's start, alpha_2 (eq. ngp; 0
          // while nothing has moved) and f_ov (eq. fov)
          const double msd = m2 / (double)s->n, mqd = m4 / (double)s->n;
          r[6] = msd;
          r[7] = mqd;
          r[8] = msd > 0.0 ? s->d * mqd / ((s->d + 2) * msd * msd) - 1.0 : 0.0;
          r[9] = ov / (double)s->n;
        }
      }
    }
    if (tid == 0) {
      if (rb) {
        s->pcur ^= 1;
        s->builds++;
      } else {
        s->xcur ^= 1;
      }
      s->maxdisp2 = 0ull;
      s->force_rebuild = 0;
      if (s->mode == MODE_MD) {
        s->step++;
        if (s->step > s->nsteps) s->status = SLOT_DONE;
      }
      if (s->err) s->status = SLOT_DONE;
    }
    __syncthreads();
  }
}

// FIRE 2.0 control for one system (semi-implicit Euler variant, unit masses):
// fixed-order reductions of the wave partials, convergence test on the
// current forces, then the P = F.v branch, dt / alpha updates and the mixing
// coefficients.  |v + dt F|^2 is formed from |v|^2, F.v and |F|^2.
__global__ __launch_bounds__(256) void k_fire_ctrl(KArgs a) {
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  for (int t = blockIdx.x;; t += gridDim.x) {
    SysDev* s;
    if (!fetch_sys(a, t, s)) break;
    if (!running(s) || s->mode != MODE_FIRE) continue;
    const int nw = s->nwaves, per = (nw + 255) / 256;
    double pe = 0, fv = 0, ff = 0, vv = 0, fm = 0;
    for (int w = tid * per; w < min(nw, (tid + 1) * per); w++) {
      const double* p = s->part + (size_t)w * kPart;
      pe += p[P_PE];
      fv += p[P_FV];
      ff += p[P_FF];
      vv += p[P_VV];
      fm = fmax(fm, p[P_FMAX2]);
    }
    pe = block_sum<256>(pe, sh);
    fv = block_sum<256>(fv, sh);
    ff = block_sum<256>(ff, sh);
    vv = block_sum<256>(vv, sh);
    fm = block_max<256>(fm, sh);
    if (tid == 0) {
      const FireCtl& c = s->fc;
      s->pe = pe;
      s->fmax = sqrt(fm);
      if (!isfinite(pe) || !isfinite(ff)) {
        s->err |= ERR_RUN_NAN;
        s->status = SLOT_DONE;
        s->fstatus = -5;
      } else if (sqrt(fm) < c.ftol || (c.etol > 0.0 && pe / (double)s->n < c.etol)) {
        s->status = SLOT_DONE;
        s->fstatus = 0;
      } else if (s->iters >= c.maxiter) {
        s->status = SLOT_DONE;
        s->fstatus = 1;
      } else {
        double dt = s->fdt, alpha = s->falpha;
        int zero = 0;
        bool stop = false;
        if (fv > 0.0) {
          s->npos++;
          s->nneg = 0;
          if (s->npos > c.ndelay) {
            dt = fmin(dt * c.finc, c.dtmax);
            alpha *= c.falpha;
          }
        } else {
          s->npos = 0;
          s->nneg++;
          if (s->nneg > c.nnegmax) {
            stop = true;
          } else {
            if (!(c.initdelay && s->iters < c.ndelay)) {
              if (dt * c.fdec >= c.dtmin) dt *= c.fdec;
              alpha = c.alpha0;
            }
            zero = 1;
          }
        }
        if (stop) {
          s->status = SLOT_DONE;
          s->fstatus = 1;
        } else {
          const double v2 = zero ? dt * dt * ff : vv + 2.0 * dt * fv + dt * dt * ff;
          const double vn = sqrt(v2), fn = sqrt(ff);
          s->fdt = dt;
          s->falpha = alpha;
          s->c_zero = zero;
          s->c_dt = dt;
          s->c_keep = fn > 0.0 ? 1.0 - alpha : 1.0;
          s->c_mix = fn > 0.0 ? alpha * vn / fn : 0.0;
          s->iters++;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// canonical CSR export (caller ids, ascending rows)
// ---------------------------------------------------------------------------
__global__ void k_export_lens(const SysDev* s, int64_t* row_ptr) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= s->n) return;
  row_ptr[s->oid[s->pcur][p] + 1] = min(s->nlen[p], s->width);
}

__global__ void k_export_fill(const SysDev* s, const int64_t* row_ptr, int32_t* cols) {
  __shared__ int keys[kSortCap];
  const int p = blockIdx.x;
  if (p >= s->n) return;
  const int pc = s->pcur, npad = s->npad;
  const int a = s->oid[pc][p];
  const int len = min(s->nlen[p], s->width);
  int* out = cols + row_ptr[a];
  int* buf = len <= kSortCap ? keys : out;
  for (int k = threadIdx.x; k < len; k += blockDim.x) buf[k] = s->oid[pc][s->nl[(size_t)k * npad + p]];
  __syncthreads();
  bitonic_sort<false>(buf, nullptr, len);
  if (buf == keys)
    for (int k = threadIdx.x; k < len; k += blockDim.x) out[k] = keys[k];
}

__global__ __launch_bounds__(256) void k_reduce_pe(const SysDev* s, double* out) {
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  const int nw = s->nwaves, per = (nw + 255) / 256;
  double pe = 0.0;
  for (int w = tid * per; w < min(nw, (tid + 1) * per); w++) pe += s->part[(size_t)w * kPart + P_PE];
  pe = block_sum<256>(pe, sh);
  if (tid == 0) *out = pe;
}

// Inclusive scan of row lengths into CSR row pointers (row_ptr[0] = 0).
__global__ __launch_bounds__(1024) void k_export_scan(int n, int64_t* row_ptr) {
  __shared__ int64_t sh[1024];
  const int tid = threadIdx.x;
  int64_t carry = 0;
  if (tid == 0) row_ptr[0] = 0;
  for (int b = 0; b < n; b += 1024) {
    const int r = b + tid;
    const int64_t v = r < n ? row_ptr[r + 1] : 0;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int64_t x = tid >= off ? sh[tid - off] : 0;
      __syncthreads();
      sh[tid] += x;
      __syncthreads();
    }
    if (r < n) row_ptr[r + 1] = carry + sh[tid];
    carry += sh[1023];
    __syncthreads();
  }
}

void launch_setdesc(SysDev* dst, const SysDev& val, hipStream_t st) {
  k_setdesc<<<1, 64, 0, st>>>(dst, val);
}
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return;
  int64_t g = (n + 255) / 256;
  k_fill_i32<<<(int)(g < 4096 ? g : 4096), 256, 0, st>>>(p, n, v);
}
void launch_scan1(const KArgs& a, int grid, hipStream_t st) { k_scan1<<<grid, 256, 0, st>>>(a); }
void launch_scan2(const KArgs& a, int grid, hipStream_t st) { k_scan2<<<grid, 256, 0, st>>>(a); }
void launch_scatter(const KArgs& a, int grid, hipStream_t st) {
  k_scatter<<<grid, kTile, 0, st>>>(a);
}
void launch_finalize(const KArgs& a, int grid, hipStream_t st) {
  k_finalize<<<grid, 256, 0, st>>>(a);
}
void launch_fire_ctrl(const KArgs& a, int grid, hipStream_t st) {
  k_fire_ctrl<<<grid, 256, 0, st>>>(a);
}
// slot_of[caller id] = position in subcell order
__global__ __launch_bounds__(256) void k_slot_of(const SysDev* s, int32_t* slot_of) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < s->n) slot_of[s->oid[s->pcur][p]] = p;
}

void launch_slot_of(const SysDev* s, int n, int32_t* slot_of, hipStream_t st) {
  k_slot_of<<<(n + 255) / 256, 256, 0, st>>>(s, slot_of);
}

// SWAP set-up: zeroes the round counters (ctl[0..2]) and flags in ctl[3] any
// pair id outside [0, n).
__global__ __launch_bounds__(256) void k_swap_init(int64_t n_att, const int32_t* pairs, int n,
                                                   long long* ctl) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t == 0) {
    ctl[0] = 0;
    ctl[1] = 0;
    ctl[2] = 0;
  }
  bool bad = false;
  for (int64_t k = t; k < 2 * n_att; k += (int64_t)gridDim.x * 256) {
    const int32_t v = pairs[k];
    bad = bad || v < 0 || v >= n;
  }
  if (bad) atomicOr(reinterpret_cast<unsigned long long*>(ctl + 3), 1ull);
}

void launch_swap_init(int64_t n_att, const int32_t* pairs, int n, long long* ctl, hipStream_t st) {
  const int64_t g = (2 * n_att + 255) / 256;
  k_swap_init<<<(int)(g < 1 ? 1 : (g > 1024 ? 1024 : g)), 256, 0, st>>>(n_att, pairs, n, ctl);
}

void launch_reduce_pe(const SysDev* s, double* out, hipStream_t st) {
  k_reduce_pe<<<1, 256, 0, st>>>(s, out);
}
void launch_export(const SysDev* s, int n, int64_t* row_ptr, int32_t* cols, hipStream_t st,
                   int phase) {
  if (phase == 0) k_export_lens<<<(n + 255) / 256, 256, 0, st>>>(s, row_ptr);
  else if (phase == 1) k_export_scan<<<1, 1024, 0, st>>>(n, row_ptr);
  else k_export_fill<<<n, 256, 0, st>>>(s, row_ptr, cols);
}
void launch_set_status(SysDev* s, int32_t status, hipStream_t st) {
  k_set_status<<<1, 64, 0, st>>>(s, status);
}
void launch_poll(const Table* t, int max_slots, int32_t* state, int64_t* iters, hipStream_t st) {
  k_poll<<<(max_slots + 255) / 256, 256, 0, st>>>(t, state, iters);
}

}  // namespace hdmd
