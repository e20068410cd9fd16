"""Thin ctypes binding of libhdmd.so (declared in include/hdmd.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors) and the stream.  The
names are those of the C ABI.  If the native library is missing the first call
raises; there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhdmd.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hdmd.h")

HDMD_OK = 0
HDMD_NOT_CONVERGED = 1
HDMD_ERR_ARG = -1
HDMD_ERR_BOX = -2
HDMD_ERR_WORKSPACE = -3
HDMD_ERR_NLIST_OVERFLOW = -4
HDMD_ERR_NONFINITE = -5
HDMD_ERR_HIP = -6
HDMD_ERR_STATE = -7
HDMD_WCA = 0
HDMD_HARMONIC = 1
HDMD_MORSE = 2
MORSE_A = 30.0  # the paper's Morse stiffness (Sec. II.A)
HDMD_FP64 = 0
HDMD_MIXED = 1
HDMD_SUBCELLS_AUTO = 0
HDMD_SUBCELLS_FULL = 1
HDMD_SUBCELLS_HALF = 2
HDMD_SLOT_EMPTY = 0
HDMD_SLOT_RUNNING = 1
HDMD_SLOT_DONE = 2
THERMO_COLS = 10  # columns of a thermo row of hdmd_step
WCA_CUT = 2.0 ** (1.0 / 6.0)


class HdmdError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__("%s failed with status %d: %s" % (where, status, msg))
        self.status = status


class hdmd_system(C.Structure):
    _fields_ = [("d", C.c_int32), ("potential", C.c_int32), ("precision", C.c_int32),
                ("max_neighbors", C.c_int32), ("n", C.c_int64), ("box_l", C.c_double),
                ("cutoff", C.c_double), ("skin", C.c_double), ("epsilon", C.c_double),
                ("sigma_max", C.c_double), ("morse_a", C.c_double),
                ("thermostat_tau", C.c_double), ("target_temp", C.c_double),
                ("subcells", C.c_int32), ("pad", C.c_int32)]


class hdmd_fire_params(C.Structure):
    _fields_ = [("dt0", C.c_double), ("dt_max", C.c_double), ("dt_min", C.c_double),
                ("f_inc", C.c_double), ("f_dec", C.c_double), ("alpha0", C.c_double),
                ("f_alpha", C.c_double), ("n_delay", C.c_int64), ("n_neg_max", C.c_int64),
                ("max_iter", C.c_int64), ("initial_delay", C.c_int64), ("f_tol", C.c_double),
                ("e_tol", C.c_double)]


class hdmd_fire_result(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("builds", C.c_int64), ("fmax", C.c_double),
                ("energy", C.c_double), ("status", C.c_int32), ("pad", C.c_int32)]


class hdmd_step_stats(C.Structure):
    _fields_ = [("steps_done", C.c_int64), ("builds", C.c_int64), ("ke", C.c_double),
                ("pe", C.c_double), ("max_row", C.c_int32), ("pad", C.c_int32),
                ("step_kernel_ms", C.c_double), ("step_kernels", C.c_int64),
                ("build_kernel_ms", C.c_double), ("build_kernels", C.c_int64)]


_lib = None
_vp = C.c_void_p
_SIGS = {
    "hdmd_last_error": (C.c_char_p, []),
    "hdmd_fire_defaults": (None, [C.POINTER(hdmd_fire_params), C.c_double, C.c_double, C.c_int64]),
    "hdmd_workspace_bytes": (C.c_size_t, [C.POINTER(hdmd_system)]),
    "hdmd_cells_per_axis": (C.c_int, [C.POINTER(hdmd_system)]),
    "hdmd_build_config": (C.c_int, [C.POINTER(hdmd_system), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]),
    "hdmd_build_nlist": (C.c_int, [C.POINTER(hdmd_system), _vp, _vp, _vp, C.c_size_t,
                                   C.POINTER(C.c_int32), _vp]),
    "hdmd_nlist_export": (C.c_int, [C.POINTER(hdmd_system), _vp, _vp, _vp, C.c_int64,
                                    C.POINTER(C.c_int64), _vp]),
    "hdmd_forces": (C.c_int, [C.POINTER(hdmd_system), _vp, _vp, _vp, C.c_size_t, _vp, _vp, _vp]),
    "hdmd_forces_noalloc_bytes": (C.c_size_t, []),
    "hdmd_forces_noalloc": (C.c_int, [C.POINTER(hdmd_system), _vp, _vp, _vp, _vp, _vp]),
    "hdmd_step": (C.c_int, [C.POINTER(hdmd_system), _vp, _vp, _vp, _vp, C.c_size_t, C.c_int64,
                            C.c_double, C.c_int64, _vp, C.POINTER(hdmd_step_stats), _vp]),
    "hdmd_step_resume": (C.c_int, [C.POINTER(hdmd_system), _vp, _vp, _vp, _vp, C.c_size_t,
                                   C.c_int64, C.c_double, C.c_int64, _vp,
                                   C.POINTER(hdmd_step_stats), _vp]),
    "hdmd_van_hove": (C.c_int, [C.POINTER(hdmd_system), _vp, C.c_size_t, C.c_int32, C.c_double,
                                _vp, _vp, _vp]),
    "hdmd_swap": (C.c_int, [C.POINTER(hdmd_system), _vp, _vp, _vp, C.c_size_t, C.c_int64, _vp, _vp,
                            C.c_double, _vp, C.POINTER(C.c_int64), _vp]),
    "hdmd_fire_minimize": (C.c_int, [C.POINTER(hdmd_system), _vp, _vp, _vp, C.c_size_t,
                                     C.POINTER(hdmd_fire_params), C.POINTER(hdmd_fire_result), _vp]),
    "hdmd_batch_bytes": (C.c_size_t, [C.c_int32, C.c_int64, C.c_int64]),
    "hdmd_batch_init": (C.c_int, [_vp, C.c_size_t, C.c_int32, C.c_int64, C.c_int64, _vp]),
    "hdmd_batch_add_fire": (C.c_int, [_vp, C.c_int32, C.POINTER(hdmd_system), _vp, _vp, _vp,
                                      C.c_size_t, C.POINTER(hdmd_fire_params), _vp]),
    "hdmd_batch_add_md": (C.c_int, [_vp, C.c_int32, C.POINTER(hdmd_system), _vp, _vp, _vp, _vp,
                                    C.c_size_t, C.c_int64, C.c_double, _vp]),
    "hdmd_batch_run": (C.c_int, [_vp, C.c_int32, _vp]),
    "hdmd_batch_poll": (C.c_int, [_vp, _vp, _vp, _vp]),
    "hdmd_batch_take": (C.c_int, [_vp, C.c_int32, _vp, _vp, C.POINTER(hdmd_fire_result), _vp]),
}


def header_symbols() -> list[str]:
    """Every function the public header declares."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hdmd_[a-z_0-9]+)\s*\(", txt)))


def lib() -> C.CDLL:
    """Loads libhdmd.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhdmd.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().hdmd_last_error().decode()


def _check(rc: int, where: str, ok=(HDMD_OK,)):
    if rc not in ok:
        raise HdmdError(rc, where, last_error())
    return rc


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("%s must be a contiguous float64 CUDA tensor" % name)
    return t


@dataclasses.dataclass
class System:
    """Python view of hdmd_system."""
    d: int
    n: int
    box_l: float
    potential: int = HDMD_WCA
    cutoff: float = WCA_CUT
    skin: float = 0.3
    epsilon: float = 1.0
    sigma_max: float = 1.0
    precision: int = HDMD_FP64
    max_neighbors: int = 64
    morse_a: float = MORSE_A
    thermostat_tau: float = 0.0   # Berendsen time constant of MD runs (0: NVE)
    target_temp: float = 0.0
    subcells: int = HDMD_SUBCELLS_AUTO  # grid of the list build (autotuned, full or half-size)

    def c(self) -> hdmd_system:
        return hdmd_system(self.d, self.potential, self.precision, self.max_neighbors, self.n,
                           self.box_l, self.cutoff, self.skin, self.epsilon, self.sigma_max,
                           self.morse_a, self.thermostat_tau, self.target_temp, self.subcells, 0)


def hdmd_fire_defaults(dt0: float = 0.05, f_tol: float = 1e-10,
                       max_iter: int = 100000) -> hdmd_fire_params:
    p = hdmd_fire_params()
    lib().hdmd_fire_defaults(C.byref(p), dt0, f_tol, max_iter)
    return p


def hdmd_workspace_bytes(sys: System) -> int:
    b = lib().hdmd_workspace_bytes(C.byref(sys.c()))
    if b == 0:
        raise HdmdError(HDMD_ERR_ARG, "hdmd_workspace_bytes", last_error())
    return int(b)


def hdmd_cells_per_axis(sys: System) -> int:
    return int(lib().hdmd_cells_per_axis(C.byref(sys.c())))


def hdmd_build_config(sys: System) -> tuple:
    """(tuned, reach, cells per axis, build variant, lanes per atom) that calls
    on sys use now."""
    r, nc, v, la = C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_int32(0)
    rc = lib().hdmd_build_config(C.byref(sys.c()), C.byref(r), C.byref(nc), C.byref(v),
                                 C.byref(la))
    if rc < 0:
        raise HdmdError(rc, "hdmd_build_config", last_error())
    return bool(rc), int(r.value), int(nc.value), int(v.value), int(la.value)


def workspace(sys: System, device="cuda") -> torch.Tensor:
    return torch.empty(hdmd_workspace_bytes(sys), dtype=torch.uint8, device=device)


def hdmd_build_nlist(sys: System, pos, diam, ws, stream=None) -> tuple[int, int]:
    """Returns (status, required_width); raises on errors other than overflow."""
    rw = C.c_int32(0)
    rc = lib().hdmd_build_nlist(C.byref(sys.c()), _ptr(_dev_f64(pos, "pos")),
                                _ptr(_dev_f64(diam, "diam")), _ptr(ws), ws.numel(), C.byref(rw),
                                _stream(stream))
    _check(rc, "hdmd_build_nlist", ok=(HDMD_OK, HDMD_ERR_NLIST_OVERFLOW))
    return rc, int(rw.value)


def hdmd_nlist_export(sys: System, ws, stream=None) -> tuple[torch.Tensor, torch.Tensor]:
    """Canonical CSR (caller ids, ascending rows) of the list held in ws."""
    dev = ws.device
    row_ptr = torch.zeros(sys.n + 1, dtype=torch.int64, device=dev)
    nnz = C.c_int64(0)
    rc = lib().hdmd_nlist_export(C.byref(sys.c()), _ptr(ws), _ptr(row_ptr), None, 0,
                                 C.byref(nnz), _stream(stream))
    _check(rc, "hdmd_nlist_export", ok=(HDMD_OK, HDMD_ERR_WORKSPACE))
    cols = torch.empty(max(int(nnz.value), 1), dtype=torch.int32, device=dev)
    rc = lib().hdmd_nlist_export(C.byref(sys.c()), _ptr(ws), _ptr(row_ptr), _ptr(cols),
                                 cols.numel(), C.byref(nnz), _stream(stream))
    _check(rc, "hdmd_nlist_export")
    return row_ptr, cols[: int(nnz.value)]


def build_with_width(sys: System, pos, diam, width: int | None = None, slack: float = 1.5):
    """Builds the list, growing max_neighbors until no row overflows.
    Returns (system with the final width, workspace)."""
    if width is not None:
        sys = dataclasses.replace(sys, max_neighbors=width)
    while True:
        ws = workspace(sys, pos.device)
        rc, rw = hdmd_build_nlist(sys, pos, diam, ws)
        if rc == HDMD_OK:
            return sys, ws
        del ws
        sys = dataclasses.replace(sys, max_neighbors=int(rw * slack) + 16)


def hdmd_forces(sys: System, pos, diam, ws, stream=None) -> tuple[torch.Tensor, torch.Tensor]:
    F = torch.empty((sys.n, sys.d), dtype=torch.float64, device=pos.device)
    E = torch.zeros((), dtype=torch.float64, device=pos.device)
    rc = lib().hdmd_forces(C.byref(sys.c()), _ptr(_dev_f64(pos, "pos")),
                           _ptr(_dev_f64(diam, "diam")), _ptr(ws), ws.numel(), _ptr(F), _ptr(E),
                           _stream(stream))
    _check(rc, "hdmd_forces")
    return F, E


def hdmd_step(sys: System, pos, vel, diam, ws, nsteps: int, dt: float, thermo_every: int = 0,
              stream=None, resume: bool = False):
    """Runs nsteps of velocity Verlet in place on pos/vel.
    Returns (stats, thermo rows (k, THERMO_COLS) or None); the columns are
    step, KE, PE, KE+PE, W (virial sum over pairs of r_ij . F_ij), Z (mean
    neighbours inside the cutoff), <|dr|^2>, <|dr|^4>, alpha_2 and f_ov of the
    unwrapped displacement dr since step 0 of this call.  resume: continue
    the run the last call left in ws (hdmd_step_resume; pos/vel/diam must be
    the arrays that call returned)."""
    th = None
    if thermo_every > 0:
        th = torch.zeros((nsteps // thermo_every + 1, THERMO_COLS), dtype=torch.float64,
                         device=pos.device)
    st = hdmd_step_stats()
    fn = lib().hdmd_step_resume if resume else lib().hdmd_step
    rc = fn(C.byref(sys.c()), _ptr(_dev_f64(pos, "pos")), _ptr(_dev_f64(vel, "vel")),
            _ptr(_dev_f64(diam, "diam")), _ptr(ws), ws.numel(), nsteps, dt,
            thermo_every, _ptr(th), C.byref(st), _stream(stream))
    _check(rc, "hdmd_step_resume" if resume else "hdmd_step")
    return st, th


def hdmd_van_hove(sys: System, ws, nbins: int, bin_width: float, disp: bool = False,
                  stream=None):
    """Histogram of |dr| (nbins + 1 counts, the last one beyond nbins * bin_width)
    of the unwrapped displacements of the hdmd_step call last run on ws, and
    with disp also dr itself in caller order (n, d); G_s(r_b) = hist[b] / (n w)."""
    hist = torch.empty(nbins + 1, dtype=torch.int64, device=ws.device)
    dr = torch.empty((sys.n, sys.d), dtype=torch.float64, device=ws.device) if disp else None
    rc = lib().hdmd_van_hove(C.byref(sys.c()), _ptr(ws), ws.numel(), nbins, bin_width,
                             _ptr(hist), _ptr(dr), _stream(stream))
    _check(rc, "hdmd_van_hove")
    return hist, dr


def hdmd_swap(sys: System, pos, diam, ws, pairs, u, temperature: float, stream=None):
    """SWAP Monte Carlo attempts in order on the device (diam updated in place).
    pairs: (m, 2) int32 caller ids, u: m uniforms (device tensors).
    Returns (accepted flags (m,) int32, number accepted)."""
    m = int(pairs.shape[0]) if pairs is not None else 0
    acc = torch.zeros(m, dtype=torch.int32, device=ws.device)
    na = C.c_int64(0)
    if m:
        assert pairs.dtype == torch.int32 and pairs.is_contiguous() and pairs.shape[1] == 2
    rc = lib().hdmd_swap(C.byref(sys.c()), _ptr(_dev_f64(pos, "pos")), _ptr(_dev_f64(diam, "diam")),
                         _ptr(ws), ws.numel(), m, _ptr(pairs) if m else None,
                         _ptr(_dev_f64(u, "u")) if m else None, temperature, _ptr(acc) if m else None,
                         C.byref(na), _stream(stream))
    _check(rc, "hdmd_swap")
    return acc, int(na.value)


def step_auto(sys: System, pos, vel, diam, nsteps: int, dt: float, thermo_every: int = 0,
              slack: float = 1.5):
    """hdmd_step with a workspace sized from a first build, regrown and re-run
    from the untouched inputs whenever a Verlet row overflows mid-run.
    Returns (system with the final width, stats, thermo)."""
    sys, ws = build_with_width(sys, pos, diam, slack=slack)
    while True:
        try:
            st, th = hdmd_step(sys, pos, vel, diam, ws, nsteps, dt, thermo_every)
            return sys, st, th
        except HdmdError as e:
            if e.status != HDMD_ERR_NLIST_OVERFLOW:
                raise
            sys = dataclasses.replace(sys, max_neighbors=int(sys.max_neighbors * slack) + 16)
            del ws
            ws = workspace(sys, pos.device)


def fire_auto(sys: System, pos, diam, params: hdmd_fire_params | None = None,
              slack: float = 1.5):
    """hdmd_fire_minimize with the same regrow-and-retry policy as step_auto."""
    sys, ws = build_with_width(sys, pos, diam, slack=slack)
    while True:
        try:
            return sys, hdmd_fire_minimize(sys, pos, diam, ws, params)
        except HdmdError as e:
            if e.status != HDMD_ERR_NLIST_OVERFLOW:
                raise
            sys = dataclasses.replace(sys, max_neighbors=int(sys.max_neighbors * slack) + 16)
            del ws
            ws = workspace(sys, pos.device)


def hdmd_fire_minimize(sys: System, pos, diam, ws, params: hdmd_fire_params | None = None,
                       stream=None) -> hdmd_fire_result:
    params = params or hdmd_fire_defaults()
    res = hdmd_fire_result()
    rc = lib().hdmd_fire_minimize(C.byref(sys.c()), _ptr(_dev_f64(pos, "pos")),
                                  _ptr(_dev_f64(diam, "diam")), _ptr(ws), ws.numel(),
                                  C.byref(params), C.byref(res), _stream(stream))
    _check(rc, "hdmd_fire_minimize", ok=(HDMD_OK, HDMD_NOT_CONVERGED))
    return res


class Batch:
    """A batch table of up to max_slots systems (hdmd_batch_* calls)."""

    def __init__(self, max_slots: int, max_atoms: int, max_cells: int, device="cuda", stream=None):
        nbytes = lib().hdmd_batch_bytes(max_slots, max_atoms, max_cells)
        if nbytes == 0:
            raise HdmdError(HDMD_ERR_ARG, "hdmd_batch_bytes", "bad batch capacities")
        self.table = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        self.max_slots = max_slots
        self.stream = stream
        self._keep = {}
        _check(lib().hdmd_batch_init(_ptr(self.table), self.table.numel(), max_slots, max_atoms,
                                     max_cells, _stream(stream)), "hdmd_batch_init")

    def hdmd_batch_add_fire(self, slot: int, sys: System, pos, diam, ws, params=None):
        params = params or hdmd_fire_defaults()
        rc = lib().hdmd_batch_add_fire(_ptr(self.table), slot, C.byref(sys.c()),
                                       _ptr(_dev_f64(pos, "pos")), _ptr(_dev_f64(diam, "diam")),
                                       _ptr(ws), ws.numel(), C.byref(params), _stream(self.stream))
        _check(rc, "hdmd_batch_add_fire")
        self._keep[slot] = (sys, ws)

    def hdmd_batch_add_md(self, slot: int, sys: System, pos, vel, diam, ws, nsteps: int,
                          dt: float):
        rc = lib().hdmd_batch_add_md(_ptr(self.table), slot, C.byref(sys.c()),
                                     _ptr(_dev_f64(pos, "pos")), _ptr(_dev_f64(vel, "vel")),
                                     _ptr(_dev_f64(diam, "diam")), _ptr(ws), ws.numel(), nsteps,
                                     dt, _stream(self.stream))
        _check(rc, "hdmd_batch_add_md")
        self._keep[slot] = (sys, ws)

    def hdmd_batch_run(self, iterations: int):
        _check(lib().hdmd_batch_run(_ptr(self.table), iterations, _stream(self.stream)),
               "hdmd_batch_run")

    def hdmd_batch_poll(self):
        import numpy as np
        state = np.zeros(self.max_slots, dtype=np.int32)
        iters = np.zeros(self.max_slots, dtype=np.int64)
        _check(lib().hdmd_batch_poll(_ptr(self.table), state.ctypes.data_as(C.c_void_p),
                                     iters.ctypes.data_as(C.c_void_p), _stream(self.stream)),
               "hdmd_batch_poll")
        return state, iters

    def hdmd_batch_take(self, slot: int, want_vel: bool = False):
        sys, ws = self._keep[slot]
        pos = torch.empty((sys.n, sys.d), dtype=torch.float64, device=ws.device)
        vel = torch.empty_like(pos) if want_vel else None
        res = hdmd_fire_result()
        rc = lib().hdmd_batch_take(_ptr(self.table), slot, _ptr(pos), _ptr(vel), C.byref(res),
                                   _stream(self.stream))
        del self._keep[slot]
        _check(rc, "hdmd_batch_take", ok=(HDMD_OK, HDMD_NOT_CONVERGED))
        return pos, vel, res
