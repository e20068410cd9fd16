"""ctypes wrapper over the plain CPU oracle (``hdmd_oracle.c``).

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  The product library never imports this module and
this module never imports the product package.

Positions are numpy arrays of shape (n, d), float64, row-major.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hdmd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")  # the same source with -fopenmp (CPU baseline)

WCA = 0
HARMONIC = 1
MORSE = 2
MORSE_A = 30.0
WCA_CUT = 2.0 ** (1.0 / 6.0)


def _compile(out: str, extra: list[str]) -> None:
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(
        ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared",
         *extra, "-o", tmp, SRC, "-lm"])
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off, no fast-math), and
    the same source with -fopenmp for the all-core CPU baseline."""
    for out, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
            _compile(out, extra)
    return LIB


class FireParams(C.Structure):
    _fields_ = [("dt0", C.c_double), ("dtmax", C.c_double), ("dtmin", C.c_double),
                ("finc", C.c_double), ("fdec", C.c_double), ("alpha0", C.c_double),
                ("falpha", C.c_double), ("ndelay", C.c_int64), ("nneg_max", C.c_int64),
                ("maxiter", C.c_int64), ("initial_delay", C.c_int64), ("ftol", C.c_double),
                ("etol", C.c_double)]


class FireResult(C.Structure):
    _fields_ = [("iters", C.c_int64), ("builds", C.c_int64), ("fmax", C.c_double),
                ("energy", C.c_double), ("status", C.c_int64)]


def fire_params(dt0=0.05, ftol=1e-10, maxiter=100000, etol=0.0, **kw) -> FireParams:
    """FIRE 2.0 defaults of the publication the paper cites (Guenole et al. 2020):
    N_delay=20, f_inc=1.1, f_dec=0.5, alpha_start=0.25, f_alpha=0.99,
    dt_max=10 dt0, dt_min=0.02 dt0, N_neg_max=2000, initial delay on."""
    p = dict(dt0=dt0, dtmax=10.0 * dt0, dtmin=0.02 * dt0, finc=1.1, fdec=0.5, alpha0=0.25,
             falpha=0.99, ndelay=20, nneg_max=2000, maxiter=maxiter, initial_delay=1, ftol=ftol,
             etol=etol)
    p.update(kw)
    return FireParams(**p)


_lib = None
_lib_omp = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        _lib = _configure(C.CDLL(LIB))
    return _lib


def lib_omp():
    """The OpenMP build (per-atom forces and per-subcell list build on all
    threads); only the CPU baseline uses it."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(LIB_OMP) or os.path.getmtime(LIB_OMP) < os.path.getmtime(SRC):
            build(force=True)
        _lib_omp = _configure(C.CDLL(LIB_OMP))
    return _lib_omp


def _configure(L):
    if True:
        L.orc_sphere_volume.restype = C.c_double
        L.orc_sphere_volume.argtypes = [C.c_int, C.c_double]
        L.orc_set_morse_a.restype = None
        L.orc_set_morse_a.argtypes = [C.c_double]
        L.orc_ncell.restype = C.c_int
        L.orc_ncell.argtypes = [C.c_double, C.c_double]
        L.orc_wrap1.restype = C.c_double
        L.orc_wrap1.argtypes = [C.c_double, C.c_double]
        for name in ("orc_nlist_brute",):
            f = getattr(L, name)
            f.restype = C.c_void_p
            f.argtypes = [C.c_int, C.c_int64, C.c_double, _dp, _dp, C.c_double, C.c_double]
        L.orc_nlist_cells.restype = C.c_void_p
        L.orc_nlist_cells.argtypes = [C.c_int, C.c_int64, C.c_double, _dp, _dp, C.c_double,
                                      C.c_double, C.c_int]
        L.orc_nlist_row.restype = C.c_int64
        L.orc_nlist_row.argtypes = [C.c_int, C.c_int64, C.c_double, _dp, _dp, C.c_double,
                                    C.c_double, C.c_int64, _i32p, C.c_int64]
        L.orc_list_nnz.restype = C.c_int64
        L.orc_list_nnz.argtypes = [C.c_void_p]
        L.orc_list_copy.restype = None
        L.orc_list_copy.argtypes = [C.c_void_p, _i64p, _i32p]
        L.orc_list_free.restype = None
        L.orc_list_free.argtypes = [C.c_void_p]
        L.orc_forces.restype = C.c_double
        L.orc_forces.argtypes = [C.c_int, C.c_int64, C.c_double, _dp, _dp, C.c_int, C.c_double,
                                 C.c_double, _i64p, _i32p, _dp, _dp]
        L.orc_virial.restype = None
        L.orc_virial.argtypes = [C.c_int, C.c_int64, C.c_double, _dp, _dp, C.c_int, C.c_double,
                                 C.c_double, _i64p, _i32p, _dp]
        L.orc_force_one.restype = C.c_double
        L.orc_force_one.argtypes = [C.c_int, C.c_int64, C.c_double, _dp, _dp, C.c_int,
                                    C.c_double, C.c_double, C.c_int64, _dp]
        L.orc_vv.restype = C.c_int64
        L.orc_vv.argtypes = [C.c_int, C.c_int64, C.c_double, C.c_int, C.c_double, C.c_double,
                             C.c_double, _dp, _dp, _dp, C.c_int64, C.c_double, C.c_double,
                             C.c_double, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_swap.restype = C.c_int64
        L.orc_swap.argtypes = [C.c_int, C.c_int64, C.c_double, _dp, _dp, C.c_int, C.c_double,
                               C.c_double, C.c_int64, _i32p, _dp, C.c_double, _i32p, _dp]
        L.orc_van_hove.restype = None
        L.orc_van_hove.argtypes = [C.c_int, C.c_int64, _dp, C.c_int32, C.c_double, _i64p]
        L.orc_disp_moments.restype = None
        L.orc_disp_moments.argtypes = [C.c_int, C.c_int64, _dp, _dp]
        L.orc_fire.restype = None
        L.orc_fire.argtypes = [C.c_int, C.c_int64, C.c_double, C.c_int, C.c_double, C.c_double,
                               C.c_double, _dp, _dp, C.POINTER(FireParams),
                               C.POINTER(FireResult)]
        L.orc_fire_traced.restype = None
        L.orc_fire_traced.argtypes = [C.c_int, C.c_int64, C.c_double, C.c_int, C.c_double,
                                      C.c_double, C.c_double, _dp, _dp, C.POINTER(FireParams),
                                      C.POINTER(FireResult), C.c_void_p, C.c_int64]
    return L


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_morse_a(a: float) -> None:
    """Morse stiffness for every later call (default 30, the paper's value)."""
    lib().orc_set_morse_a(a)


def sphere_volume(d: int, sigma: float) -> float:
    return lib().orc_sphere_volume(d, sigma)


def ncell(L: float, rlmax: float) -> int:
    return lib().orc_ncell(L, rlmax)


def wrap(x, L):
    w = lib().orc_wrap1
    x = _f64(x)
    return np.vectorize(lambda t: w(float(t), L))(x) if x.size else x.copy()


def _take_list(h, n, L=None):
    L = L or lib()
    nnz = L.orc_list_nnz(h)
    rp = np.zeros(n + 1, dtype=np.int64)
    cols = np.zeros(max(nnz, 1), dtype=np.int32)
    L.orc_list_copy(h, rp, cols)
    L.orc_list_free(h)
    return rp, cols[:nnz]


def nlist_brute(x, sig, L, c, s):
    """Definition of the Verlet list: CSR (row_ptr, cols), rows ascending."""
    x = _f64(x)
    n, d = x.shape
    return _take_list(lib().orc_nlist_brute(d, n, L, x, _f64(sig), c, s), n)


def nlist_cells(x, sig, L, c, s, ncell_override=0, omp=False):
    """The paper's subcell algorithm; canonical CSR (rows ascending).  omp:
    the OpenMP build (same rows)."""
    x = _f64(x)
    n, d = x.shape
    lb = lib_omp() if omp else lib()
    return _take_list(lb.orc_nlist_cells(d, n, L, x, _f64(sig), c, s, ncell_override), n, lb)


def nlist_row(x, sig, L, c, s, i):
    x = _f64(x)
    n, d = x.shape
    sig = _f64(sig)
    cap = 4096
    while True:
        out = np.zeros(cap, dtype=np.int32)
        m = lib().orc_nlist_row(d, n, L, x, sig, c, s, i, out, cap)
        if m <= cap:
            return out[:m]
        cap = int(m)


def forces(x, sig, L, pot, c, eps, rp, cols, omp=False):
    """(F (n,d), per-atom energy (n,), total energy) from a CSR list.  omp: the
    OpenMP build (same forces; the total energy summed in another order)."""
    x = _f64(x)
    n, d = x.shape
    F = np.zeros((n, d))
    e = np.zeros(n)
    E = (lib_omp() if omp else lib()).orc_forces(d, n, L, x, _f64(sig), pot, c, eps, np.ascontiguousarray(rp, np.int64),
                         np.ascontiguousarray(cols, np.int32), F, e)
    return F, e, E


def virial(x, sig, L, pot, c, eps, rp, cols):
    """(W, Z): sum over pairs of r_ij . F_ij, and mean neighbours inside the cutoff."""
    x = _f64(x)
    n, d = x.shape
    out = np.zeros(2)
    lib().orc_virial(d, n, L, x, _f64(sig), pot, c, eps, np.ascontiguousarray(rp, np.int64),
                     np.ascontiguousarray(cols, np.int32), out)
    return float(out[0]), float(out[1])


def force_one(x, sig, L, pot, c, eps, i):
    x = _f64(x)
    n, d = x.shape
    Fi = np.zeros(d)
    ei = lib().orc_force_one(d, n, L, x, _f64(sig), pot, c, eps, i, Fi)
    return Fi, ei


def vv(x, v, sig, L, pot, c, s, eps, nsteps, dt, obs=False, tau=0.0, T0=0.0):
    """Run velocity Verlet (NVE, or with the Berendsen thermostat when tau > 0);
    returns (x, v, thermo[nsteps+1, 2] = (KE, PE), builds) and, with obs, also
    the displacement observables [nsteps+1, 4] = (<|dr|^2>, <|dr|^4>, alpha_2,
    f_ov) since step 0 and the final unwrapped displacements dr[n, d] (Sec. II.E)."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    n, d = x.shape
    th = np.zeros((nsteps + 1, 2))
    ob = np.zeros((nsteps + 1, 4)) if obs else None
    dr = np.zeros((n, d)) if obs else None
    b = lib().orc_vv(d, n, L, pot, c, s, eps, x, v, _f64(sig), nsteps, dt, tau, T0,
                     th.ctypes.data_as(C.c_void_p),
                     ob.ctypes.data_as(C.c_void_p) if obs else None,
                     dr.ctypes.data_as(C.c_void_p) if obs else None)
    return (x, v, th, b, ob, dr) if obs else (x, v, th, b)


def swap(x, sig, L, pot, c, eps, pairs, u, T):
    """SWAP Monte Carlo attempts in order (Sec. II.D); returns (new diameters,
    accepted flags, energy changes dE, number accepted)."""
    x = _f64(x)
    n, d = x.shape
    sig = _f64(sig).copy()
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    m = len(pairs)
    acc = np.zeros(m, dtype=np.int32)
    de = np.zeros(m)
    na = lib().orc_swap(d, n, L, x, sig, pot, c, eps, m, pairs.ravel(), _f64(u), T, acc, de)
    return sig, acc, de, na


def van_hove(dr, nbins, w):
    """Displacement-length histogram behind G_s(r) (eq. VGC): nbins + 1 counts,
    the last one for |dr| >= nbins * w."""
    dr = _f64(dr)
    n, d = dr.shape
    h = np.zeros(nbins + 1, dtype=np.int64)
    lib().orc_van_hove(d, n, dr, nbins, w, h)
    return h


def disp_moments(dr):
    """(<|dr|^2>, <|dr|^4>, alpha_2, f_ov) of unwrapped displacements dr[n, d]
    (Sec. II.E, eqs. ngp and fov)."""
    dr = _f64(dr)
    n, d = dr.shape
    out = np.zeros(4)
    lib().orc_disp_moments(d, n, dr, out)
    return out


FIRE_TRACE_COLS = ("P", "dt", "alpha", "npos", "nneg", "back")


def fire(x, sig, L, pot, c, s, eps, params: FireParams, trace: bool = False):
    """FIRE 2.0 minimisation (Sec. II.B).  Returns (x, result) and, with trace,
    also one row per iteration of FIRE_TRACE_COLS: the power P = F.v, the dt
    and alpha the update used, the P > 0 / P <= 0 run counts after the control
    step and 1 where the iteration stepped back and zeroed v."""
    x = _f64(x).copy()
    n, d = x.shape
    res = FireResult()
    if not trace:
        lib().orc_fire(d, n, L, pot, c, s, eps, x, _f64(sig), C.byref(params), C.byref(res))
        return x, res
    cap = int(params.maxiter)
    tr = np.zeros((max(cap, 1), len(FIRE_TRACE_COLS)))
    lib().orc_fire_traced(d, n, L, pot, c, s, eps, x, _f64(sig), C.byref(params), C.byref(res),
                          tr.ctypes.data_as(C.c_void_p), cap)
    return x, res, tr[:min(int(res.iters), cap)]
