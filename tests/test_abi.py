"""The C ABI on the CPU: the library loads, exports every function the header
declares, and its host-only planning calls (no device work) behave as the
header documents.  No compute call is made here."""
import ctypes
import dataclasses
import math

import pytest

from paper_2112_12271_amd import hdmd as H


def test_library_exports_every_header_symbol():
    names = H.header_symbols()
    assert len(names) == 22
    raw = ctypes.CDLL(H.LIB_PATH)
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing
    # the binding knows the signature of every declared function
    assert set(names) == set(H._SIGS), set(names) ^ set(H._SIGS)


def test_binding_uses_native_library():
    L = H.lib()
    assert L._name == H.LIB_PATH


def test_fire_defaults_are_fire2_defaults():
    p = H.hdmd_fire_defaults(dt0=0.05, f_tol=1e-7, max_iter=1234)
    assert (p.dt0, p.dt_max, p.dt_min) == (0.05, 0.5, 0.001)
    assert (p.f_inc, p.f_dec, p.alpha0, p.f_alpha) == (1.1, 0.5, 0.25, 0.99)
    assert (p.n_delay, p.n_neg_max, p.max_iter, p.initial_delay) == (20, 2000, 1234, 1)
    assert p.f_tol == 1e-7


def _sys(**kw):
    base = dict(d=6, n=262144, box_l=11.0, potential=H.HDMD_WCA, cutoff=H.WCA_CUT, skin=0.25,
                sigma_max=1.2, precision=H.HDMD_FP64, max_neighbors=256)
    base.update(kw)
    return H.System(**base)


def test_cells_per_axis_follows_subcell_rule():
    # eq. setnc: n_cell = floor(L / (c sigma_max + s)) ...
    rl = H.WCA_CUT * 1.2 + 0.25
    for d, L in [(3, 10.0), (4, 9.0), (6, 11.0), (8, 5.0)]:
        s = _sys(d=d, box_l=L, n=4 * 4 ** d)
        assert H.hdmd_cells_per_axis(s) == math.floor(L / rl)
    # ... lowered while the subcell count exceeds four per atom
    s = _sys(d=4, box_l=20.0, n=100)         # floor(20/1.597)=12; 12^4 > 400 -> 4^4=256
    assert H.hdmd_cells_per_axis(s) == 4
    # a box exactly n_cell list radii wide keeps n_cell (rounding guard only lowers it
    # when a subcell is narrower than the radius by more than rounding)
    s = _sys(d=3, box_l=5 * rl, n=4000)
    assert H.hdmd_cells_per_axis(s) in (4, 5)
    s = _sys(d=3, box_l=5 * rl * (1 - 1e-6), n=4000)
    assert H.hdmd_cells_per_axis(s) == 4


def test_half_size_subcells_follow_their_rule():
    # half-size subcells (Sec. II.C): floor(2 L / r_l,max) per axis, at least 5
    rl = H.WCA_CUT * 1.2 + 0.25
    for d, L in [(2, 10.0), (3, 10.0), (4, 9.0), (6, 11.0)]:
        s = _sys(d=d, box_l=L, n=4 * 4 ** d, subcells=H.HDMD_SUBCELLS_HALF)
        assert H.hdmd_cells_per_axis(s) == math.floor(2 * L / rl)
        tuned, reach, nc, var, lanes = H.hdmd_build_config(s)
        assert (reach, nc) == (2, math.floor(2 * L / rl))
    # fewer than five per axis: the 5^d stencil would alias -> refused
    s = _sys(d=3, box_l=2.4 * rl, n=100, subcells=H.HDMD_SUBCELLS_HALF)
    assert H.hdmd_cells_per_axis(s) == H.HDMD_ERR_ARG
    assert "5 r_l,max / 2" in H.last_error()
    s = _sys(d=3, box_l=2.5 * rl * (1 + 1e-9), n=100, subcells=H.HDMD_SUBCELLS_HALF)
    assert H.hdmd_cells_per_axis(s) == 5
    # an unknown grid value is an argument error
    assert H.hdmd_cells_per_axis(_sys(subcells=3)) == H.HDMD_ERR_ARG


def test_autotuned_grid_before_any_build():
    # before its first build an autotuned system reports the defaults: subcells
    # of side >= r_l,max and the one-wave candidate-lane build; its workspace
    # holds the cell arrays of the half-size grid too, where that grid applies
    rl = H.WCA_CUT * 1.2 + 0.25
    s = _sys(d=3, box_l=30.0, n=20000)
    tuned, reach, nc, var, lanes = H.hdmd_build_config(s)
    assert (tuned, reach, nc) == (False, 1, math.floor(30.0 / rl))
    assert var in (1, 2, 4, 64, 128, 256)
    full = H.hdmd_workspace_bytes(dataclasses.replace(s, subcells=H.HDMD_SUBCELLS_FULL))
    half = H.hdmd_workspace_bytes(dataclasses.replace(s, subcells=H.HDMD_SUBCELLS_HALF))
    auto = H.hdmd_workspace_bytes(s)
    nh = math.floor(2 * 30.0 / rl)
    assert auto >= full and auto - full >= 12 * (nh ** 3 - math.floor(30.0 / rl) ** 3) - 6 * 256
    assert half >= full - 16 * 20032  # no 16-bit wrapped copies on the half grid
    assert H.hdmd_cells_per_axis(s) == math.floor(30.0 / rl)


def test_cells_per_axis_rejects_tiny_box():
    s = _sys(d=3, box_l=2.0, n=10)          # L < 2 c sigma_max
    assert H.hdmd_cells_per_axis(s) == H.HDMD_ERR_BOX


@pytest.mark.parametrize("bad", [dict(d=1), dict(d=11), dict(n=0), dict(skin=-0.1),
                                 dict(max_neighbors=0), dict(box_l=float("nan")),
                                 dict(thermostat_tau=-1.0), dict(target_temp=float("inf"))])
def test_invalid_system_has_no_workspace(bad):
    assert H.lib().hdmd_workspace_bytes(ctypes.byref(_sys(**bad).c())) == 0
    with pytest.raises(H.HdmdError):
        H.hdmd_workspace_bytes(_sys(**bad))


def test_workspace_grows_with_row_capacity_and_precision_form():
    a = H.hdmd_workspace_bytes(_sys(max_neighbors=128))
    b = H.hdmd_workspace_bytes(_sys(max_neighbors=256))
    assert a > 0 and b > a
    # the row array alone accounts for the difference (128 int32 entries per atom or more)
    assert b - a >= 128 * 4 * 262144
    m = H.hdmd_workspace_bytes(_sys(precision=H.HDMD_MIXED))
    assert m > 0


def test_batch_bytes_host_only():
    L = H.lib()
    assert L.hdmd_batch_bytes(0, 10, 10) == 0
    assert L.hdmd_batch_bytes(4, 1 << 16, 1 << 12) > 0
    assert L.hdmd_batch_bytes(8, 1 << 16, 1 << 12) >= L.hdmd_batch_bytes(4, 1 << 16, 1 << 12)
    assert L.hdmd_batch_bytes(1025, 10, 10) == 0


def test_binding_constants_match_the_header():
    """The binding's thermo-row width and potential codes are the header's."""
    import re
    hdr = open(H.HEADER).read()
    assert int(re.search(r"#define HDMD_THERMO_COLS (\d+)", hdr).group(1)) == H.THERMO_COLS
    for name in ("HDMD_WCA", "HDMD_HARMONIC", "HDMD_MORSE", "HDMD_FP64", "HDMD_MIXED"):
        m = re.search(name + r"\s*=\s*(\d+)", hdr)
        assert m and int(m.group(1)) == getattr(H, name), name
