"""GPU FIRE 2.0 against the oracle: short horizon, convergence, and the
oracle's force definition evaluated at the GPU's minimum."""
import numpy as np
import pytest

from paper_2112_12271_amd import hdmd as H
from paper_2112_12271_amd import inputs
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


def _jam_case(d, n, phi, seed):
    sig = inputs.bidisperse(n, 1.0, 1.4, seed)
    L = inputs.box_for_packing(d, sig, phi)
    x = inputs.uniform_positions(n, d, L, seed + 1)
    return x, sig, L


def _gpu_fire(sysd, x, sig, params):
    sysf, ws = H.build_with_width(sysd, dev(x), dev(sig))
    X = dev(x)
    res = H.hdmd_fire_minimize(sysf, X, dev(sig), ws, params)
    return X.cpu().numpy(), res


@pytest.mark.parametrize("d,n,phi", [(3, 300, 0.6), (4, 400, 0.45), (6, 500, 0.2)])
def test_short_horizon_matches_oracle(orc, d, n, phi):
    x, sig, L = _jam_case(d, n, phi, 10 * d)
    for iters in (5, 40):
        po = orc.fire_params(dt0=0.05, ftol=1e-14, maxiter=iters)
        xo, ro = orc.fire(x, sig, L, 1, 1.0, 0.25, 1.0, po)
        pg = H.hdmd_fire_defaults(0.05, 1e-14, iters)
        sysd = H.System(d=d, n=n, box_l=L, potential=H.HDMD_HARMONIC, cutoff=1.0, skin=0.25,
                        sigma_max=1.4)
        xg, rg = _gpu_fire(sysd, x, sig, pg)
        assert rg.iterations == ro.iters == iters
        dx = xg - xo
        dx -= L * np.round(dx / L)
        assert np.abs(dx).max() < 1e-9
        assert rg.energy == pytest.approx(ro.energy, rel=1e-9)


def test_below_jamming_reaches_zero_energy():
    x, sig, L = _jam_case(3, 400, 0.45, 5)
    sysd = H.System(d=3, n=400, box_l=L, potential=H.HDMD_HARMONIC, cutoff=1.0, skin=0.25,
                    sigma_max=1.4)
    xg, res = _gpu_fire(sysd, x, sig, H.hdmd_fire_defaults(0.05, 1e-10, 100000))
    assert res.status == 0 and res.fmax < 1e-10
    assert res.energy / 400 < 1e-18


@pytest.mark.parametrize("prec,tol", [(H.HDMD_FP64, 1e-10), (H.HDMD_MIXED, 1e-5)])
def test_jammed_minimum_checked_by_oracle(orc, prec, tol):
    """A jammed packing: the GPU's final state has |F|max below tol under the
    oracle's own force definition (FP64)."""
    d, n = 3, 256
    x, sig, L = _jam_case(d, n, 0.75, 8)
    sysd = H.System(d=d, n=n, box_l=L, potential=H.HDMD_HARMONIC, cutoff=1.0, skin=0.25,
                    sigma_max=1.4, precision=prec)
    xg, res = _gpu_fire(sysd, x, sig, H.hdmd_fire_defaults(0.05, tol, 200000))
    assert res.status == 0 and res.fmax < tol
    assert res.energy / n > 1e-8
    rp, cols = orc.nlist_brute(xg, sig, L, 1.0, 0.25)
    F, _, E = orc.forces(xg, sig, L, 1, 1.0, 1.0, rp, cols)
    assert np.sqrt((F * F).sum(axis=1)).max() < (tol if prec == H.HDMD_FP64 else 10 * tol)
    assert E == pytest.approx(res.energy, rel=1e-9 if prec == H.HDMD_FP64 else 1e-4)


def test_two_particles_separate():
    x = np.array([[0.0, 0.0, 0.0], [0.5, 0.2, 0.0]])
    sig = np.array([1.0, 1.4])
    sysd = H.System(d=3, n=2, box_l=6.0, potential=H.HDMD_HARMONIC, cutoff=1.0, skin=0.25,
                    sigma_max=1.4)
    xg, res = _gpu_fire(sysd, x, sig, H.hdmd_fire_defaults(0.05, 1e-12, 10000))
    assert res.status == 0
    assert np.linalg.norm(xg[0] - xg[1]) >= 1.2 * (1 - 1e-10)


def test_workspace_reused_across_potentials():
    """One workspace serves a harmonic and then a Morse minimisation of the same
    size: the Morse result equals the one on a fresh workspace (the captured
    launch chunks are keyed by the force kernel's potential class)."""
    d, n = 4, 500
    sig = inputs.bidisperse(n, 1.0, 1.4, 11)
    L = inputs.box_for_packing(d, sig, 0.48)
    x = inputs.uniform_positions(n, d, L, 12)
    kw = dict(d=d, n=n, box_l=L, cutoff=1.0, skin=0.25, sigma_max=1.4, max_neighbors=96)
    sys_h = H.System(potential=H.HDMD_HARMONIC, **kw)
    sys_m = H.System(potential=H.HDMD_MORSE, morse_a=5.0, **kw)
    p = H.hdmd_fire_defaults(0.05, 1e-10, 300)
    Xh = dev(x)
    H.hdmd_fire_minimize(sys_h, Xh, dev(sig), H.workspace(sys_h), p)   # relaxed start
    x0 = Xh.cpu().numpy()
    ws = H.workspace(sys_m)
    Xa = dev(x0)
    H.hdmd_fire_minimize(sys_h, Xa, dev(sig), ws, p)                    # harmonic on ws
    Xb, Xc = dev(x0), dev(x0)
    rb = H.hdmd_fire_minimize(sys_m, Xb, dev(sig), ws, p)               # Morse on the same ws
    rc = H.hdmd_fire_minimize(sys_m, Xc, dev(sig), H.workspace(sys_m), p)
    assert rb.iterations == rc.iterations and rb.energy == rc.energy
    assert np.array_equal(Xb.cpu().numpy(), Xc.cpu().numpy())
    assert rb.energy > 0.0
