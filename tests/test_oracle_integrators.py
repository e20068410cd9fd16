"""Pins of the oracle's velocity Verlet and FIRE 2.0 (CPU only)."""
import numpy as np
import pytest

from paper_2112_12271_amd import inputs

C6 = 2.0 ** (1.0 / 6.0)


def _fluid(d=3, m=5, a=1.12, seed=0, T=0.5, jitter=0.15):
    x, L = inputs.jittered_lattice(d, m, a, jitter, seed)
    n = len(x)
    sig = inputs.bidisperse(n, 1.0, 1.1, seed)
    v = inputs.gaussian_velocities(n, d, T, seed + 1)
    return x, v, sig, L


@pytest.mark.parametrize("pot,c,dts", [(0, C6, (0.004, 0.002)), (2, 1.0, (0.0032, 0.0016))])
def test_vv_energy_error_scales_as_dt_squared(orc, pot, c, dts):
    """Energy fluctuation of velocity Verlet ~ dt^2: WCA, and the Morse potential
    (a = 30) at twice and at the paper's step dt = 6/(125 a) = 0.0016 (Sec. II.A),
    from a barely overlapping start."""
    x, v, sig, L = _fluid(jitter=0.15 if pot == 0 else 0.02)
    tot = 1.0 if pot == 0 else 0.5
    fl = []
    for dt in dts:
        _, _, th, _ = orc.vv(x, v, sig, L, pot, c, 0.3, 1.0, int(round(tot / dt)), dt)
        e = th.sum(axis=1)
        fl.append(np.sqrt(np.mean((e - e[0]) ** 2)))
    ratio = fl[0] / fl[1]
    assert 3.0 < ratio < 5.0, ratio


def test_vv_momentum_and_reversibility(orc):
    x, v, sig, L = _fluid(d=4, m=4, a=1.15, seed=3)
    n = 300
    x1, v1, th, builds = orc.vv(x, v, sig, L, 0, C6, 0.3, 1.0, n, 0.003)
    assert builds >= 2                       # the rebuild trigger fired during the run
    assert np.abs(v1.sum(axis=0) - v.sum(axis=0)).max() < 1e-11
    x2, v2, _, _ = orc.vv(x1, -v1, sig, L, 0, C6, 0.3, 1.0, n, 0.003)
    dx = x2 - x
    dx -= L * np.round(dx / L)
    assert np.abs(dx).max() < 1e-8
    assert np.abs(v2 + v).max() < 1e-8


def test_fire_two_overlapping_particles(orc):
    """Two overlapping harmonic spheres end exactly at contact or beyond: no force left."""
    x = np.array([[0.0, 0.0, 0.0], [0.5, 0.2, 0.0]])
    sig = np.array([1.0, 1.4])
    x1, res = orc.fire(x, sig, 6.0, 1, 1.0, 0.25, 1.0, orc.fire_params(ftol=1e-12))
    assert res.status == 0
    r = np.linalg.norm(x1[0] - x1[1])
    assert r >= 1.2 * (1 - 1e-10)
    assert res.energy < 1e-20


def test_fire_below_jamming_reaches_zero_energy(orc):
    d, n = 3, 256
    sig = inputs.bidisperse(n, 1.0, 1.4, 5)
    L = inputs.box_for_packing(d, sig, 0.45)
    x = inputs.uniform_positions(n, d, L, 6)
    x1, res = orc.fire(x, sig, L, 1, 1.0, 0.25, 1.0, orc.fire_params(ftol=1e-10))
    assert res.status == 0 and res.fmax < 1e-10
    assert res.energy / n < 1e-18


def test_fire_jammed_converges_with_positive_energy(orc):
    d, n = 3, 128
    sig = inputs.bidisperse(n, 1.0, 1.4, 8)
    L = inputs.box_for_packing(d, sig, 0.75)
    x = inputs.uniform_positions(n, d, L, 9)
    x1, res = orc.fire(x, sig, L, 1, 1.0, 0.25, 1.0, orc.fire_params(ftol=1e-10))
    assert res.status == 0 and res.fmax < 1e-10
    assert res.energy / n > 1e-6
    rp, cols = orc.nlist_brute(x1, sig, L, 1.0, 0.25)
    F, _, E = orc.forces(x1, sig, L, 1, 1.0, 1.0, rp, cols)
    assert np.sqrt((F * F).sum(axis=1)).max() < 1e-10
    assert E == pytest.approx(res.energy, rel=1e-12)


def _free_lattice(d, m=3, a=2.0):
    """Atoms on a lattice wider than the WCA range, all with one velocity: no
    force acts at any step."""
    x, L = inputs.jittered_lattice(d, m, a, 0.0, 0)
    n = len(x)
    vel = np.linspace(0.6, 1.4, d) * np.where(np.arange(d) % 2 == 0, 1.0, -1.0)
    return x, np.tile(vel, (n, 1)), np.ones(n), L


@pytest.mark.parametrize("d,tau_steps", [(3, 10.0), (4, 1.0), (5, 37.5)])
def test_berendsen_relaxes_free_atoms_geometrically(orc, d, tau_steps):
    """Without forces each step rescales v by lambda, so
    T_t - T0 = (1 - dt/tau)^t (T_0 - T0) exactly (tau = dt reaches T0 in one
    step), T = 2 KE / (d (n-1))."""
    x, v, sig, L = _free_lattice(d)
    n = len(x)
    dt, T0, nsteps = 0.01, 0.25, 200
    tau = tau_steps * dt
    _, _, th, _ = orc.vv(x, v, sig, L, 0, C6, 0.3, 1.0, nsteps, dt, tau=tau, T0=T0)
    T = 2.0 * th[:, 0] / (d * (n - 1))
    ref = T0 + (1.0 - dt / tau) ** np.arange(nsteps + 1) * (T[0] - T0)
    assert np.allclose(T, ref, rtol=1e-12, atol=1e-15)
    assert np.all(th[:, 1] == 0.0)


def test_berendsen_liquid_reaches_target(orc):
    """An interacting liquid started hot settles at the target temperature
    (time average over the second half within 3 %); tau = 0 is NVE bit for bit."""
    x, v, sig, L = _fluid(d=3, m=5, a=1.12, seed=7, T=1.5)
    n = len(x)
    dt, T0 = 0.004, 0.5
    _, _, th, _ = orc.vv(x, v, sig, L, 0, C6, 0.3, 1.0, 1500, dt, tau=0.1, T0=T0)
    T = 2.0 * th[:, 0] / (3 * (n - 1))
    assert abs(T[750:].mean() / T0 - 1.0) < 0.03
    a = orc.vv(x, v, sig, L, 0, C6, 0.3, 1.0, 50, dt)
    b = orc.vv(x, v, sig, L, 0, C6, 0.3, 1.0, 50, dt, tau=0.0, T0=T0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
