"""Batched uneven replicas: each result in the mix equals the same system run
alone, bit for bit (FIRE and MD), including slots admitted mid-run, and every
slot's result is checked against the oracle: FIRE positions after 5 and 40
iterations, converged states under the oracle's forces, MD trajectories."""
import numpy as np
import pytest
import torch

from paper_2112_12271_amd import hdmd as H
from paper_2112_12271_amd import inputs
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


def _fire_case(d, n, phi, seed, pot=H.HDMD_HARMONIC):
    sig = inputs.bidisperse(n, 1.0, 1.4, seed)
    L = inputs.box_for_packing(d, sig, phi)
    x = inputs.uniform_positions(n, d, L, seed + 1)
    if pot == H.HDMD_MORSE:
        # the Morse minimisation starts from the harmonic jammed packing (the
        # uniform start's deep overlaps would throw atoms many boxes per step)
        X = dev(x)
        sysh = H.System(d=d, n=n, box_l=L, potential=H.HDMD_HARMONIC, cutoff=1.0, skin=0.25,
                        sigma_max=1.4, max_neighbors=64)
        H.fire_auto(sysh, X, dev(sig), H.hdmd_fire_defaults(0.05, 1e-8, 2000))
        x = X.cpu().numpy()
    # a = 5: a Morse wall on the time scale of the other systems' FIRE step
    sysd = H.System(d=d, n=n, box_l=L, potential=pot, cutoff=1.0, skin=0.25,
                    sigma_max=1.4, max_neighbors=64, morse_a=5.0)
    sysd, _ = H.build_with_width(sysd, dev(x), dev(sig), slack=2.0)
    return sysd, x, sig


def _oracle_fmax(orc, sysd, x, sig):
    """max_i |F_i| of the oracle's forces at x (the oracle's own list)."""
    if sysd.potential == H.HDMD_MORSE:
        orc.set_morse_a(sysd.morse_a)
    try:
        rp, cols = orc.nlist_cells(x, sig, sysd.box_l, sysd.cutoff, sysd.skin)
        F, _, _ = orc.forces(x, sig, sysd.box_l, sysd.potential, sysd.cutoff, 1.0, rp, cols)
    finally:
        orc.set_morse_a(30.0)
    return float(np.sqrt((F * F).sum(axis=1)).max())


def _alone_fire(sysd, x, sig, params):
    """Runs alone (regrowing the row width if a row overflows) and returns the
    final positions, result and the width used, which the batch then reuses:
    the width only sizes the workspace, it does not change any result."""
    X = dev(x)
    sysf, res = H.fire_auto(sysd, X, dev(sig), params)
    return X.cpu().numpy(), res, sysf


# the last two: a Morse system (its own force launch) and a d = 9 system (the
# classes above 8 keep per-class build and force launches)
CASES = [(3, 700, 0.62, 1), (4, 450, 0.44, 2), (5, 900, 0.3, 3), (6, 1300, 0.2, 4),
         (3, 2500, 0.66, 5), (6, 600, 0.22, 6), (4, 500, 0.48, 7, H.HDMD_MORSE),
         (9, 3100, 0.02, 8)]


def _run_batch(systems, params, max_slots=8):
    """All systems in one batch; returns {slot: (positions, result)}."""
    B = H.Batch(max_slots=max_slots, max_atoms=30000, max_cells=200000)
    keep = []
    for k, (s, x, sig) in enumerate(systems):
        ws = H.workspace(s)
        X, SG = dev(x), dev(sig)
        keep.append((X, SG, ws))
        B.hdmd_batch_add_fire(k, s, X, SG, ws, params)
    done = {}
    for _ in range(10000):
        B.hdmd_batch_run(25)
        state, _ = B.hdmd_batch_poll()
        for k in range(len(systems)):
            if k not in done and state[k] == H.HDMD_SLOT_DONE:
                pos, _, res = B.hdmd_batch_take(k)
                done[k] = (pos.cpu().numpy(), res)
        if len(done) == len(systems):
            return done
    raise AssertionError("batch did not finish")


@pytest.mark.parametrize("iters", [5, 40])
def test_fire_batch_matches_oracle_short_horizon(orc, iters):
    """Every class of the batch (d = 3..6, the Morse system, d = 9) after 5 and
    40 FIRE iterations in one batch: positions within 1e-9 of the oracle's
    FIRE 2.0 (FP64)."""
    params = H.hdmd_fire_defaults(0.05, 1e-12, iters)
    systems = [_fire_case(*case) for case in CASES]
    # the row capacity each system needs over these iterations, from a lone run
    systems = [(_alone_fire(s, x, sig, params)[2], x, sig) for s, x, sig in systems]
    done = _run_batch(systems, params)
    for k, (s, x, sig) in enumerate(systems):
        xb, rb = done[k]
        assert rb.iterations == iters, k
        if s.potential == H.HDMD_MORSE:
            orc.set_morse_a(s.morse_a)
        try:
            xo, ro = orc.fire(x, sig, s.box_l, s.potential, s.cutoff, s.skin, 1.0,
                              orc.fire_params(dt0=0.05, ftol=1e-12, maxiter=iters))
        finally:
            orc.set_morse_a(30.0)
        assert ro.iters == iters
        dx = xb - xo
        dx -= s.box_l * np.round(dx / s.box_l)
        assert np.abs(dx).max() < 1e-9, (k, np.abs(dx).max())


@pytest.mark.parametrize("prec", [H.HDMD_FP64, H.HDMD_MIXED])
def test_fire_mix_equals_alone(orc, prec):
    params = H.hdmd_fire_defaults(0.05, 1e-10 if prec == H.HDMD_FP64 else 1e-5, 3000)
    systems = []
    for case in CASES:
        sysd, x, sig = _fire_case(*case)
        sysd.precision = prec
        systems.append((sysd, x, sig))
    alone = [_alone_fire(s, x, sig, params) for s, x, sig in systems]
    systems = [(a[2], x, sig) for a, (s, x, sig) in zip(alone, systems)]
    B = H.Batch(max_slots=8, max_atoms=30000, max_cells=200000)
    keep = []
    for k, (s, x, sig) in enumerate(systems[:4]):
        ws = H.workspace(s)
        X, SG = dev(x), dev(sig)
        keep.append((X, SG))
        B.hdmd_batch_add_fire(k, s, X, SG, ws, params)
    done = {}
    admitted = 4
    for rnd in range(10000):
        B.hdmd_batch_run(25)
        state, iters = B.hdmd_batch_poll()
        for k in range(8):
            if state[k] == H.HDMD_SLOT_DONE:
                pos, _, res = B.hdmd_batch_take(k)
                done[k if k < 4 else k] = (pos.cpu().numpy(), res)
        # admit the remaining systems into fresh slots while others run
        if rnd == 2:
            for k in range(4, len(systems)):
                s, x, sig = systems[k]
                ws = H.workspace(s)
                X, SG = dev(x), dev(sig)
                keep.append((X, SG))
                B.hdmd_batch_add_fire(k, s, X, SG, ws, params)
            admitted = len(systems)
        if len(done) == admitted == len(systems):
            break
    assert len(done) == len(systems)
    for k in range(len(systems)):
        xb, rb = done[k]
        xa, ra, _ = alone[k]
        assert rb.iterations == ra.iterations, k
        assert rb.status == ra.status
        assert np.array_equal(xb, xa), k
        assert rb.energy == ra.energy
        # a converged slot is a minimum under the oracle's own forces (the
        # precision form stores forces in FP32, so its bound has room for that)
        if rb.status == 0:
            s, x, sig = systems[k]
            tol = params.f_tol if prec == H.HDMD_FP64 else 1.5 * params.f_tol
            assert _oracle_fmax(orc, s, xb, sig) < tol, k


def test_md_mix_equals_alone(orc):
    """Classes holding systems of both precision forms (d = 4) and of both
    potential classes (d = 3) take one step launch per kind; a slot with the
    Berendsen thermostat (d = 5) runs as it does alone.  Every slot's final
    positions and velocities against the oracle's velocity Verlet: within
    1e-9 / 1e-8 (FP64), 1e-4 (the precision form)."""
    W, M = H.HDMD_WCA, H.HDMD_MORSE
    cases = [(3, 8, 1.12, 1, H.HDMD_FP64, W, 0.0), (4, 5, 1.1, 2, H.HDMD_FP64, W, 0.0),
             (6, 4, 1.05, 3, H.HDMD_FP64, W, 0.0), (4, 5, 1.12, 4, H.HDMD_MIXED, W, 0.0),
             (3, 8, 1.15, 5, H.HDMD_FP64, M, 0.0), (5, 4, 1.1, 6, H.HDMD_FP64, W, 0.05)]
    nsteps, dt = 60, 0.003
    alone, states = [], []
    for d, m, a, seed, prec, pot, tau in cases:
        x, L = inputs.jittered_lattice(d, m, a, (0.12 if pot == W else 0.02) * a, seed)
        n = len(x)
        sig = inputs.bidisperse(n, 1.0, 1.2 if pot == W else 1.1, seed)
        v = inputs.gaussian_velocities(n, d, 1.0 if pot == W else 0.25, seed + 1)
        sysd = H.System(d=d, n=n, box_l=L, potential=pot,
                        cutoff=inputs.WCA_CUT if pot == W else 1.0, skin=0.3, sigma_max=1.2,
                        precision=prec, max_neighbors=64, thermostat_tau=tau, target_temp=0.4)
        sysd, _ = H.build_with_width(sysd, dev(x), dev(sig), slack=2.0)
        ws = H.workspace(sysd)
        X, V = dev(x), dev(v)
        H.hdmd_step(sysd, X, V, dev(sig), ws, nsteps, dt)
        alone.append((X.cpu().numpy(), V.cpu().numpy()))
        states.append((sysd, x, v, sig))
        # the oracle's trajectory of the same slot
        xo, vo, _, _ = orc.vv(x, v, sig, L, pot, sysd.cutoff, sysd.skin, 1.0, nsteps, dt,
                              tau=tau, T0=0.4 if tau else 0.0)
        dx = X.cpu().numpy() - xo
        dx -= L * np.round(dx / L)
        tx, tv = (1e-9, 1e-8) if prec == H.HDMD_FP64 else (1e-4, 1e-4)
        assert np.abs(dx).max() < tx, (d, prec, pot, np.abs(dx).max())
        assert np.abs(V.cpu().numpy() - vo).max() < tv, (d, prec, pot)
    B = H.Batch(max_slots=8, max_atoms=10000, max_cells=100000)
    for k, (s, x, v, sig) in enumerate(states):
        B.hdmd_batch_add_md(k, s, dev(x), dev(v), dev(sig), H.workspace(s), nsteps, dt)
    for _ in range(100):
        B.hdmd_batch_run(10)
        state, iters = B.hdmd_batch_poll()
        if all(state[k] == H.HDMD_SLOT_DONE for k in range(len(states))):
            break
    for k in range(len(states)):
        pos, vel, res = B.hdmd_batch_take(k, want_vel=True)
        assert res.iterations == nsteps
        assert np.array_equal(pos.cpu().numpy(), alone[k][0])
        assert np.array_equal(vel.cpu().numpy(), alone[k][1])
