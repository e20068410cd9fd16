"""Lanes per atom of the force kernels (1, 2 or 4 lanes share an atom's row,
Sec. II.B getforce): forces, velocity-Verlet runs and FIRE against the
oracle with each count; batches whose systems take 2 or 4 lanes give the
bits of their lone runs; the autotuner's choice is recorded per key and
precision form and taken by later systems of the key."""
import os

import numpy as np
import pytest
import torch

from paper_2112_12271_amd import hdmd as H
from paper_2112_12271_amd import inputs
from tests.gpu_util import dev, force_err

pytestmark = pytest.mark.gpu
C6 = inputs.WCA_CUT


class _lanes:
    """HDMD_LPA set for the duration of a block (the forced lane count)."""

    def __init__(self, v):
        self.v = v

    def __enter__(self):
        self.old = os.environ.get("HDMD_LPA")
        os.environ["HDMD_LPA"] = str(self.v)

    def __exit__(self, *a):
        if self.old is None:
            os.environ.pop("HDMD_LPA", None)
        else:
            os.environ["HDMD_LPA"] = self.old


def _liquid(d, n, phi, seed, pot=H.HDMD_WCA):
    sig = inputs.bidisperse(n, 1.0, 1.2, seed)
    L = inputs.box_for_packing(d, sig, phi)
    x = inputs.uniform_positions(n, d, L, seed + 1)
    return x, sig, L


# jittered lattices (no deep overlaps: the precision form's bound holds) for
# d <= 8, a dilute uniform gas for d = 10
CASES = [(2, "lat", 50, 1.1), (3, "lat", 14, 1.1), (4, "lat", 7, 1.1), (6, "lat", 4, 1.1),
         (8, "lat", 3, 1.1), (10, "gas", 2000, 5e-4)]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("lanes", [1, 2, 4])
def test_forces_with_each_lane_count(orc, case, lanes):
    d, kind, m, a = case
    if kind == "lat":
        x, L = inputs.jittered_lattice(d, m, a, 0.15 * a, 10 * d)
        sig = inputs.bidisperse(len(x), 1.0, 1.2, 10 * d)
    else:
        x, sig, L = _liquid(d, m, a, 10 * d)
    n = len(x)
    rp, cols = orc.nlist_cells(x, sig, L, C6, 0.3)
    Fo, _, Eo = orc.forces(x, sig, L, H.HDMD_WCA, C6, 1.0, rp, cols)
    with _lanes(lanes):
        # forces: 1e-12 (FP64) and 1e-5 (precision form) of F_rms; energy: 1e-12
        # and 1e-8 relative (the precision form's fixed-point positions)
        for prec, ftol, etol in ((H.HDMD_FP64, 1e-12, 1e-12), (H.HDMD_MIXED, 1e-5, 1e-8)):
            sysd = H.System(d=d, n=n, box_l=L, cutoff=C6, skin=0.3, sigma_max=1.2, precision=prec)
            assert H.hdmd_build_config(sysd)[4] == lanes
            sysd, ws = H.build_with_width(sysd, dev(x), dev(sig))
            F, E = H.hdmd_forces(sysd, dev(x), dev(sig), ws)
            assert force_err(F.cpu().numpy(), Fo) < ftol, (prec, lanes)
            assert abs(float(E) - Eo) <= etol * abs(Eo), (prec, lanes)


@pytest.mark.parametrize("lanes", [2, 4])
def test_md_and_fire_with_more_lanes(orc, lanes):
    """60 velocity-Verlet steps (d = 4) and 40 FIRE iterations (d = 3) with 2
    and 4 lanes per atom: within 1e-9 of the oracle."""
    with _lanes(lanes):
        x, L = inputs.jittered_lattice(4, 7, 1.1, 0.13, 3)
        n = len(x)
        sig = inputs.bidisperse(n, 1.0, 1.2, 3)
        v = inputs.gaussian_velocities(n, 4, 1.0, 4)
        sysd = H.System(d=4, n=n, box_l=L, cutoff=C6, skin=0.3, sigma_max=1.2)
        sysd, st, _ = H.step_auto(sysd, X := dev(x), V := dev(v), dev(sig), 60, 0.004)
        xo, vo, _, bo = orc.vv(x, v, sig, L, H.HDMD_WCA, C6, 0.3, 1.0, 60, 0.004)
        dx = X.cpu().numpy() - xo
        dx -= L * np.round(dx / L)
        assert np.abs(dx).max() < 1e-9
        assert np.abs(V.cpu().numpy() - vo).max() < 1e-8
        x, sig, L = _liquid(3, 1500, 0.7, 5)
        sysf = H.System(d=3, n=1500, box_l=L, potential=H.HDMD_HARMONIC, cutoff=1.0, skin=0.25,
                        sigma_max=1.2)
        Xf = dev(x)
        _, res = H.fire_auto(sysf, Xf, dev(sig), H.hdmd_fire_defaults(0.05, 1e-12, 40))
        xo, ro = orc.fire(x, sig, L, H.HDMD_HARMONIC, 1.0, 0.25, 1.0,
                          orc.fire_params(dt0=0.05, ftol=1e-12, maxiter=40))
        dx = Xf.cpu().numpy() - xo
        dx -= L * np.round(dx / L)
        assert np.abs(dx).max() < 1e-9


@pytest.mark.parametrize("lanes", [2, 4])
def test_batch_with_more_lanes_equals_alone(lanes):
    """FIRE systems in the all-class launch's classes (d = 3, 5) and in a class
    of its own (d = 9), and an MD system, all with 2 or 4 lanes per atom: the
    batch takes a launch per class and kind for them and gives the lone bits."""
    params = H.hdmd_fire_defaults(0.05, 1e-10, 500)
    with _lanes(lanes):
        fire_cases = [(3, 1200, 0.62, 1), (5, 900, 0.3, 2), (9, 600, 0.002, 3)]
        systems, alone = [], []
        for d, n, phi, seed in fire_cases:
            sig = inputs.bidisperse(n, 1.0, 1.4, seed)
            L = inputs.box_for_packing(d, sig, phi)
            x = inputs.uniform_positions(n, d, L, seed + 1)
            s = H.System(d=d, n=n, box_l=L, potential=H.HDMD_HARMONIC, cutoff=1.0, skin=0.25,
                         sigma_max=1.4, max_neighbors=64)
            s, _ = H.build_with_width(s, dev(x), dev(sig), slack=2.0)
            X = dev(x)
            s, res = H.fire_auto(s, X, dev(sig), params)
            alone.append((X.cpu().numpy(), res))
            systems.append((s, x, sig))
        xm, Lm = inputs.jittered_lattice(4, 5, 1.1, 0.13, 7)
        nm = len(xm)
        sm = inputs.bidisperse(nm, 1.0, 1.2, 7)
        vm = inputs.gaussian_velocities(nm, 4, 1.0, 8)
        smd = H.System(d=4, n=nm, box_l=Lm, cutoff=C6, skin=0.3, sigma_max=1.2, max_neighbors=64)
        smd, _ = H.build_with_width(smd, dev(xm), dev(sm), slack=2.0)
        Xm, Vm = dev(xm), dev(vm)
        H.hdmd_step(smd, Xm, Vm, dev(sm), H.workspace(smd), 50, 0.004)
        B = H.Batch(max_slots=8, max_atoms=20000, max_cells=200000)
        keep = []
        for k, (s, x, sig) in enumerate(systems):
            X, SG, ws = dev(x), dev(sig), H.workspace(s)
            keep.append((X, SG, ws))
            B.hdmd_batch_add_fire(k, s, X, SG, ws, params)
        B.hdmd_batch_add_md(5, smd, dev(xm), dev(vm), dev(sm), H.workspace(smd), 50, 0.004)
        done = {}
        for _ in range(1000):
            B.hdmd_batch_run(25)
            state, _ = B.hdmd_batch_poll()
            for k in list(range(len(systems))) + [5]:
                if k not in done and state[k] == H.HDMD_SLOT_DONE:
                    pos, vel, res = B.hdmd_batch_take(k, want_vel=(k == 5))
                    done[k] = (pos.cpu().numpy(), vel, res)
            if len(done) == len(systems) + 1:
                break
    assert len(done) == len(systems) + 1
    for k in range(len(systems)):
        assert np.array_equal(done[k][0], alone[k][0]), k
        assert done[k][2].iterations == alone[k][1].iterations
        assert done[k][2].energy == alone[k][1].energy
    assert np.array_equal(done[5][0], Xm.cpu().numpy())
    assert np.array_equal(done[5][1].cpu().numpy(), Vm.cpu().numpy())


def test_autotuned_lanes_are_recorded(orc):
    """A system's first build times 1, 2 and 4 lanes per atom for its key
    (d = 5, FP64, expected rows of ~127 atoms); a second system with the same
    key takes the recorded count, and its forces equal, bit for bit, those of
    the same system with that count forced."""
    rl = C6 * 1.2 + 0.3
    L = 5 * rl * 1.01

    def make(n, seed):
        x = inputs.uniform_positions(n, 5, L, seed)
        sig = inputs.bidisperse(n, 1.0, 1.2, seed + 1)
        return H.System(d=5, n=n, box_l=L, cutoff=C6, skin=0.3, sigma_max=1.2,
                        max_neighbors=400, subcells=H.HDMD_SUBCELLS_FULL), x, sig

    s1, x1, g1 = make(80000, 31)
    H.hdmd_build_nlist(s1, dev(x1), dev(g1), H.workspace(s1))
    lanes = H.hdmd_build_config(s1)[4]
    assert lanes in (1, 2, 4)
    s2, x2, g2 = make(78000, 41)
    assert H.hdmd_build_config(s2)[4] == lanes
    F2, E2 = H.hdmd_forces(s2, dev(x2), dev(g2), H.workspace(s2))
    with _lanes(lanes):
        F3, E3 = H.hdmd_forces(s2, dev(x2), dev(g2), H.workspace(s2))
    assert torch.equal(F2, F3) and float(E2) == float(E3)
    rp, cols = orc.nlist_cells(x2, g2, L, C6, 0.3)
    Fo, _, _ = orc.forces(x2, g2, L, H.HDMD_WCA, C6, 1.0, rp, cols)
    assert force_err(F2.cpu().numpy(), Fo) < 1e-12
