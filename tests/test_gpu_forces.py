"""GPU forces and energies against the oracle: 1e-12 (FP64) and 1e-5 (mixed)
of F_rms, the bar the hot path is held to."""
import numpy as np
import pytest

from paper_2112_12271_amd import hdmd as H
from paper_2112_12271_amd import inputs
from tests.gpu_util import dev, force_err, partnered

pytestmark = pytest.mark.gpu
C6 = inputs.WCA_CUT
TOL = {H.HDMD_FP64: 1e-12, H.HDMD_MIXED: 1e-5}


def _liquid(d, m, a, jitter, seed, vacancy=0.0):
    x, L = inputs.jittered_lattice(d, m, a, jitter, seed, vacancy)
    sig = inputs.bidisperse(len(x), 1.0, 1.2, seed)
    return x, sig, L


def _gpu_forces(sysd, x, sig):
    sysf, ws = H.build_with_width(sysd, dev(x), dev(sig))
    F, E = H.hdmd_forces(sysf, dev(x), dev(sig), ws)
    return F.cpu().numpy(), float(E.cpu())


# FP64 is checked on heavily overlapped lattices (spacing 1.0 for diameters up
# to 1.2, forces spanning four decades); the mixed form on liquid-like states
# (spacing 1.2, no pair closer than ~0.95 sigma), where FP32 pair forces of the
# r^-14 WCA law are good to ~1e-6 relative.
CASES = {H.HDMD_FP64: (1.0, 0.3), H.HDMD_MIXED: (1.2, 0.12)}


@pytest.mark.parametrize("prec", [H.HDMD_FP64, H.HDMD_MIXED])
@pytest.mark.parametrize("pot,c", [(H.HDMD_WCA, C6), (H.HDMD_HARMONIC, 1.0),
                                   (H.HDMD_MORSE, 1.0)])
@pytest.mark.parametrize("d,m,vac", [(2, 20, 0.0), (3, 9, 0.0), (4, 6, 0.0), (6, 4, 0.0),
                                     (8, 3, 0.3), (10, 3, 0.92)])
def test_forces_match_oracle(orc, prec, pot, c, d, m, vac):
    a, jit = CASES[prec]
    if pot == H.HDMD_HARMONIC:
        a = 1.0
    elif pot == H.HDMD_MORSE:   # a = 30: overlaps of up to ~0.3 sigma (U up to ~10^7 eps)
        a, jit = (1.05, 0.12) if prec == H.HDMD_FP64 else (1.12, 0.05)
    x, sig, L = _liquid(d, m, a, jit, 10 * d + pot, vac)
    rp, cols = orc.nlist_cells(x, sig, L, c, 0.3)
    Fo, _, Eo = orc.forces(x, sig, L, pot, c, 1.0, rp, cols)
    sysd = H.System(d=d, n=len(x), box_l=L, potential=pot, cutoff=c, skin=0.3, sigma_max=1.2,
                    precision=prec)
    Fg, Eg = _gpu_forces(sysd, x, sig)
    assert force_err(Fg, Fo) < TOL[prec]
    assert abs(Eg - Eo) <= TOL[prec] * abs(Eo)
    # Newton's third law on the GPU result
    assert np.abs(Fg.sum(axis=0)).max() <= 10 * TOL[prec] * np.abs(Fg).sum() / len(Fg) * np.sqrt(len(Fg))


def test_two_particle_closed_form():
    """WCA contact: U = eps, |F| = 24 eps / sigma, across the periodic face."""
    d, L = 3, 5.0
    x = np.array([[-2.4, 0.1, 0.0], [2.4, 0.1, 0.0]])   # minimum-image distance 0.2
    sig = np.array([0.2, 0.2])
    sysd = H.System(d=d, n=2, box_l=L, cutoff=C6, skin=0.1, sigma_max=0.2)
    Fg, Eg = _gpu_forces(sysd, x, sig)
    assert Eg == pytest.approx(1.0, rel=1e-12)
    assert np.linalg.norm(Fg[0]) == pytest.approx(24.0 / 0.2, rel=1e-11)
    assert Fg[0, 0] > 0   # the partner of atom 0 sits at -0.2 through the periodic face


def test_translation_and_permutation(orc):
    x, sig, L = _liquid(5, 4, 1.05, 0.3, 5)
    sysd = H.System(d=5, n=len(x), box_l=L, cutoff=C6, skin=0.3, sigma_max=1.2)
    F0, E0 = _gpu_forces(sysd, x, sig)
    y = orc.wrap(x + np.random.default_rng(0).uniform(-L, L, x.shape[1]), L)
    F1, E1 = _gpu_forces(sysd, y, sig)
    assert force_err(F1, F0) < 1e-10
    perm = np.random.default_rng(2).permutation(len(x))
    F2, E2 = _gpu_forces(sysd, x[perm], sig[perm])
    assert force_err(F2, F0[perm]) < 1e-13
    assert E1 == pytest.approx(E0, rel=1e-12) and E2 == pytest.approx(E0, rel=1e-13)


@pytest.mark.parametrize("name", ["c3", "c5"])
@pytest.mark.parametrize("prec", [H.HDMD_FP64, H.HDMD_MIXED])
def test_full_size_sampled_forces(orc, name, prec):
    """Full-size C3/C5 inputs (relaxed from a jittered lattice of the config's
    density so that no pair is pathologically close): sampled atoms against the
    definition (every other atom)."""
    cfg = inputs.CONFIGS[name]
    sig = cfg.diameters()
    L = cfg.box(sig)
    m = int(round(cfg.n ** (1.0 / cfg.d)))
    x, _ = inputs.jittered_lattice(cfg.d, m, L / m, 0.15 * L / m, 3)
    x = x[: cfg.n]
    sig = sig[: len(x)]
    sysd = H.System(d=cfg.d, n=len(x), box_l=L, cutoff=C6, skin=cfg.skin,
                    sigma_max=float(sig.max()), precision=prec, max_neighbors=1024)
    Fg, Eg = _gpu_forces(sysd, x, sig)
    frms = np.sqrt((Fg * Fg).sum() / len(Fg))
    g = np.random.default_rng(4)
    for i in g.choice(len(x), 12, replace=False):
        Fi, _ = orc.force_one(x, sig, L, 0, C6, 1.0, int(i))
        assert np.linalg.norm(Fg[i] - Fi) <= TOL[prec] * frms
