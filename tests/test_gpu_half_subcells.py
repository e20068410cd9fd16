"""Half-size subcells with the 5^d stencil (Sec. II.C: subcells of side at
least r_l,max/2, each linked to the 5^d - 1 around it).  Lists against the
oracle's definition for d = 2..10 with every build variant in both precision
forms, pairs at their list radius +- ulps across subcell and box faces, the
same lists as the grid of side >= r_l,max; forces, a velocity-Verlet run, FIRE
and SWAP against the oracle on the half-size grid; a batch mixing both grids
equal to the lone runs; and the autotuner's recorded choice."""
import os

import numpy as np
import pytest
import torch

from paper_2112_12271_amd import hdmd as H
from paper_2112_12271_amd import inputs
from tests.gpu_util import csr_equal, dev, force_err, gpu_list, partnered

pytestmark = pytest.mark.gpu
C6 = inputs.WCA_CUT
HALF, FULL = H.HDMD_SUBCELLS_HALF, H.HDMD_SUBCELLS_FULL


class _blk:
    """HDMD_BUILD_BLK set for the duration of a block (the forced build variant)."""

    def __init__(self, v):
        self.v = v

    def __enter__(self):
        self.old = os.environ.get("HDMD_BUILD_BLK")
        os.environ["HDMD_BUILD_BLK"] = str(self.v)

    def __exit__(self, *a):
        if self.old is None:
            os.environ.pop("HDMD_BUILD_BLK", None)
        else:
            os.environ["HDMD_BUILD_BLK"] = self.old


# per d: half-size subcells per axis and atoms (d >= 8: 5 per axis, 5^d
# subcells, most of them empty)
SIZES = {2: (9, 900), 3: (8, 1500), 4: (7, 1500), 5: (6, 1200), 6: (6, 1500), 7: (5, 800),
         8: (5, 600), 9: (5, 400), 10: (5, 300)}


@pytest.mark.parametrize("d", range(2, 11))
def test_half_grid_lists_equal_definition(orc, d):
    """Every candidate-lane variant (1, 2, 4 waves per subcell; pair tests on
    the vector units or the matrix cores) and, for d <= 7,
    the home-lane build (64/128/256 lanes) on half-size subcells give the
    definition's list in both precision forms (atoms placed in pairs 0.5 to
    1.1 r_l,max apart, diameters 1 and 1.4)."""
    c, s = C6, 0.3
    rlmax = c * 1.4 + s
    nh, n = SIZES[d]
    L = nh * 0.5 * rlmax * 1.02
    x, sig = partnered(d, n, L, 700 + d, rlmax)
    ref = orc.nlist_brute(x, sig, L, c, s)
    for blk in (1, 2, 4, 1025, 1026, 1028) + ((64, 128, 256) if d <= 7 else ()):
        with _blk(blk):
            for prec in (H.HDMD_FP64, H.HDMD_MIXED):
                sysd = H.System(d=d, n=n, box_l=L, cutoff=c, skin=s, sigma_max=1.4,
                                precision=prec, max_neighbors=16, subcells=HALF)
                assert H.hdmd_build_config(sysd)[1:3] == (2, nh)
                got, _, _ = gpu_list(sysd, x, sig)
                assert csr_equal(got, ref), (d, blk, prec)


def _boundary(d, L, rl, n_pairs, seed):
    """Pairs r_l +- a few ulps apart, one end on a subcell or box face or corner."""
    g = np.random.default_rng(seed)
    h = 0.5 * L
    xs = []
    for p in range(n_pairs):
        a = g.uniform(-h, h, d)
        if p % 3 == 1:
            a[g.integers(d)] = -h
        elif p % 3 == 2:
            a[:] = np.where(g.uniform(size=d) < 0.5, -h, h - 1e-12)
        u = g.normal(size=d)
        u /= np.linalg.norm(u)
        r = rl + g.integers(-4, 5) * np.spacing(rl)
        b = a + r * u
        b = np.where(b >= h, b - L, b)
        b = np.where(b < -h, b + L, b)
        b = np.where(b >= h, -h, b)
        xs += [a, b]
    return np.array(xs)


@pytest.mark.parametrize("d", [2, 3, 4, 6])
@pytest.mark.parametrize("nh", [5, 6, 7])
def test_half_grid_boundary_band(orc, d, nh):
    """Subcells exactly r_l/2 wide (to rounding): pairs two subcells apart at
    r_l +- ulps are the stencil's outer layer."""
    c, s = 1.0, 0.25
    rl = c + s
    L = nh * 0.5 * rl * (1.0 + 4e-9)
    x = _boundary(d, L, rl, 200, seed=41 * d + nh)
    sig = np.ones(len(x))
    ref = orc.nlist_brute(x, sig, L, c, s)
    for prec in (H.HDMD_FP64, H.HDMD_MIXED):
        sysd = H.System(d=d, n=len(x), box_l=L, cutoff=c, skin=s, sigma_max=1.0,
                        precision=prec, max_neighbors=8, subcells=HALF)
        assert H.hdmd_cells_per_axis(sysd) == nh
        got, _, _ = gpu_list(sysd, x, sig)
        assert csr_equal(got, ref), prec


@pytest.mark.parametrize("d,phi,n", [(3, 0.6, 4000), (4, 0.45, 5000), (6, 0.3, 20000)])
def test_half_and_full_grids_one_list_and_forces(orc, d, phi, n):
    """One system on both grids: the same list, and forces within 1e-12 F_rms
    of the oracle's on each (the sums run in each grid's atom order)."""
    sig = inputs.bidisperse(n, 1.0, 1.2, 3 * d)
    L = inputs.box_for_packing(d, sig, phi)
    x = inputs.uniform_positions(n, d, L, 3 * d + 1)
    rp, cols = orc.nlist_cells(x, sig, L, C6, 0.3)
    Fo, _, Eo = orc.forces(x, sig, L, H.HDMD_WCA, C6, 1.0, rp, cols)
    lists = []
    for grid in (FULL, HALF):
        sysd = H.System(d=d, n=n, box_l=L, cutoff=C6, skin=0.3, sigma_max=1.2, subcells=grid)
        got, sysf, ws = gpu_list(sysd, x, sig)
        lists.append(got)
        F, E = H.hdmd_forces(sysf, dev(x), dev(sig), ws)
        assert force_err(F.cpu().numpy(), Fo) < 1e-12, grid
        assert abs(float(E) - Eo) <= 1e-12 * abs(Eo)
    assert csr_equal(lists[0], lists[1])
    assert csr_equal(lists[0], (rp, cols))


@pytest.mark.parametrize("d,m,a", [(3, 10, 1.12), (4, 7, 1.1), (6, 4, 1.05)])
@pytest.mark.parametrize("prec", [H.HDMD_FP64, H.HDMD_MIXED])
def test_half_grid_md_matches_oracle(orc, d, m, a, prec):
    """100 velocity-Verlet steps on half-size subcells: positions within 1e-9
    (FP64; 1e-4 in the precision form) of the oracle's, with its rebuilds."""
    x, L = inputs.jittered_lattice(d, m, a, 0.12 * a, 9 * d)
    n = len(x)
    sig = inputs.bidisperse(n, 1.0, 1.2, 9 * d)
    v = inputs.gaussian_velocities(n, d, 1.0, 9 * d + 1)
    sysd = H.System(d=d, n=n, box_l=L, cutoff=C6, skin=0.3, sigma_max=1.2, precision=prec,
                    subcells=HALF)
    assert H.hdmd_build_config(sysd)[1] == 2
    sysd, _ = H.build_with_width(sysd, dev(x), dev(sig), slack=2.0)
    ws = H.workspace(sysd)
    X, V = dev(x), dev(v)
    st, _ = H.hdmd_step(sysd, X, V, dev(sig), ws, 100, 0.003)
    xo, vo, _, bo = orc.vv(x, v, sig, L, H.HDMD_WCA, C6, 0.3, 1.0, 100, 0.003)
    dx = X.cpu().numpy() - xo
    dx -= L * np.round(dx / L)
    tx = 1e-9 if prec == H.HDMD_FP64 else 1e-4
    assert np.abs(dx).max() < tx
    assert np.abs(V.cpu().numpy() - vo).max() < 10 * tx
    if prec == H.HDMD_FP64:
        assert st.builds + 1 == bo


def test_half_grid_fire_matches_oracle(orc):
    """40 FIRE iterations (harmonic, d = 4) on half-size subcells: positions
    within 1e-9 of the oracle's FIRE 2.0."""
    d, n = 4, 1500
    sig = inputs.bidisperse(n, 1.0, 1.4, 5)
    L = inputs.box_for_packing(d, sig, 0.5)
    x = inputs.uniform_positions(n, d, L, 6)
    sysd = H.System(d=d, n=n, box_l=L, potential=H.HDMD_HARMONIC, cutoff=1.0, skin=0.25,
                    sigma_max=1.4, max_neighbors=64, subcells=HALF)
    sysd, _ = H.build_with_width(sysd, dev(x), dev(sig), slack=2.0)
    X = dev(x)
    sysf, res = H.fire_auto(sysd, X, dev(sig), H.hdmd_fire_defaults(0.05, 1e-12, 40))
    assert res.iterations == 40
    xo, ro = orc.fire(x, sig, L, H.HDMD_HARMONIC, 1.0, 0.25, 1.0,
                      orc.fire_params(dt0=0.05, ftol=1e-12, maxiter=40))
    dx = X.cpu().numpy() - xo
    dx -= L * np.round(dx / L)
    assert np.abs(dx).max() < 1e-9


def test_half_grid_swap_matches_oracle(orc):
    """SWAP attempts search the 5^d linked subcells of each atom on the half
    grid: decisions and final diameters equal the oracle's."""
    d = 3
    x, L = inputs.jittered_lattice(d, 10, 1.4, 0.2, 13)
    n = len(x)
    sig = inputs.bidisperse(n, 1.0, 1.4, 13)
    g = np.random.default_rng(14)
    natt = 500
    pairs = g.integers(0, n, size=(natt, 2)).astype(np.int32)
    u = g.uniform(size=natt)
    T = 0.5
    sig_o, acc_o, de_o, na_o = orc.swap(x, sig, L, H.HDMD_WCA, C6, 1.0, pairs, u, T)
    thr = np.where(de_o <= 0, 2.0, np.exp(-np.maximum(de_o, 0) / T))
    assert np.all((de_o <= 0) | (np.abs(u - thr) > 1e-9))
    assert 0 < na_o < natt
    sysd = H.System(d=d, n=n, box_l=L, cutoff=C6, skin=0.25, sigma_max=1.4, max_neighbors=64,
                    subcells=HALF)
    assert H.hdmd_build_config(sysd)[1] == 2
    sysd, ws = H.build_with_width(sysd, dev(x), dev(sig))
    D = dev(sig)
    acc, na = H.hdmd_swap(sysd, dev(x), D, ws, torch.as_tensor(pairs, device="cuda"), dev(u), T)
    assert na == na_o
    assert np.array_equal(acc.cpu().numpy(), acc_o)
    assert np.array_equal(D.cpu().numpy(), sig_o)


def test_batch_mixing_grids_equals_alone(orc):
    """FIRE systems on half-size subcells (d = 3, 4 in the all-class build
    launch, d = 9 in a launch of its own) batched with systems on the grid of
    side >= r_l,max: every slot gives the bits of its lone run."""
    cases = [(3, 1200, 0.55, 1, HALF), (3, 900, 0.6, 2, FULL), (4, 1000, 0.45, 3, HALF),
             (4, 800, 0.5, 4, FULL), (9, 600, 1e-4, 5, HALF)]
    params = H.hdmd_fire_defaults(0.05, 1e-10, 400)
    systems, alone = [], []
    for d, n, phi, seed, grid in cases:
        sig = inputs.bidisperse(n, 1.0, 1.4, seed)
        L = inputs.box_for_packing(d, sig, phi)
        x = inputs.uniform_positions(n, d, L, seed + 1)
        sysd = H.System(d=d, n=n, box_l=L, potential=H.HDMD_HARMONIC, cutoff=1.0, skin=0.25,
                        sigma_max=1.4, max_neighbors=64, subcells=grid)
        assert H.hdmd_build_config(sysd)[1] == (2 if grid == HALF else 1)
        sysd, _ = H.build_with_width(sysd, dev(x), dev(sig), slack=2.0)
        X = dev(x)
        sysf, res = H.fire_auto(sysd, X, dev(sig), params)
        alone.append((X.cpu().numpy(), res))
        systems.append((sysf, x, sig))
    B = H.Batch(max_slots=8, max_atoms=20000, max_cells=4000000)
    keep = []
    for k, (s, x, sig) in enumerate(systems):
        X, SG, ws = dev(x), dev(sig), H.workspace(s)
        keep.append((X, SG, ws))
        B.hdmd_batch_add_fire(k, s, X, SG, ws, params)
    done = {}
    for _ in range(1000):
        B.hdmd_batch_run(25)
        state, _ = B.hdmd_batch_poll()
        for k in range(len(systems)):
            if k not in done and state[k] == H.HDMD_SLOT_DONE:
                pos, _, res = B.hdmd_batch_take(k)
                done[k] = (pos.cpu().numpy(), res)
        if len(done) == len(systems):
            break
    assert len(done) == len(systems)
    for k in range(len(systems)):
        assert np.array_equal(done[k][0], alone[k][0]), k
        assert done[k][1].iterations == alone[k][1].iterations
        assert done[k][1].energy == alone[k][1].energy


def test_autotuner_records_one_grid_per_key(orc):
    """An autotuned system with a key no other test meets (d = 7, two subcells
    of side >= r_l,max per axis, about 150 atoms in each; five half-size ones
    per axis) is untuned before its first build and tuned after it; a second
    system with the same key takes the recorded grid and variant without
    timing, and its forces are those of the same system requested on that
    grid explicitly, bit for bit."""
    d = 7
    rl = C6 * 1.2 + 0.3
    L = 2.5 * rl * 1.01

    def make(n, seed, grid=H.HDMD_SUBCELLS_AUTO):
        x = inputs.uniform_positions(n, d, L, seed)
        sig = inputs.bidisperse(n, 1.0, 1.2, seed + 1)
        return H.System(d=d, n=n, box_l=L, cutoff=C6, skin=0.3, sigma_max=1.2,
                        max_neighbors=400, subcells=grid), x, sig

    s1, x1, sg1 = make(20000, 61)
    tuned, reach0, nc0, _, _ = H.hdmd_build_config(s1)
    assert not tuned and reach0 == 1 and nc0 == 2
    H.hdmd_build_nlist(s1, dev(x1), dev(sg1), H.workspace(s1))
    tuned, reach, nc, var, lanes = H.hdmd_build_config(s1)
    assert tuned and reach in (1, 2)
    assert nc == (2 if reach == 1 else 5)
    s2, x2, sg2 = make(19600, 71)            # the same key: d, wrapped, occupancy bucket
    assert H.hdmd_build_config(s2) == (True, reach, nc, var, lanes)
    F2, E2 = H.hdmd_forces(s2, dev(x2), dev(sg2), H.workspace(s2))
    s3 = make(19600, 71, HALF if reach == 2 else FULL)[0]
    F3, E3 = H.hdmd_forces(s3, dev(x2), dev(sg2), H.workspace(s3))
    assert torch.equal(F2, F3) and float(E2) == float(E3)
    rp, cols = orc.nlist_cells(x2, sg2, L, C6, 0.3)
    Fo, _, _ = orc.forces(x2, sg2, L, H.HDMD_WCA, C6, 1.0, rp, cols)
    assert force_err(F2.cpu().numpy(), Fo) < 1e-12
