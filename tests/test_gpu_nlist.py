"""GPU Verlet lists against the oracle's definition: bit-exact sets (FP64
decisions in both precision forms)."""
import math

import numpy as np
import pytest

from paper_2112_12271_amd import hdmd as H
from paper_2112_12271_amd import inputs
from tests.gpu_util import csr_equal, dev, gpu_list, partnered

pytestmark = pytest.mark.gpu
C6 = inputs.WCA_CUT


@pytest.mark.parametrize("d", range(2, 11))
@pytest.mark.parametrize("nc", [1, 2, 3, 4])
def test_list_equals_definition_small(orc, d, nc):
    c, s = C6, 0.3
    rlmax = c * 1.4 + s
    L = nc * rlmax * 1.05 if nc > 1 else max(2.0 * c * 1.4, 1.2 * rlmax)
    n = int(min(1200, max(64, 3 * nc ** min(d, 4))))
    x, sig = partnered(d, n, L, 1000 * d + nc, rlmax)
    ref = orc.nlist_brute(x, sig, L, c, s)
    for prec in (H.HDMD_FP64, H.HDMD_MIXED):
        sysd = H.System(d=d, n=n, box_l=L, cutoff=c, skin=s, sigma_max=1.4, precision=prec,
                        max_neighbors=8)
        got, sysf, _ = gpu_list(sysd, x, sig)
        assert H.hdmd_cells_per_axis(sysf) <= max(nc, 1) or nc >= 3
        assert csr_equal(got, ref), (d, nc, prec)


def _boundary(d, L, rl, n_pairs, seed):
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


@pytest.mark.parametrize("d", [2, 3, 4, 6, 8])
@pytest.mark.parametrize("nc", [2, 3, 5])
def test_boundary_band_bit_exact(orc, d, nc):
    """Pairs at r_l +- a few ulps across subcell and periodic faces and corners."""
    c, s = 1.0, 0.25
    rl = c + s
    L = nc * rl * (1.0 + 4e-9) if nc > 2 else 2.02 * rl
    x = _boundary(d, L, rl, 200, seed=31 * d + nc)
    sig = np.ones(len(x))
    ref = orc.nlist_brute(x, sig, L, c, s)
    sysd = H.System(d=d, n=len(x), box_l=L, cutoff=c, skin=s, sigma_max=1.0, max_neighbors=8)
    got, _, _ = gpu_list(sysd, x, sig)
    assert csr_equal(got, ref)


@pytest.mark.parametrize("d,nc", [(3, 3), (4, 3), (6, 3), (3, 5), (5, 4)])
def test_pair_radius_band_bidisperse(orc, d, nc):
    """Pairs at their own list radius c sigma_ij + s, a few ulps either side,
    with diameters 1 and 2 mixed (n_cell >= 3): the prefilter's per-atom
    shares of the pair threshold keep every pair the definition lists."""
    c, s = 1.0, 0.25
    sig_v = np.array([1.0, 2.0])
    rlmax = c * 2.0 + s
    L = nc * rlmax * (1.0 + 4e-9)
    g = np.random.default_rng(53 * d + nc)
    h = 0.5 * L
    xs, sig = [], []
    for p in range(300):
        sa, sb = sig_v[g.integers(2)], sig_v[g.integers(2)]
        a = g.uniform(-h, h, d)
        u = g.normal(size=d)
        u /= np.linalg.norm(u)
        rl = c * 0.5 * (sa + sb) + s
        b = a + (rl + g.integers(-4, 5) * np.spacing(rl)) * u
        b = np.where(b >= h, b - L, b)
        b = np.where(b < -h, b + L, b)
        b = np.where(b >= h, -h, b)
        xs += [a, b]
        sig += [sa, sb]
    x, sig = np.array(xs), np.array(sig)
    ref = orc.nlist_brute(x, sig, L, c, s)
    assert len(ref[1]) > 300
    for prec in (H.HDMD_FP64, H.HDMD_MIXED):
        sysd = H.System(d=d, n=len(x), box_l=L, cutoff=c, skin=s, sigma_max=2.0,
                        precision=prec, max_neighbors=8)
        assert H.hdmd_cells_per_axis(sysd) == nc
        got, _, _ = gpu_list(sysd, x, sig)
        assert csr_equal(got, ref), prec


@pytest.mark.parametrize("d,m,kmax", [(3, 6, 4), (4, 5, 4), (6, 4, 2), (8, 3, 2), (10, 3, 1)])
def test_lattice_shells(d, m, kmax):
    """Closed-form coordination shells of a lattice filling the periodic box."""
    x, L = inputs.jittered_lattice(d, m, 1.0, 0.0, 0)
    c = math.comb
    shells = {1: 2 * d, 2: 4 * c(d, 2), 3: 8 * c(d, 3), 4: 2 * d + 16 * c(d, 4)}
    expect = sum(shells[k] for k in range(1, kmax + 1))
    rl = 0.5 * (math.sqrt(kmax) + math.sqrt(kmax + 1))
    sysd = H.System(d=d, n=len(x), box_l=L, cutoff=1.0, skin=rl - 1.0, sigma_max=1.0,
                    max_neighbors=expect + 4)
    (rp, cols), _, _ = gpu_list(sysd, x, np.ones(len(x)))
    assert np.all(np.diff(rp) == expect)


def test_c1_shape(orc):
    """C1-shaped input: d=3, N=1000, 50:50 sigma 1.0/1.4 at number density 0.8."""
    cfg = inputs.C1
    sig = cfg.diameters()
    L = cfg.box(sig)
    x = cfg.positions(L)
    ref = orc.nlist_cells(x, sig, L, C6, cfg.skin)
    sysd = H.System(d=3, n=cfg.n, box_l=L, cutoff=C6, skin=cfg.skin, sigma_max=1.4)
    got, _, _ = gpu_list(sysd, x, sig)
    assert csr_equal(got, ref)


def test_d4_4096(orc):
    d, n = 4, 4096
    sig = np.ones(n)
    L = inputs.box_for_packing(d, sig, 0.4)
    x = inputs.uniform_positions(n, d, L, 4)
    ref = orc.nlist_cells(x, sig, L, C6, 0.3)
    got, _, _ = gpu_list(H.System(d=d, n=n, box_l=L, cutoff=C6, skin=0.3, sigma_max=1.0), x, sig)
    assert csr_equal(got, ref)


def test_one_big_subcell_global_sort(orc):
    """n_cell = 1 with 6000 atoms: the subcell sort and the row export take their
    global-memory paths (more than 4096 entries)."""
    d, n, L = 2, 6000, 2.6
    x = inputs.uniform_positions(n, d, L, 8)
    sig = np.full(n, 1.0)
    ref = orc.nlist_brute(x, sig, L, 1.0, 0.4)
    sysd = H.System(d=d, n=n, box_l=L, cutoff=1.0, skin=0.4, sigma_max=1.0,
                    potential=H.HDMD_HARMONIC, max_neighbors=6000)
    assert H.hdmd_cells_per_axis(sysd) == 1
    got, _, _ = gpu_list(sysd, x, sig)
    assert csr_equal(got, ref)


@pytest.mark.parametrize("name", ["c3", "c5"])
def test_full_size_sampled_rows(orc, name):
    """Full-size C3 (d=6, N=262144) and C5 (d=8, N=131072, n_cell = 2) inputs:
    sampled rows against the definition, plus list symmetry as a whole."""
    cfg = inputs.CONFIGS[name]
    sig = cfg.diameters()
    L = cfg.box(sig)
    x = cfg.positions(L)
    width = 320 if name == "c3" else 1600
    sysd = H.System(d=cfg.d, n=cfg.n, box_l=L, cutoff=C6, skin=cfg.skin,
                    sigma_max=float(sig.max()), max_neighbors=width)
    (rp, cols), sysf, _ = gpu_list(sysd, x, sig)
    g = np.random.default_rng(1)
    for i in g.choice(cfg.n, 24, replace=False):
        ref = orc.nlist_row(x, sig, L, C6, cfg.skin, int(i))
        assert np.array_equal(cols[rp[i]:rp[i + 1]], ref), i
    rows = np.repeat(np.arange(cfg.n), np.diff(rp))
    fwd = rows.astype(np.int64) * cfg.n + cols
    bwd = cols.astype(np.int64) * cfg.n + rows
    assert np.array_equal(np.sort(fwd), np.sort(bwd))


@pytest.mark.parametrize("d,nc,per_cell", [(3, 3, 150), (4, 3, 140), (6, 3, 10), (8, 3, 1),
                                           (3, 2, 200), (6, 2, 40), (8, 2, 4), (4, 1, 300)])
def test_every_build_variant_equals_definition(orc, d, nc, per_cell):
    """Each list-build variant (candidate-lane with 1, 2 or 4 waves per subcell,
    with the pair tests on the vector units or the matrix cores, 8 or 16 waves
    for the crowded subcells of n_cell <= 2, home-lane with 64/128/256 lanes),
    forced in turn, gives the definition's list; crowded
    subcells (more than 64 and 128 atoms) take several home passes; n_cell =
    2 and 1 take the wrapped-coordinate prefilter."""
    import os
    c, s = C6, 0.3
    rlmax = c * 1.4 + s
    L = nc * rlmax * 1.02 if nc > 1 else max(2.0 * c * 1.4 * 1.001, 1.02 * rlmax)
    n = per_cell * nc ** d
    x, sig = partnered(d, n, L, 77 * d + nc, rlmax)
    ref = orc.nlist_brute(x, sig, L, c, s)
    old = os.environ.get("HDMD_BUILD_BLK")
    try:
        for blk in (1, 2, 4, 1025, 1026, 1028, 8, 16, 64, 128, 256):
            os.environ["HDMD_BUILD_BLK"] = str(blk)
            for prec in (H.HDMD_FP64, H.HDMD_MIXED):
                sysd = H.System(d=d, n=n, box_l=L, cutoff=c, skin=s, sigma_max=1.4,
                                precision=prec, max_neighbors=16)
                assert H.hdmd_cells_per_axis(sysd) == nc
                got, _, _ = gpu_list(sysd, x, sig)
                assert csr_equal(got, ref), (d, blk, prec)
    finally:
        if old is None:
            os.environ.pop("HDMD_BUILD_BLK", None)
        else:
            os.environ["HDMD_BUILD_BLK"] = old


# (d, subcells per axis, atoms): dense grids (rows of several chunks, up to
# ~200 atoms per subcell: two home sets, two blocks of 32 kept atoms; at d = 5
# with ~150 atoms per subcell a pass can hold more survivors, ~700, than one
# round of listed codes) down to sparse ones (four rows per round)
MF_CASES = [(2, 5, 5000), (3, 4, 9000), (4, 3, 8000), (5, 3, 9000), (5, 3, 36000),
            (6, 3, 12000), (7, 3, 9000), (8, 3, 8000), (9, 3, 10000), (10, 3, 16000)]


@pytest.mark.parametrize("d,nc,n", MF_CASES)
def test_matrix_core_build_equals_definition(orc, d, nc, n):
    """The candidate-lane build with its pair tests on the matrix cores (one
    f16 32x32x16 product per 32 candidates and 32 kept home atoms, exact in
    f32), with 1, 2 and 4 waves per subcell, gives the definition's list in
    both precision forms for d = 2..10."""
    import os
    c, s = C6, 0.3
    rlmax = c * 1.4 + s
    L = nc * rlmax * 1.02
    x, sig = partnered(d, n, L, 91 * d + nc, rlmax)
    ref = orc.nlist_brute(x, sig, L, c, s)
    old = os.environ.get("HDMD_BUILD_BLK")
    try:
        for blk in (1025, 1026, 1028):
            os.environ["HDMD_BUILD_BLK"] = str(blk)
            for prec in (H.HDMD_FP64, H.HDMD_MIXED):
                sysd = H.System(d=d, n=n, box_l=L, cutoff=c, skin=s, sigma_max=1.4,
                                precision=prec, max_neighbors=32,
                                subcells=H.HDMD_SUBCELLS_FULL)
                assert H.hdmd_cells_per_axis(sysd) == nc
                got, _, _ = gpu_list(sysd, x, sig)
                assert csr_equal(got, ref), (d, blk, prec)
    finally:
        if old is None:
            os.environ.pop("HDMD_BUILD_BLK", None)
        else:
            os.environ["HDMD_BUILD_BLK"] = old


@pytest.mark.parametrize("d,n,L", [(3, 1600, 13.0), (5, 1500, 7.0)])
@pytest.mark.parametrize("prec", [H.HDMD_FP64, H.HDMD_MIXED])
def test_sparse_system_with_one_crowded_subcell(orc, d, n, L, prec):
    """A sparse system (few atoms per subcell on average, so the candidate-lane
    build takes four rows per round) with 90 atoms packed into one subcell:
    the rounds whose rows reach that subcell exceed one chunk and fall back
    to the row-by-row walk; the lists still match brute force."""
    g = np.random.default_rng(50 + d)
    x = inputs.uniform_positions(n, d, L, 40 + d)
    rl = 1.4 + 0.3
    lsc = L / orc.ncell(L, rl)
    x[:90] = -L / 2 + g.uniform(0.05, 0.95, size=(90, d)) * lsc
    sig = inputs.bidisperse(n, 1.0, 1.4, 60 + d)
    ref = orc.nlist_brute(x, sig, L, 1.0, 0.3)
    sysd = H.System(d=d, n=n, box_l=L, potential=H.HDMD_HARMONIC, cutoff=1.0, skin=0.3,
                    sigma_max=1.4, precision=prec, max_neighbors=128)
    got, _, _ = gpu_list(sysd, x, sig)
    assert csr_equal(got, ref)


def test_c2_full_size_list_and_forces(orc):
    """The d = 4 workload at its full size (N = 65536, phi = 0.4, n_cell = 10),
    from its seeded uniform start: the whole list equals the oracle's subcell
    path in both precision forms (lists are FP64-exact in both), and the FP64
    forces over it (the workload's precision) agree with the oracle's within
    1e-12 F_rms.  (The precision form's force errors are stated on relaxed and
    lattice states: at the uniform start's near-coincident pairs an FP32
    force store alone exceeds 1e-5 of F_rms.)"""
    from tests.gpu_util import force_err
    cfg = inputs.C2
    sig = cfg.diameters()
    L = cfg.box(sig)
    x = cfg.positions(L)
    ref = orc.nlist_cells(x, sig, L, C6, cfg.skin)
    Fo, _, Eo = orc.forces(x, sig, L, 0, C6, 1.0, *ref)
    for prec in (H.HDMD_FP64, H.HDMD_MIXED):
        sysd = H.System(d=4, n=cfg.n, box_l=L, cutoff=C6, skin=cfg.skin,
                        sigma_max=float(sig.max()), precision=prec, max_neighbors=64)
        assert H.hdmd_cells_per_axis(sysd) == 10
        got, sysf, ws = gpu_list(sysd, x, sig)
        assert csr_equal(got, ref), prec
        if prec == H.HDMD_FP64:
            F, E = H.hdmd_forces(sysf, dev(x), dev(sig), ws)
            assert force_err(F.cpu().numpy(), Fo) < 1e-12
            assert abs(float(E) - Eo) <= 1e-12 * abs(Eo)
