"""Pins of the oracle's geometry against the paper and closed forms (CPU only)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("d,expected", [
    (1, 1.0),                 # a segment of length sigma
    (2, math.pi / 4.0),       # disc of diameter 1
    (3, math.pi / 6.0),       # ball of diameter 1
    (4, math.pi ** 2 / 32.0),
])
def test_ball_volume_closed_forms(orc, d, expected):
    """eq. (vofsigma) against textbook values of unit-diameter balls."""
    assert orc.sphere_volume(d, 1.0) == pytest.approx(expected, rel=1e-14)


@pytest.mark.parametrize("d", range(3, 11))
def test_ball_volume_recursion(orc, d):
    """V_d(r) = 2 pi r^2 / d * V_{d-2}(r), with r = sigma/2."""
    s = 1.3
    r = 0.5 * s
    assert orc.sphere_volume(d, s) == pytest.approx(
        2 * math.pi * r * r / d * orc.sphere_volume(d - 2, s), rel=1e-13)


def _sigma_pdf(d, R):
    """eq. (sigmadist): P(sigma) = (d-1) sigma^-d / (R^((d-1)/2d) - R^(-(d-1)/2d))."""
    lo, hi = R ** (-1.0 / (2 * d)), R ** (1.0 / (2 * d))
    norm = R ** ((d - 1) / (2 * d)) - R ** (-(d - 1) / (2 * d))
    return (lambda s: (d - 1) * s ** (-d) / norm), lo, hi


def test_sigma_pdf_normalised():
    for d in range(3, 7):
        p, lo, hi = _sigma_pdf(d, float(d))
        assert integrate.quad(p, lo, hi)[0] == pytest.approx(1.0, rel=1e-12)


def test_paper_ncell_example(orc):
    """Sec. III.B: n_cell = 4 for N = 10^5, d = 6 at phi*_6 with R = d, s = 0.25."""
    g = json.load(open(os.path.join(GOLDEN, "paper_ncell.json")))
    d, N, R, phi, s, cut = g["d"], g["N"], g["R"], g["phi"], g["skin"], g["cut"]
    p, lo, hi = _sigma_pdf(d, R)
    vmean = integrate.quad(lambda t: p(t) * orc.sphere_volume(d, t), lo, hi)[0]
    L = (N * vmean / phi) ** (1.0 / d)
    rlmax = cut * hi + s                      # largest diameter R^(1/2d) plus skin
    assert orc.ncell(L, rlmax) == g["ncell"]


@pytest.mark.parametrize("L,rl", [(10.0, 2.0), (10.0, 2.0 + 1e-15), (6.818, 1.597), (3.02, 1.3725),
                                  (1.0, 2.0), (8.0, 0.5), (5.0 * 1.1, 1.1)])
def test_ncell_guard(orc, L, rl):
    """Subcells are never narrower than the list radius; count is maximal."""
    n = orc.ncell(L, rl)
    assert n >= 1
    if n > 1:
        assert L / n >= rl
    # one more subcell would be too narrow (or only rounding-close)
    assert L / (n + 1) < rl * (1 + 1e-9)


def test_wrap_properties(orc):
    L = 6.818
    g = np.random.default_rng(5)
    xs = np.concatenate([g.uniform(-1.5 * L, 1.5 * L, 2000),
                         [0.5 * L, -0.5 * L, -0.5 * L - 1e-17, 0.5 * L - 1e-16, 1.5 * L - 1e-13]])
    w = orc.wrap(xs, L)
    assert np.all(w >= -0.5 * L) and np.all(w < 0.5 * L)
    # same point modulo L (up to the one rounding of the shift)
    k = np.round((xs - w) / L)
    assert np.all(np.abs(xs - w - k * L) <= 4 * np.spacing(L))
    assert np.all(orc.wrap(w, L) == w)      # idempotent
