"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This module holds no step of the method (no binning, lists, forces or
integrators): only seeded random numbers, box sizing and the workload recipes.
Every generator draws from numpy's PCG64 with an explicit seed.

Workloads (synthetic stand-ins for the paper's liquids; the paper uses no
public dataset):

* ``c1`` d=3, N=1000, 50:50 WCA mixture sigma 1.0/1.4, number density 0.8.
* ``c2`` d=4, N=65536, monodisperse WCA, packing fraction 0.4.
* ``c3`` d=6, N=262144, 50:50 WCA mixture sigma 1.0/1.2, packing fraction 0.42.
* ``c4`` 512 harmonic soft-sphere FIRE requests, d in {3,4,5,6},
  N log-uniform in [256, 8192], 50:50 sigma 1.0/1.4, phi near phi_J.
* ``c5`` d=8, N=131072, monodisperse WCA, packing fraction 0.3 (n_cell = 2).
* ``p6`` the paper's d=6 state point: N=10^5, polydisperse P(6, 6, sigma),
  Morse a=30, phi = 0.1850, T = 0.25, dt = 0.0016.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

WCA_CUT = 2.0 ** (1.0 / 6.0)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def ball_volume(d: int, sigma: float) -> float:
    """Volume of a d-ball of diameter sigma (used only to size boxes)."""
    return math.pi ** (0.5 * d) * sigma ** d / (2.0 ** d * math.gamma(1.0 + 0.5 * d))


def box_for_packing(d: int, sig: np.ndarray, phi: float) -> float:
    """Side of the hypercube whose packing fraction is phi."""
    uniq, counts = np.unique(np.asarray(sig, dtype=np.float64), return_counts=True)
    vol = float(sum(c * ball_volume(d, float(s)) for s, c in zip(uniq, counts)))
    return (vol / phi) ** (1.0 / d)


def box_for_density(d: int, n: int, rho: float) -> float:
    return (n / rho) ** (1.0 / d)


def bidisperse(n: int, s_a: float, s_b: float, seed: int) -> np.ndarray:
    """50:50 mixture: n//2 atoms of s_a and the rest s_b, in seeded order."""
    sig = np.full(n, s_b, dtype=np.float64)
    sig[: n // 2] = s_a
    rng(seed).shuffle(sig)
    return sig


def polydisperse(n: int, d: int, R: float, seed: int) -> np.ndarray:
    """Diameters drawn from the paper's distribution P(d, R, sigma) (Sec. II.A,
    eq. sigmadist): density proportional to sigma^-d on [R^(-1/2d), R^(1/2d)],
    R the ratio of the largest to the smallest particle volume, so that every
    diameter interval of equal width holds the same particle volume.  Drawn by
    inverting the cumulative distribution,
    F(sigma) = (lo^(1-d) - sigma^(1-d)) / (lo^(1-d) - hi^(1-d))."""
    lo, hi = R ** (-0.5 / d), R ** (0.5 / d)
    u = rng(seed).uniform(size=n)
    a, b = lo ** (1 - d), hi ** (1 - d)
    return (a - u * (a - b)) ** (1.0 / (1 - d))


def polydispersity_index(d: int, R: float) -> float:
    """Delta = sqrt(<sigma^2> - <sigma>^2) / <sigma> of P(d, R, sigma), from its
    moments in closed form: <sigma^k> = int sigma^(k-d) / int sigma^(-d) over
    [R^(-1/2d), R^(1/2d)]."""
    lo, hi = R ** (-0.5 / d), R ** (0.5 / d)

    def mom(k: int) -> float:  # integral of sigma^(k-d) over [lo, hi]
        e = k - d + 1
        return math.log(hi / lo) if e == 0 else (hi ** e - lo ** e) / e

    m0 = mom(0)
    m1, m2 = mom(1) / m0, mom(2) / m0
    return math.sqrt(m2 - m1 * m1) / m1


def uniform_positions(n: int, d: int, L: float, seed: int) -> np.ndarray:
    """Uniform positions in [-L/2, L/2)^d, shape (n, d)."""
    x = rng(seed).uniform(-0.5 * L, 0.5 * L, size=(n, d))
    x[x >= 0.5 * L] = -0.5 * L
    return x


def gaussian_velocities(n: int, d: int, T: float, seed: int) -> np.ndarray:
    """Unit-mass Gaussian velocities, centre-of-mass motion removed, rescaled so
    that 2 KE / (d (N-1)) = T exactly."""
    v = rng(seed).normal(0.0, math.sqrt(T), size=(n, d))
    v -= v.mean(axis=0, keepdims=True)
    t_now = float((v * v).sum()) / (d * (n - 1))
    if t_now > 0:
        v *= math.sqrt(T / t_now)
    return v


def jittered_lattice(d: int, m: int, a: float, jitter: float, seed: int,
                     vacancy: float = 0.0) -> tuple[np.ndarray, float]:
    """Hypercubic lattice of m^d sites with spacing a, each site displaced
    uniformly by up to +-jitter per axis; a seeded fraction of sites removed.
    Returns (positions (n,d) in [-L/2,L/2), L = m a)."""
    L = m * a
    idx = np.indices((m,) * d).reshape(d, -1).T.astype(np.float64)
    x = -0.5 * L + (idx + 0.5) * a
    g = rng(seed)
    if jitter > 0:
        x += g.uniform(-jitter, jitter, size=x.shape)
    if vacancy > 0:
        keep = g.uniform(size=x.shape[0]) >= vacancy
        x = x[keep]
    x = np.where(x >= 0.5 * L, x - L, x)
    x = np.where(x < -0.5 * L, x + L, x)
    return np.ascontiguousarray(x), L


@dataclasses.dataclass
class MDConfig:
    name: str
    d: int
    n: int
    sig_a: float
    sig_b: float
    phi: float | None
    rho: float | None
    dt: float
    skin: float
    steps: int
    T: float = 1.0
    cutoff: float = WCA_CUT
    seed: int = 0
    potential: int = 0      # 0 WCA, 2 Morse (a = 30)
    poly_R: float = 0.0     # > 0: diameters from P(d, R, sigma) with R = poly_R

    def diameters(self) -> np.ndarray:
        if self.poly_R > 0:
            return polydisperse(self.n, self.d, self.poly_R, self.seed + 1)
        if self.sig_a == self.sig_b:
            return np.full(self.n, self.sig_a)
        return bidisperse(self.n, self.sig_a, self.sig_b, self.seed + 1)

    def box(self, sig: np.ndarray) -> float:
        if self.rho is not None:
            return box_for_density(self.d, self.n, self.rho)
        return box_for_packing(self.d, sig, self.phi)

    def positions(self, L: float) -> np.ndarray:
        return uniform_positions(self.n, self.d, L, self.seed + 2)

    def velocities(self) -> np.ndarray:
        return gaussian_velocities(self.n, self.d, self.T, self.seed + 3)


C1 = MDConfig("c1_d3_n1000", 3, 1000, 1.0, 1.4, None, 0.8, 0.005, 0.3, 1000, seed=1000)
C2 = MDConfig("c2_d4_n65536", 4, 65536, 1.0, 1.0, 0.4, None, 0.005, 0.3, 10000, seed=2000)
C3 = MDConfig("c3_d6_n262144", 6, 262144, 1.0, 1.2, 0.42, None, 0.002, 0.25, 10000, seed=3000)
C5 = MDConfig("c5_d8_n131072", 8, 131072, 1.0, 1.0, 0.3, None, 0.002, 0.25, 5000, seed=5000)
# C5 geometry at a liquid packing fraction: same d, N, n_cell = 2, WCA, dt and T,
# for the NVE part of the precision stress (at 0.3 the relaxed state keeps
# ~100 overlaps per atom and WCA dynamics at dt = 0.002 diverge)
C5_MD = MDConfig("c5md_d8_n131072", 8, 131072, 1.0, 1.0, 0.05, None, 0.002, 0.25, 5000, seed=5000)
# The paper's own d = 6 state point (Sec. IV, Table tab:phiefftab): N = 10^5,
# diameters from P(6, R = 6, sigma), truncated and shifted Morse with a = 30,
# phi = phi*_6 = 0.1850, k_B T = 0.25, dt = 0.0016; unit masses and one epsilon.
P6 = MDConfig("p6_d6_n100000", 6, 100000, 6.0 ** (-1 / 12), 6.0 ** (1 / 12), 0.1850, None, 0.0016,
              0.25, 10000, T=0.25, cutoff=1.0, seed=6000, potential=2, poly_R=6.0)
CONFIGS = {"c1": C1, "c2": C2, "c3": C3, "c5": C5, "c5md": C5_MD, "p6": P6}


@dataclasses.dataclass
class FireRequest:
    """One jamming minimisation request of the batched/served workload."""
    rid: int
    d: int
    n: int
    phi: float
    L: float
    sig: np.ndarray
    arrival: float
    pos_seed: int

    def positions(self) -> np.ndarray:
        return uniform_positions(self.n, self.d, self.L, self.pos_seed)


def fire_requests(count: int, phij: dict[int, float], rate: float, seed: int = 4000,
                  n_lo: int = 256, n_hi: int = 8192, d_choices=(3, 4, 5, 6),
                  min_box: float = 2.8) -> list[FireRequest]:
    """Seeded request stream: d uniform over d_choices, N log-uniform in
    [n_lo, n_hi], phi uniform in [phi_J - 0.02, phi_J + 0.05], 50:50 diameters
    1.0/1.4, uniform positions; Poisson arrivals at `rate` per second (arrival
    seed `seed + 999`).  N is redrawn until the box side is at least `min_box`
    (twice the largest diameter, so the minimum image stays valid)."""
    arr = rng(seed + 999).exponential(1.0 / rate, size=count).cumsum() if rate > 0 else \
        np.zeros(count)
    out = []
    for k in range(count):
        g = rng(seed + k)
        d = int(g.choice(np.asarray(d_choices)))
        while True:
            n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
            n = max(n, 2)
            phi = float(g.uniform(phij[d] - 0.02, phij[d] + 0.05))
            sig = np.full(n, 1.4)
            sig[: n // 2] = 1.0
            g.shuffle(sig)
            L = box_for_packing(d, sig, phi)
            if L >= min_box:
                break
        out.append(FireRequest(k, d, n, phi, L, sig, float(arr[k]), int(g.integers(1 << 62))))
    return out
