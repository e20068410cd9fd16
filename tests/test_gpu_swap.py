"""SWAP Monte Carlo on the GPU (Sec. II.D) against the oracle: every
attempt's decision and the final diameters, in the order the attempts run."""
import numpy as np
import pytest
import torch

from paper_2112_12271_amd import hdmd as H
from paper_2112_12271_amd import inputs
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu
C6 = inputs.WCA_CUT


def _case(d, m, a, seed, s_big):
    x, L = inputs.jittered_lattice(d, m, a, 0.15 * a, seed)
    sig = inputs.bidisperse(len(x), 1.0, s_big, seed)
    return x, sig, L


@pytest.mark.parametrize("d,m,a,pot,c,s_big,prec", [
    (3, 8, 1.4, H.HDMD_WCA, C6, 1.4, H.HDMD_FP64),         # n_cell >= 3
    (4, 5, 1.3, H.HDMD_HARMONIC, 1.0, 1.4, H.HDMD_FP64),   # n_cell = 3
    (6, 4, 1.35, H.HDMD_WCA, C6, 1.4, H.HDMD_MIXED),      # n_cell = 2: every subcell
    (3, 8, 1.45, H.HDMD_MORSE, 1.0, 1.1, H.HDMD_FP64),
])
def test_swap_matches_oracle(orc, d, m, a, pot, c, s_big, prec):
    x, sig, L = _case(d, m, a, 10 + d, s_big)
    n = len(x)
    g = np.random.default_rng(20 + d)
    natt = 600
    pairs = g.integers(0, n, size=(natt, 2)).astype(np.int32)
    pairs[::97, 1] = pairs[::97, 0]                     # a few self-exchanges
    u = g.uniform(size=natt)
    T = 0.5
    sig_o, acc_o, de_o, na_o = orc.swap(x, sig, L, pot, c, 1.0, pairs, u, T)
    # no decision of the oracle sits within rounding of the Metropolis threshold
    thr = np.where(de_o <= 0, 2.0, np.exp(-np.maximum(de_o, 0) / T))
    assert np.all((de_o <= 0) | (np.abs(u - thr) > 1e-9))
    assert 0 < na_o < natt
    sysd = H.System(d=d, n=n, box_l=L, potential=pot, cutoff=c, skin=0.25, sigma_max=s_big,
                    precision=prec, max_neighbors=64)
    sysd, ws = H.build_with_width(sysd, dev(x), dev(sig))
    D = dev(sig)
    acc, na = H.hdmd_swap(sysd, dev(x), D, ws, torch.as_tensor(pairs, device="cuda"), dev(u), T)
    assert na == na_o
    assert np.array_equal(acc.cpu().numpy(), acc_o)
    assert np.array_equal(D.cpu().numpy(), sig_o)


def test_swap_rejects_bad_input():
    x, sig, L = _case(3, 5, 1.4, 1, 1.4)
    n = len(x)
    sysd = H.System(d=3, n=n, box_l=L, cutoff=C6, skin=0.25, sigma_max=1.4)
    sysd, ws = H.build_with_width(sysd, dev(x), dev(sig))
    u = dev(np.full(2, 0.5))
    bad = torch.as_tensor(np.array([[0, 1], [2, n]], dtype=np.int32), device="cuda")
    with pytest.raises(H.HdmdError) as e:
        H.hdmd_swap(sysd, dev(x), dev(sig), ws, bad, u, 0.5)
    assert e.value.status == H.HDMD_ERR_ARG
    ok = torch.as_tensor(np.array([[0, 1], [2, 3]], dtype=np.int32), device="cuda")
    with pytest.raises(H.HdmdError) as e:
        H.hdmd_swap(sysd, dev(x), dev(sig), ws, ok, u, 0.0)
    assert e.value.status == H.HDMD_ERR_ARG
    D = dev(sig)
    acc, na = H.hdmd_swap(sysd, dev(x), D, ws, ok[:0], u[:0], 0.5)   # nothing to attempt
    assert na == 0 and np.array_equal(D.cpu().numpy(), sig)


def test_swap_chain_of_interfering_attempts(orc):
    """Every attempt exchanges atom 0 with another atom, so each one depends on
    the one before: the batches settle one attempt at a time and still give
    the serial outcome."""
    x, sig, L = _case(3, 6, 1.4, 31, 1.4)
    n = len(x)
    g = np.random.default_rng(32)
    m = 300
    pairs = np.stack([np.zeros(m, dtype=np.int32), g.integers(1, n, size=m).astype(np.int32)], 1)
    u = g.uniform(size=m)
    sig_o, acc_o, de_o, na_o = orc.swap(x, sig, L, H.HDMD_WCA, C6, 1.0, pairs, u, 2.0)
    thr = np.where(de_o <= 0, 2.0, np.exp(-np.maximum(de_o, 0) / 2.0))
    assert np.all((de_o <= 0) | (np.abs(u - thr) > 1e-9))
    sysd = H.System(d=3, n=n, box_l=L, cutoff=C6, skin=0.25, sigma_max=1.4)
    sysd, ws = H.build_with_width(sysd, dev(x), dev(sig))
    D = dev(sig)
    acc, na = H.hdmd_swap(sysd, dev(x), D, ws, torch.as_tensor(pairs, device="cuda"), dev(u), 2.0)
    assert na == na_o and 0 < na < m
    assert np.array_equal(acc.cpu().numpy(), acc_o)
    assert np.array_equal(D.cpu().numpy(), sig_o)
