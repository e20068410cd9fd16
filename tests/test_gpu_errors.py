"""Documented status codes for invalid inputs, forced from the host side."""
import numpy as np
import pytest

from paper_2112_12271_amd import hdmd as H
from paper_2112_12271_amd import inputs
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


def _case(n=200, d=3, L=6.0):
    return inputs.uniform_positions(n, d, L, 1), np.ones(n)


def test_box_too_small():
    x, sig = _case(L=1.5)
    s = H.System(d=3, n=200, box_l=1.5, cutoff=1.0, skin=0.2, sigma_max=1.0)
    with pytest.raises(H.HdmdError) as e:
        H.hdmd_build_nlist(s, dev(x), dev(sig), H.workspace(H.System(d=3, n=200, box_l=6.0)))
    assert e.value.status == H.HDMD_ERR_BOX


def test_bad_dimension_and_workspace():
    x, sig = _case()
    s = H.System(d=11, n=200, box_l=6.0)
    with pytest.raises(H.HdmdError) as e:
        H.hdmd_workspace_bytes(s)
    assert e.value.status == H.HDMD_ERR_ARG
    s = H.System(d=3, n=200, box_l=6.0, sigma_max=1.0)
    import torch
    tiny = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(H.HdmdError) as e:
        H.hdmd_build_nlist(s, dev(x), dev(sig), tiny)
    assert e.value.status == H.HDMD_ERR_WORKSPACE


def test_nonfinite_and_out_of_box():
    x, sig = _case()
    s = H.System(d=3, n=200, box_l=6.0, sigma_max=1.0)
    ws = H.workspace(s)
    y = x.copy()
    y[7, 1] = np.nan
    with pytest.raises(H.HdmdError) as e:
        H.hdmd_build_nlist(s, dev(y), dev(sig), ws)
    assert e.value.status == H.HDMD_ERR_NONFINITE
    y = x.copy()
    y[3, 0] = 100.0
    with pytest.raises(H.HdmdError) as e:
        H.hdmd_build_nlist(s, dev(y), dev(sig), ws)
    assert e.value.status == H.HDMD_ERR_ARG
    big = sig.copy()
    big[0] = 2.0
    with pytest.raises(H.HdmdError) as e:
        H.hdmd_build_nlist(s, dev(x), dev(big), ws)
    assert e.value.status == H.HDMD_ERR_ARG


def test_overflow_reports_width(orc):
    x, L = inputs.jittered_lattice(3, 6, 1.0, 0.1, 0)
    sig = np.ones(len(x))
    s = H.System(d=3, n=len(x), box_l=L, cutoff=1.0, skin=0.9, sigma_max=1.0, max_neighbors=4)
    rc, rw = H.hdmd_build_nlist(s, dev(x), dev(sig), H.workspace(s))
    assert rc == H.HDMD_ERR_NLIST_OVERFLOW
    rp, _ = orc.nlist_brute(x, sig, L, 1.0, 0.9)
    assert rw == np.diff(rp).max()
    s2, ws = H.build_with_width(s, dev(x), dev(sig))
    assert s2.max_neighbors >= rw
