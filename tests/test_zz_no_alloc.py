"""hdmd_forces_noalloc: hdmd_forces with the workspace in the library's own
scratch array (for callers that cannot allocate device memory).  Called
through the C ABI, its forces and energy equal hdmd_forces' bit for bit on two
calls in a row, the second on a smaller system, and match the oracle; a system
too large for the array is refused."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2112_12271_amd import hdmd as H
from paper_2112_12271_amd import inputs
from tests.gpu_util import dev, force_err

pytestmark = pytest.mark.gpu
C6 = inputs.WCA_CUT


def _lib():
    L = H.lib()
    L.hdmd_forces_noalloc.restype = C.c_int
    L.hdmd_forces_noalloc.argtypes = [C.POINTER(H.hdmd_system), C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p]
    L.hdmd_forces_noalloc_bytes.restype = C.c_size_t
    L.hdmd_forces_noalloc_bytes.argtypes = []
    return L


def _noalloc(sysd, x, sig):
    L = _lib()
    F = torch.empty((sysd.n, sysd.d), dtype=torch.float64, device="cuda")
    E = torch.empty((), dtype=torch.float64, device="cuda")
    X, S = dev(x), dev(sig)
    rc = L.hdmd_forces_noalloc(C.byref(sysd.c()), C.c_void_p(X.data_ptr()),
                               C.c_void_p(S.data_ptr()), C.c_void_p(F.data_ptr()),
                               C.c_void_p(E.data_ptr()), None)
    return rc, F, E


def _case(d, n, phi, seed, pot):
    sig = inputs.bidisperse(n, 1.0, 1.2, seed)
    L = inputs.box_for_packing(d, sig, phi)
    x = inputs.uniform_positions(n, d, L, seed + 1)
    cut = C6 if pot == H.HDMD_WCA else 1.0
    sysd = H.System(d=d, n=n, box_l=L, potential=pot, cutoff=cut, skin=0.3, sigma_max=1.2)
    return sysd, x, sig


def test_noalloc_forces_equal_hdmd_forces_twice(orc):
    cap = _lib().hdmd_forces_noalloc_bytes()
    assert cap == 16 << 20
    # the larger system first, then a smaller one over the same scratch array
    for d, n, phi, seed, pot in ((4, 6000, 0.42, 3, H.HDMD_WCA), (3, 700, 0.6, 5, H.HDMD_HARMONIC)):
        sysd, x, sig = _case(d, n, phi, seed, pot)
        sysd, ws = H.build_with_width(sysd, dev(x), dev(sig))
        assert H.hdmd_workspace_bytes(sysd) <= cap
        Fr, Er = H.hdmd_forces(sysd, dev(x), dev(sig), ws)
        rc, F, E = _noalloc(sysd, x, sig)
        assert rc == H.HDMD_OK, H.last_error()
        assert np.array_equal(F.cpu().numpy(), Fr.cpu().numpy()), (d, n)
        assert float(E) == float(Er)
        ref = orc.nlist_cells(x, sig, sysd.box_l, sysd.cutoff, sysd.skin)
        Fo, _, Eo = orc.forces(x, sig, sysd.box_l, pot, sysd.cutoff, 1.0, *ref)
        assert force_err(F.cpu().numpy(), Fo) < 1e-12
        assert abs(float(E) - Eo) <= 1e-12 * abs(Eo)


def test_noalloc_refuses_a_system_beyond_the_array():
    cap = _lib().hdmd_forces_noalloc_bytes()
    sysd, x, sig = _case(6, 200000, 0.3, 9, H.HDMD_WCA)
    sysd.max_neighbors = 128
    assert H.hdmd_workspace_bytes(sysd) > cap
    rc, _, _ = _noalloc(sysd, x, sig)
    assert rc == H.HDMD_ERR_WORKSPACE
    assert "scratch" in H.last_error()
