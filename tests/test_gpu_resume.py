"""hdmd_step_resume: a velocity-Verlet run split into calls continues without a
reload or a list rebuild, and gives the bits of one longer call (the list,
the atom order and the trigger's reference positions carry over)."""
import numpy as np
import pytest
import torch

from paper_2112_12271_amd import hdmd as H
from paper_2112_12271_amd import inputs
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu
C6 = inputs.WCA_CUT


def _state(d, m, a, seed, T=1.0):
    x, L = inputs.jittered_lattice(d, m, a, 0.12 * a, seed)
    n = len(x)
    sig = inputs.bidisperse(n, 1.0, 1.2, seed)
    v = inputs.gaussian_velocities(n, d, T, seed + 1)
    return x, v, sig, L


@pytest.mark.parametrize("d,m,a,skin,prec,tau", [(3, 8, 1.12, 0.3, H.HDMD_FP64, 0.0),
                                                 (4, 5, 1.1, 0.3, H.HDMD_FP64, 0.0),
                                                 (6, 4, 1.05, 0.25, H.HDMD_FP64, 0.0),
                                                 (6, 4, 1.05, 0.25, H.HDMD_MIXED, 0.0),
                                                 (3, 8, 1.12, 0.3, H.HDMD_FP64, 0.05)])
def test_resume_equals_one_call_and_the_oracle(orc, d, m, a, skin, prec, tau):
    x, v, sig, L = _state(d, m, a, 5 * d)
    dt, n1, n2 = 0.004, 40, 60
    sysd = H.System(d=d, n=len(x), box_l=L, cutoff=C6, skin=skin, sigma_max=1.2, precision=prec,
                    thermostat_tau=tau, target_temp=0.5 if tau else 0.0)
    # rows grow along the run: room for that (the width changes no result)
    sysd, _ = H.build_with_width(sysd, dev(x), dev(sig))
    sysd.max_neighbors = 2 * sysd.max_neighbors + 32
    ws = H.workspace(sysd)
    # one call of n1 + n2 steps
    X1, V1, S = dev(x), dev(v), dev(sig)
    st, th = H.hdmd_step(sysd, X1, V1, S, ws, n1 + n2, dt, 1)
    # the same run split in two calls, the second resumed
    ws2 = H.workspace(sysd)
    X2, V2 = dev(x), dev(v)
    sa, tha = H.hdmd_step(sysd, X2, V2, S, ws2, n1, dt, 1)
    sb, thb = H.hdmd_step(sysd, X2, V2, S, ws2, n2, dt, 1, resume=True)
    assert np.array_equal(X1.cpu().numpy(), X2.cpu().numpy())
    assert np.array_equal(V1.cpu().numpy(), V2.cpu().numpy())
    th, tha, thb = th.cpu().numpy(), tha.cpu().numpy(), thb.cpu().numpy()
    assert np.array_equal(thb[:, 1:4], th[n1:, 1:4])          # KE, PE, E at every step
    assert sa.builds + sb.builds == st.builds                 # no extra build at the resume
    assert np.all(thb[0, 6:8] == 0.0)                        # observables restart from zero
    assert sb.steps_done == n2
    if prec == H.HDMD_FP64 and tau == 0.0:
        xo, vo, tho, bo = orc.vv(x, v, sig, L, 0, C6, skin, 1.0, n1 + n2, dt)
        dx = X2.cpu().numpy() - xo
        dx -= L * np.round(dx / L)
        assert np.abs(dx).max() < 1e-9
        assert np.abs(V2.cpu().numpy() - vo).max() < 1e-8
        assert sa.builds + sb.builds + 1 == bo


def test_resume_refuses_a_changed_state():
    x, v, sig, L = _state(3, 6, 1.12, 2)
    sysd = H.System(d=3, n=len(x), box_l=L, cutoff=C6, skin=0.3, sigma_max=1.2)
    sysd, _ = H.build_with_width(sysd, dev(x), dev(sig))
    sysd.max_neighbors = 2 * sysd.max_neighbors + 32
    ws = H.workspace(sysd)
    H.hdmd_build_nlist(sysd, dev(x), dev(sig), ws)
    X, V, S = dev(x), dev(v), dev(sig)
    # a workspace that holds no run
    with pytest.raises(H.HdmdError) as e:
        H.hdmd_step(sysd, X, V, S, ws, 10, 0.004, resume=True)
    assert e.value.status == H.HDMD_ERR_STATE
    H.hdmd_step(sysd, X, V, S, ws, 10, 0.004)
    for what in ("pos", "vel", "diam"):
        X2, V2, S2 = X.clone(), V.clone(), S.clone()
        if what == "diam":
            S2[7] = 1.2 if float(S[7]) == 1.0 else 1.0          # the other diameter
        else:
            t = X2 if what == "pos" else V2
            t.view(-1)[7] = t.view(-1)[7] * (1 + 1e-15) + 1e-300   # a few ulps
        assert not (torch.equal(X2, X) and torch.equal(V2, V) and torch.equal(S2, S))
        pre = X2.clone()
        with pytest.raises(H.HdmdError) as e:
            H.hdmd_step(sysd, X2, V2, S2, ws, 10, 0.004, resume=True)
        assert e.value.status == H.HDMD_ERR_STATE, what
        assert np.array_equal(X2.cpu().numpy(), pre.cpu().numpy())   # caller arrays untouched
    # another system (skin) on the same workspace
    other = H.System(d=3, n=len(x), box_l=L, cutoff=C6, skin=0.29, sigma_max=1.2,
                     max_neighbors=sysd.max_neighbors)
    with pytest.raises(H.HdmdError) as e:
        H.hdmd_step(other, X, V, S, ws, 10, 0.004, resume=True)
    assert e.value.status == H.HDMD_ERR_STATE
    # the untouched state resumes
    st, _ = H.hdmd_step(sysd, X, V, S, ws, 10, 0.004, resume=True)
    assert st.steps_done == 10
