"""Pins of the oracle's FIRE 2.0 control sequence (Sec. II.B: FIRE 2.0 with the
semi-implicit Euler update), CPU only.

The outcome pins elsewhere (separation, zero energy, converged jammed states)
would still pass with a wrong control rule.  These check the per-iteration
trace (P, dt, alpha, run counts, step-back flag) against sequences written from
the published FIRE 2.0 rules, and small two- and three-atom cases whose first
iterations are worked out here:

* P > 0: N+ += 1, N- = 0; once N+ > N_delay, dt = min(f_inc dt, dt_max) and
  alpha *= f_alpha.
* P <= 0: N+ = 0, N- += 1; unless inside the initial delay (iteration <
  N_delay), dt *= f_dec when that stays >= dt_min, and alpha = alpha_start;
  then x -= dt/2 v with that (new) dt, and v = 0.
* then v += dt F, v = (1 - alpha) v + alpha |v| F/|F|, x += dt v.
"""
import numpy as np
import pytest

HARM = 1
L_BOX = 10.0


def _two(r0=0.5):
    x = np.array([[-0.5 * r0, 0.0], [0.5 * r0, 0.0]])
    return x, np.ones(2)


def _run(orc, x, sig, maxiter, **kw):
    p = orc.fire_params(ftol=0.0, maxiter=maxiter, **kw)
    return orc.fire(x, sig, L_BOX, HARM, 1.0, 0.25, 1.0, p, trace=True)


def _expected_control(P, dt0=0.05, dtmax=None, dtmin=None, finc=1.1, fdec=0.5, a0=0.25,
                      fa=0.99, ndelay=20, initial_delay=True):
    """dt, alpha, N+, N-, step-back flag of every iteration from the sign
    sequence of P alone, by the FIRE 2.0 rules."""
    dtmax = 10 * dt0 if dtmax is None else dtmax
    dtmin = 0.02 * dt0 if dtmin is None else dtmin
    dt, a, npos, nneg = dt0, a0, 0, 0
    rows = []
    for it, p in enumerate(P):
        back = 0
        if p > 0:
            npos, nneg = npos + 1, 0
            if npos > ndelay:
                dt = min(dt * finc, dtmax)
                a = a * fa
        else:
            npos, nneg = 0, nneg + 1
            if not (initial_delay and it < ndelay):
                if dt * fdec >= dtmin:
                    dt = dt * fdec
                a = a0
            back = 1
        rows.append((dt, a, npos, nneg, back))
    return np.array(rows)


def test_hand_worked_first_three_iterations(orc):
    """Two unit harmonic spheres at r = 0.5 in d = 2, dt0 = 0.1 (worked by hand):
    iteration 0 has v = 0, so P = 0 <= 0 inside the initial delay: dt and alpha
    stay, nothing moves back; v = dt F = 0.05 along the axis, x1 = 0.255.
    Iteration 1: |F_i| = 1 - 0.51 = 0.49, P = 2 * 0.49 * 0.05 = 0.049;
    v = 0.05 + 0.049 = 0.099 (mixing keeps a velocity parallel to F);
    x1 = 0.2649.  Iteration 2: |F_i| = 0.4702, P = 2 * 0.4702 * 0.099 = 0.0930996;
    v = 0.14602, x1 = 0.279502."""
    x, sig = _two()
    want = [0.255, 0.2649, 0.279502]
    for k, w in enumerate(want, start=1):
        x1, res, tr = _run(orc, x, sig, k, dt0=0.1)
        assert res.iters == k
        assert x1[1, 0] == pytest.approx(w, abs=1e-14)
        assert x1[0, 0] == pytest.approx(-w, abs=1e-14)
        assert x1[:, 1] == pytest.approx([0.0, 0.0], abs=0)
    assert tr[:, 0] == pytest.approx([0.0, 0.049, 0.0930996], abs=1e-14)
    assert tr[:, 1] == pytest.approx([0.1, 0.1, 0.1], abs=0)
    assert list(tr[:, 5]) == [1.0, 0.0, 0.0]


def test_hand_worked_without_initial_delay(orc):
    """Same start with the initial delay off: iteration 0's P = 0 halves dt to
    0.05 at once (alpha stays alpha_start); v = 0.05 * 0.5 = 0.025, x1 = 0.25125."""
    x, sig = _two()
    x1, res, tr = _run(orc, x, sig, 1, dt0=0.1, initial_delay=0)
    assert tr[0, 1] == 0.05 and tr[0, 2] == 0.25 and tr[0, 5] == 1.0
    assert x1[1, 0] == pytest.approx(0.25125, abs=1e-15)


def _pairwise_harmonic(x, sig, L):
    """Forces of harmonic spheres, U = (1 - r/s)^2 / 2 for r < s = (s_i+s_j)/2,
    by direct summation over pairs (minimum image)."""
    n = len(x)
    F = np.zeros_like(x)
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            dx = x[j] - x[i]
            dx -= L * np.round(dx / L)
            r = np.sqrt((dx * dx).sum())
            s = 0.5 * (sig[i] + sig[j])
            if r < s:
                F[i] -= (1.0 - r / s) / s * dx / r
    return F


def _worked(x0, sig, dt, iters, order="kick_then_mix", a=0.25):
    """The first iterations (inside the initial delay, so dt and alpha stay)
    with forces summed pair by pair."""
    x = x0.copy()
    v = np.zeros_like(x)
    for _ in range(iters):
        F = _pairwise_harmonic(x, sig, L_BOX)
        if not (F * v).sum() > 0:
            x = x - 0.5 * dt * v
            v = np.zeros_like(v)
        mix = lambda u: (1 - a) * u + a * np.sqrt((u * u).sum()) * F / np.sqrt((F * F).sum())
        if order == "kick_then_mix":
            v = mix(v + dt * F)
        elif order == "mix_then_kick":
            v = mix(v) + dt * F
        else:
            v = v + dt * F
        x = x + dt * v
    return x


def test_four_atoms_mix_after_kick(orc):
    """Four spheres in d = 2 whose forces turn between iterations, so the
    mixing step is visible: positions after 1, 2, 3 iterations follow
    v <- v + dt F, then v <- (1-alpha) v + alpha |v| F/|F|, then x <- x + dt v.
    Mixing before the kick, or no mixing, ends elsewhere by far more than the
    tolerance."""
    x0 = np.array([[0.0, 0.0], [0.6, 0.1], [0.1, 0.5], [-0.4, 0.3]])
    sig = np.array([1.0, 1.4, 1.0, 1.4])
    for k in (1, 2, 3):
        x1, res, tr = _run(orc, x0, sig, k, dt0=0.2)
        assert np.abs(x1 - _worked(x0, sig, 0.2, k)).max() < 1e-13, k
    good = _worked(x0, sig, 0.2, 3)
    assert np.abs(good - _worked(x0, sig, 0.2, 3, "mix_then_kick")).max() > 1e-7
    assert np.abs(good - _worked(x0, sig, 0.2, 3, "no_mix")).max() > 1e-5


def test_trace_follows_the_rules_long_positive_run(orc):
    """dt0 = 0.003: P > 0 for more than N_delay iterations, so dt grows by f_inc
    per iteration up to dt_max and alpha decays by f_alpha; when the spheres
    separate (F = 0, P = 0) dt halves and alpha resets."""
    x, sig = _two()
    x1, res, tr = _run(orc, x, sig, 200, dt0=0.003)
    P = tr[:, 0]
    first_pos = np.nonzero(P > 0)[0]
    assert first_pos[0] == 1
    ev = np.nonzero((P <= 0) & (np.arange(len(P)) > 0))[0]
    assert len(ev) and ev[0] > 40, "needs a P > 0 run well beyond N_delay"
    exp = _expected_control(P, dt0=0.003)
    assert np.array_equal(tr[:, 1], exp[:, 0]), "dt sequence"
    assert np.array_equal(tr[:, 2], exp[:, 1]), "alpha sequence"
    assert np.array_equal(tr[:, 3:6], exp[:, 2:5]), "run counts and step-back flags"
    # the delay: dt0 for the first N_delay positive iterations, then growth
    assert np.all(tr[1:21, 1] == 0.003) and tr[21, 1] > 0.003 and tr[21, 2] < 0.25
    assert tr[21, 1] == 0.003 * 1.1 and tr[22, 1] == 0.003 * 1.1 * 1.1
    assert tr[21, 2] == 0.25 * 0.99 and tr[22, 2] == 0.25 * 0.99 * 0.99
    # dt_max is reached and held (10 dt0)
    top = tr[:ev[0], 1]
    assert top.max() == 0.03 and np.all(top[np.argmax(top):] == 0.03)
    k = ev[0]
    assert tr[k - 1, 2] < 0.25 and tr[k, 2] == 0.25           # alpha resets
    assert tr[k, 1] == 0.5 * tr[k - 1, 1]                      # dt halves


def _positions(orc, x, sig, its, **kw):
    return [_run(orc, x, sig, k, **kw)[0] for k in its]


@pytest.mark.parametrize("dt0,after_delay", [(0.1, False), (0.01, True)])
def test_step_back_uses_the_new_dt(orc, dt0, after_delay):
    """At the iteration k where the spheres have just separated (F = 0, so
    P = 0): x <- x - dt_new/2 v and v = 0, with v the velocity of the previous
    drift, v = (x_k - x_{k-1}) / dt_{k-1}; F = 0 leaves nothing to kick, so
    x_{k+1} - x_k = -(dt_new / (2 dt_{k-1})) (x_k - x_{k-1}): a quarter of the
    last drift after the delay (dt halves), a half inside it (dt stays)."""
    x, sig = _two()
    _, _, tr = _run(orc, x, sig, 120, dt0=dt0)
    P = tr[:, 0]
    k = int(np.nonzero((P <= 0) & (np.arange(len(P)) > 0))[0][0])
    assert (k >= 20) == after_delay
    xm, xk, xp = _positions(orc, x, sig, (k - 1, k, k + 1), dt0=dt0)
    assert np.linalg.norm(xk[1] - xk[0]) > 1.0                 # separated: F = 0
    ratio = tr[k, 1] / (2.0 * tr[k - 1, 1])
    assert ratio == (0.25 if after_delay else 0.5)
    assert np.abs((xp - xk) + ratio * (xk - xm)).max() < 1e-15
    assert tr[k, 5] == 1.0


def test_dt_floor(orc):
    """Repeated P <= 0 after the delay halves dt only while it stays >= dt_min
    (0.02 dt0): 0.1 -> 0.05 ... 0.003125, then it holds."""
    x, sig = _two()
    _, _, tr = _run(orc, x, sig, 60, dt0=0.1)
    late = tr[23:, 1]
    assert late[0] == 0.05
    assert late.min() == 0.003125 and np.all(late >= 0.002)
    exp = _expected_control(tr[:, 0], dt0=0.1)
    assert np.array_equal(tr[:, 1:6], exp)
