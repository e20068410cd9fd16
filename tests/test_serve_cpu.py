"""The continuous-batching scheduler against a CPU stand-in executor whose
FIRE runs in the oracle (no GPU): HBM budget, arrival order, retries."""
import numpy as np
import pytest

from paper_2112_12271_amd import inputs
from paper_2112_12271_amd import serve as S


class FakeExecutor:
    """Batch-table stand-in: a slot finishes after a number of iterations that
    grows with its size; FIRE results come from the oracle."""

    def __init__(self, orc, overflow_once=()):
        self.orc = orc
        self.slots = {}
        self.overflow_once = set(overflow_once)
        self.log = []

    def workspace_bytes(self, req, width):
        return req.n * (64 + 4 * width)

    def add(self, slot, req, width):
        self.log.append(("add", req.rid, slot, width))
        self.slots[slot] = {"req": req, "width": width, "it": 0, "need": 20 + req.n // 10}

    def run(self, iterations):
        for s in self.slots.values():
            s["it"] += iterations

    def poll(self):
        state = np.zeros(16, dtype=np.int32)
        iters = np.zeros(16, dtype=np.int64)
        for k, s in self.slots.items():
            state[k] = 2 if s["it"] >= s["need"] else 1
            iters[k] = s["it"]
        return state, iters

    def take(self, slot):
        s = self.slots[slot]
        req = s["req"]
        if req.rid in self.overflow_once:
            self.overflow_once.discard(req.rid)
            return None, 0, 0.0, 0.0, -4, 0
        x, res = self.orc.fire(req.x, req.sig, req.box_l, self.orc.HARMONIC, 1.0, 0.25, 1.0,
                               self.orc.fire_params(ftol=1e-8, maxiter=20000))
        return x, res.iters, res.fmax, res.energy, 0, res.builds

    def release(self, slot):
        del self.slots[slot]


def _requests(count, rate=50.0):
    phij = {3: 0.64, 4: 0.46}
    reqs = inputs.fire_requests(count, phij, rate, seed=77, n_lo=64, n_hi=256, d_choices=(3, 4))
    out = []
    for r in reqs:
        out.append(S.Request(r.rid, "fire", r.d, r.n, r.L, r.positions(), r.sig, r.arrival))
    return out


def test_budget_order_and_results(orc):
    reqs = _requests(12)
    ex = FakeExecutor(orc, overflow_once=(3,))
    budget = max(ex.workspace_bytes(r, S.estimate_width(r.d, r.n, r.box_l, 1.65)) for r in reqs) * 3
    srv = S.Server(ex, max_slots=8, hbm_budget=budget, chunk=10)
    res = srv.serve(reqs, time_limit=120)
    assert sorted(r.rid for r in res) == list(range(12))
    assert srv.max_in_use <= budget
    assert srv.max_active <= 8
    byid = {r.rid: r for r in res}
    assert byid[3].retries == 1                      # overflow -> rerun wider
    widths = [w for (_, rid, _, w) in ex.log if rid == 3]
    assert widths[1] > widths[0]
    for r in res:
        assert r.admitted >= r.arrival - 1e-9 and r.done >= r.admitted
        assert r.status == 0 and r.fmax < 1e-8
    # admissions follow arrival order
    firsts = []
    for (_, rid, _, _) in ex.log:
        if rid not in firsts:
            firsts.append(rid)
    arr = {r.rid: r.arrival for r in reqs}
    assert [arr[r] for r in firsts] == sorted(arr[r] for r in firsts)


def test_request_larger_than_budget_rejected(orc):
    reqs = _requests(2)
    ex = FakeExecutor(orc)
    srv = S.Server(ex, max_slots=2, hbm_budget=10, chunk=10)
    with pytest.raises(ValueError):
        srv.serve(reqs, time_limit=10)


def test_percentiles_and_width_estimate():
    p = S.percentiles([1.0, 2.0, 3.0, 4.0])
    assert p["p50"] == pytest.approx(2.5)
    assert S.estimate_width(3, 1000, 10.0, 1.5) > 1000 * (4 / 3 * np.pi * 1.5 ** 3) / 1000.0
