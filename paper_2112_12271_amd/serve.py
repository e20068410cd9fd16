"""Continuous-batching server for FIRE minimisations and short MD runs.

Requests of mixed d and N arrive over time (a seeded Poisson stream).  Each
admitted request occupies one slot of a batch table and its own workspace in
device memory; admission waits until a slot is free and the request's bytes
fit in the HBM budget.  Between chunks of batched iterations (one captured
graph replay) the loop retires finished slots, frees their memory and admits
waiting requests, so new work overlaps with work already on the device.

The loop only schedules: every iteration runs in the library's kernels through
the batch entry points (hdmd_batch_add_fire / _add_md / _run / _poll / _take).
The executor is pluggable so that the bookkeeping can be tested on the CPU.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                 # "fire" or "md"
    d: int
    n: int
    box_l: float
    x: np.ndarray             # (n, d) initial positions
    sig: np.ndarray           # (n,) diameters
    arrival: float            # seconds after the start of the run
    potential: int = 1        # HDMD_HARMONIC
    cutoff: float = 1.0
    skin: float = 0.25
    v: np.ndarray | None = None
    nsteps: int = 0
    dt: float = 0.0
    width: int = 0            # Verlet row capacity (0: estimated)


@dataclasses.dataclass
class Result:
    rid: int
    kind: str
    d: int
    n: int
    arrival: float
    admitted: float
    done: float
    iterations: int
    fmax: float
    energy: float
    status: int
    retries: int
    x: np.ndarray | None = None
    builds: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def estimate_width(d: int, n: int, box_l: float, rl: float, slack: float = 1.6) -> int:
    """Row capacity from the mean count within the list radius of a uniform
    gas, with room for density fluctuations."""
    vball = math.pi ** (0.5 * d) * rl ** d / math.gamma(1.0 + 0.5 * d)
    mean = min(n - 1, n * vball / box_l ** d)
    return int(min(n - 1, slack * mean + 6.0 * math.sqrt(mean) + 16)) + 1


def percentiles(lat: list[float]) -> dict:
    if not lat:
        return {"p50": None, "p99": None, "mean": None}
    a = np.sort(np.asarray(lat))
    return {"p50": float(np.percentile(a, 50)), "p99": float(np.percentile(a, 99)),
            "mean": float(a.mean())}


class Server:
    """Admission by HBM budget + continuous batching over an executor.

    executor must provide: workspace_bytes(req, width) -> int;
    add(slot, req, width) (allocates the request's device memory);
    run(iterations); poll() -> (state[], iters[]);
    take(slot) -> (x, iterations, fmax, energy, status, builds); release(slot).
    """

    STATE_EMPTY, STATE_RUNNING, STATE_DONE = 0, 1, 2
    ERR_OVERFLOW = -4

    def __init__(self, executor, max_slots: int, hbm_budget: int, chunk: int = 50,
                 keep_positions: bool = False, clock=time.perf_counter):
        self.ex = executor
        self.max_slots = max_slots
        self.budget = hbm_budget
        self.chunk = chunk
        self.keep = keep_positions
        self.clock = clock
        self.in_use = 0
        self.slot_req: dict[int, tuple] = {}
        self.max_in_use = 0
        self.max_active = 0

    def _admit(self, req, now, retries):
        free = [s for s in range(self.max_slots) if s not in self.slot_req]
        if not free:
            return False
        width = req.width or estimate_width(req.d, req.n, req.box_l,
                                            req.cutoff * float(req.sig.max()) + req.skin)
        nbytes = self.ex.workspace_bytes(req, width)
        if self.in_use + nbytes > self.budget and self.slot_req:
            return False
        if nbytes > self.budget:
            raise ValueError("request %d needs %d bytes, more than the whole budget"
                             % (req.rid, nbytes))
        slot = free[0]
        self.ex.add(slot, req, width)
        self.slot_req[slot] = (req, now, nbytes, width, retries)
        self.in_use += nbytes
        self.max_in_use = max(self.max_in_use, self.in_use)
        self.max_active = max(self.max_active, len(self.slot_req))
        return True

    def serve(self, requests: list[Request], time_limit: float = 600.0) -> list[Result]:
        """Runs until every request is done.  Arrival times are honoured against
        the wall clock: a request is not admitted before it arrives."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque = collections.deque()
        results: list[Result] = []
        t0 = self.clock()
        while pending or waiting or self.slot_req:
            now = self.clock() - t0
            if now > time_limit:
                raise TimeoutError("serve() exceeded its time limit")
            while pending and pending[0].arrival <= now:
                waiting.append((pending.popleft(), 0))
            # admission in arrival order (head-of-line: keeps latency fair)
            while waiting:
                req, retries = waiting[0]
                if not self._admit(req, now, retries):
                    break
                waiting.popleft()
            if not self.slot_req:
                if pending:   # idle until the next arrival
                    wait = pending[0].arrival - (self.clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            self.ex.run(self.chunk)
            state, _ = self.ex.poll()
            now = self.clock() - t0
            for slot in sorted(self.slot_req):
                if state[slot] != self.STATE_DONE:
                    continue
                req, adm, nbytes, width, retries = self.slot_req.pop(slot)
                x, iters, fmax, energy, status, builds = self.ex.take(slot)
                self.ex.release(slot)
                self.in_use -= nbytes
                if status == self.ERR_OVERFLOW:
                    # rerun from the original input with a wider row capacity
                    req = dataclasses.replace(req, width=int(width * 1.5) + 16)
                    waiting.appendleft((req, retries + 1))
                    continue
                results.append(Result(req.rid, req.kind, req.d, req.n, req.arrival, adm, now,
                                      iters, fmax, energy, status, retries,
                                      x if self.keep else None, builds))
        return results


def summarize(results: list[Result], wall: float) -> dict:
    lat = [r.latency for r in results]
    out = {"completed": len(results), "wall_s": wall,
           "solves_per_s": len(results) / wall if wall > 0 else None}
    out.update({"latency_" + k: v for k, v in percentiles(lat).items()})
    return out


class GpuExecutor:
    """Executor over the library's batch table; device memory comes from torch."""

    def __init__(self, max_slots: int, max_atoms: int, max_cells: int, precision: int,
                 fire_params=None):
        import torch

        from . import hdmd as H
        self.H = H
        self.torch = torch
        self.batch = H.Batch(max_slots, max_atoms, max_cells)
        self.precision = precision
        self.params = fire_params
        self.mem: dict[int, tuple] = {}

    def system(self, req: Request, width: int):
        H = self.H
        return H.System(d=req.d, n=req.n, box_l=req.box_l, potential=req.potential,
                        cutoff=req.cutoff, skin=req.skin, sigma_max=float(req.sig.max()),
                        precision=self.precision, max_neighbors=width)

    def workspace_bytes(self, req: Request, width: int) -> int:
        return self.H.hdmd_workspace_bytes(self.system(req, width)) + req.n * (req.d + 1) * 8 * 2

    def add(self, slot: int, req: Request, width: int):
        torch, H = self.torch, self.H
        sysd = self.system(req, width)
        ws = H.workspace(sysd)
        dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64,
                                        device="cuda")
        X, SG = dev(req.x), dev(req.sig)
        if req.kind == "fire":
            self.batch.hdmd_batch_add_fire(slot, sysd, X, SG, ws, self.params)
        else:
            self.batch.hdmd_batch_add_md(slot, sysd, X, dev(req.v), SG, ws, req.nsteps, req.dt)
        self.mem[slot] = (ws, X, SG)

    def run(self, iterations: int):
        self.batch.hdmd_batch_run(iterations)

    def poll(self):
        return self.batch.hdmd_batch_poll()

    def take(self, slot: int):
        H = self.H
        try:
            pos, _, res = self.batch.hdmd_batch_take(slot)
        except H.HdmdError as e:
            return None, 0, float("nan"), float("nan"), e.status, 0
        return pos.cpu().numpy(), res.iterations, res.fmax, res.energy, res.status, res.builds

    def release(self, slot: int):
        self.mem.pop(slot, None)
