#!/usr/bin/env python
"""Throughput of the hdMD hot path on one MI355X.

One step = one pass of the whole hot path over the system: the fused
velocity-Verlet kernel (forces, kicks, drift, rebuild trigger) and, when the
largest displacement since the last build exceeds skin/2, the subcell binning,
counting sort and Verlet-list rebuild.

Workload (default): d=6, N=262144, 50:50 WCA mixture sigma 1.0/1.2 at packing
fraction 0.42, dt=0.002, skin 0.25, T=1.0.  Untimed set-up: seeded uniform
positions relaxed by FIRE on harmonic soft spheres, Gaussian velocities at
T=1, then --equil-steps FP64 steps, so that the timed steps see the liquid the
10^4-step run spends its time in rather than the heating right after the
relaxation.  Then, in FP64 and in the mixed form: one call of W warm-up steps
(it loads the state and builds the list) and three windows of exactly K steps,
each a resumed call (no reload, no extra list build), in the same launch mode
as the warm-up: kernels launched one by one with HIP events around every
fused-step and list-build kernel.  The window with the median time is
reported.  A separate --long-steps run per precision (captured-graph replay,
the library's production mode) gives the 10^4-step figures and the energy
drift.

Prints one JSON line.  `value` is atom-steps/s of the FP64 median window with
inputs resident in HBM.  `roofline` is the fused-step kernel's algorithmic
bytes per launch (the compulsory per-atom bytes of a step, step_bytes_per_atom,
times N) over its mean duration measured with HIP events inside that window.
`cpu_baseline` is the oracle built with OpenMP on the host's threads, on a
bounded sample described in the line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9   # vector lane-operations per second (MI355X)
MF_FLAG = 1024                                  # build-variant flag: pair tests on the matrix cores


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def step_bytes_per_atom(d: int, mean_row: float, mixed: bool) -> float:
    """Compulsory bytes of one fused step per atom: read x (8d), write x (8d),
    read x_ref (8d), read+write v (2 b_v d), the row (4 per entry), row length
    (4) and own diameter (8).  Gathered neighbour data is not counted."""
    bv = 4 if mixed else 8
    return 8 * d * 3 + 2 * bv * d + 4 * mean_row + 4 + 8


def build_candidates(x: np.ndarray, L: float, nc: int) -> int:
    """Candidate pairs one list build meets (Sec. II.B): for every subcell c,
    its atoms times the atoms of the 3^d subcells linked to it, from the
    subcell occupancy of positions x with nc >= 3 subcells per axis."""
    d = x.shape[1]
    idx = np.minimum((np.mod(x, L) * (nc / L)).astype(np.int64), nc - 1)
    occ = np.zeros((nc,) * d, dtype=np.int64)
    np.add.at(occ, tuple(idx.T), 1)
    linked = np.zeros_like(occ)
    for off in np.ndindex(*(3,) * d):
        linked += np.roll(occ, tuple(o - 1 for o in off), axis=tuple(range(d)))
    return int((occ * linked).sum())


def workload_name(cfg) -> str:
    if cfg.poly_R > 0:
        mix = "polydisperse P(d,R=%g,sigma)" % cfg.poly_R
    elif cfg.sig_a == cfg.sig_b:
        mix = "monodisperse sigma %.1f" % cfg.sig_a
    else:
        mix = "50:50 sigma %.1f/%.1f" % (cfg.sig_a, cfg.sig_b)
    pot = {0: "WCA", 1: "harmonic", 2: "Morse a=30"}[cfg.potential]
    dens = "phi=%.4g" % cfg.phi if cfg.phi is not None else "rho=%.4g" % cfg.rho
    return "%s: d=%d N=%d %s %s %s dt=%g skin=%g T=%g" % (
        cfg.name, cfg.d, cfg.n, mix, pot, dens, cfg.dt, cfg.skin, cfg.T)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.h", "hdmd_dev.h"):
        h.update(open(os.path.join(ROOT, "paper_2112_12271_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def committed_traffic(name: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source; otherwise None."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def drift(th: np.ndarray, n: int, dt: float) -> tuple[float, float]:
    """Least-squares slope of (E_tot(t) - E_tot(0))/N per unit time, and the
    RMS fluctuation of E_tot/N."""
    t = th[:, 0] * dt
    e = th[:, 3] / n
    if len(t) < 2:
        return 0.0, 0.0
    A = np.vstack([t, np.ones_like(t)]).T
    slope = float(np.linalg.lstsq(A, e - e[0], rcond=None)[0][0])
    return slope, float(np.std(e))


def md_system(H, cfg, L, sig, prec, width=64, tau=0.0):
    return H.System(d=cfg.d, n=cfg.n, box_l=L, potential=cfg.potential, cutoff=cfg.cutoff,
                    skin=cfg.skin, sigma_max=float(sig.max()), precision=prec,
                    max_neighbors=width, thermostat_tau=tau, target_temp=cfg.T if tau else 0.0)


def sized_width(H, torch, sysd, X, V, SIG, dt):
    """Row capacity for this state: a one-step run on copies (regrown on
    overflow), with room for the rows to grow along the trajectory."""
    sysd, _, _ = H.step_auto(sysd, X.clone(), V.clone(), SIG, 1, dt)
    sysd.max_neighbors = int(sysd.max_neighbors * 1.25) + 16
    return sysd


def run_windows(H, torch, cfg, X0, V0, SIG, L, prec, steps, warmup, windows, every, profile, tau):
    """One warm-up call (load, list build, W steps) and `windows` resumed calls
    of exactly `steps` steps, all in the same launch mode; returns the record
    of each window (wall time around the call, kernel times of the call)."""
    sysd = sized_width(H, torch, md_system(H, cfg, L, SIG.cpu().numpy(), prec, tau=tau), X0, V0,
                       SIG, cfg.dt)
    if profile:
        os.environ["HDMD_PROFILE"] = "1"
    else:
        os.environ.pop("HDMD_PROFILE", None)
    try:
        for attempt in range(4):
            X, V = X0.clone(), V0.clone()
            ws = H.workspace(sysd)
            out = []
            try:
                H.hdmd_step(sysd, X, V, SIG, ws, max(warmup, 1), cfg.dt)
                for w in range(windows):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st, th = H.hdmd_step(sysd, X, V, SIG, ws, steps, cfg.dt, every, resume=True)
                    torch.cuda.synchronize()
                    out.append(dict(seconds=time.perf_counter() - t0, stats=st,
                                    thermo=th.cpu().numpy() if th is not None else None))
            except H.HdmdError as e:
                if e.status != H.HDMD_ERR_NLIST_OVERFLOW:
                    raise
                sysd.max_neighbors = int(sysd.max_neighbors * 1.5) + 16
                continue
            break
    finally:
        os.environ.pop("HDMD_PROFILE", None)
    rp, cols = H.hdmd_nlist_export(sysd, ws)
    mean_row = cols.numel() / cfg.n
    nc = H.hdmd_cells_per_axis(sysd)
    cand = build_candidates(X.cpu().numpy(), L, nc) if nc >= 3 else None
    variant = H.hdmd_build_config(sysd)[3]
    return out, dict(mean_row=mean_row, width=sysd.max_neighbors, candidates=cand,
                     build_variant=variant)


def build_kernel_name(d: int, variant: int) -> str:
    """The list-build kernel a build variant launches (n_cell >= 3)."""
    g = variant & ~MF_FLAG
    if g >= 64:
        return "k_build<%d,%d lanes>" % (d, g)
    return "k_build_t<%d,%d%s>" % (d, g, ",matrix-core tests" if variant & MF_FLAG else "")


def window_record(cfg, prec_mixed, win, meta, steps):
    """The median window (by wall time) with its kernel shares."""
    order = sorted(range(len(win)), key=lambda k: win[k]["seconds"])
    w = win[order[len(order) // 2]]
    st = w["stats"]
    ms = 1e3 * w["seconds"]
    rec = dict(value=cfg.n * steps / w["seconds"], ms_per_step=ms / steps,
               windows_ms_per_step=[1e3 * x["seconds"] / steps for x in win],
               builds=int(st.builds), steps_per_build=steps / max(st.builds, 1),
               mean_row=meta["mean_row"], max_row=int(st.max_row), width=meta["width"],
               T_end=2 * st.ke / (cfg.d * (cfg.n - 1)))
    if st.step_kernels > 0:
        avg_ms = st.step_kernel_ms / st.step_kernels
        bpa = step_bytes_per_atom(cfg.d, meta["mean_row"], prec_mixed)
        ach = cfg.n * bpa / (avg_ms * 1e-3) / 1e9
        other = ms - st.step_kernel_ms - st.build_kernel_ms
        rec.update(step_kernel_ms=avg_ms, step_kernel_gbs=ach, step_bytes_per_atom=bpa,
                   step_kernels=int(st.step_kernels),
                   build_ms=(st.build_kernel_ms / st.build_kernels if st.build_kernels else None),
                   builds_per_s=(1e3 * st.build_kernels / st.build_kernel_ms
                                 if st.build_kernels else None),
                   build_candidates=meta["candidates"], build_variant=meta["build_variant"],
                   share_step_kernel=st.step_kernel_ms / ms,
                   share_build_kernel=st.build_kernel_ms / ms,
                   other_ms=other, share_other=other / ms)
    return rec


def run_long(H, torch, cfg, X0, V0, SIG, L, prec, steps, every, tau):
    """A run of `steps` steps in the library's production mode (captured
    chunks of steps replayed as graphs) after a warm-up call: wall-clock rate,
    builds, and the energy drift and fluctuation from thermo rows every
    `every` steps."""
    sysd = sized_width(H, torch, md_system(H, cfg, L, SIG.cpu().numpy(), prec, tau=tau), X0, V0,
                       SIG, cfg.dt)
    for attempt in range(4):
        X, V = X0.clone(), V0.clone()
        ws = H.workspace(sysd)
        try:
            H.hdmd_step(sysd, X, V, SIG, ws, 50, cfg.dt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, th = H.hdmd_step(sysd, X, V, SIG, ws, steps, cfg.dt, every, resume=True)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
        except H.HdmdError as e:
            if e.status != H.HDMD_ERR_NLIST_OVERFLOW:
                raise
            sysd.max_neighbors = int(sysd.max_neighbors * 1.5) + 16
            continue
        break
    th = th.cpu().numpy()
    sl, fl = drift(th, cfg.n, cfg.dt)
    return dict(steps=steps, value=cfg.n * steps / sec, ms_per_step=1e3 * sec / steps,
                builds=int(st.builds), steps_per_build=steps / max(st.builds, 1),
                drift_per_tau=sl, rms_fluct=fl, T_end=2 * st.ke / (cfg.d * (cfg.n - 1)),
                mode="captured graphs, wall clock")


def host_cpu():
    """Model name and thread counts of the host (lscpu), and the threads the
    OpenMP oracle uses."""
    info = {}
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket",
                             "Socket(s)", "CPU max MHz"):
                info[k.strip()] = v.strip()
    except Exception as e:  # lscpu missing
        info["error"] = str(e)
    info["omp_threads"] = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return info


def cpu_baseline(cfg, steps_per_build: float, n: int = 32768, reps: int = 5, runs: int = 3,
                 full_pairs: float = 3e9):
    """The oracle built with OpenMP (the paper's per-atom force loop and
    per-subcell list loop on all host threads), timed on the workload itself
    when its subcell path tests at most `full_pairs` candidate pairs per
    build (N times the atoms of the 3^d linked subcells), else on a bounded
    sample: `n` atoms at the same density and diameters, in a box of 3
    subcells per axis, so that the subcell path links every subcell and each
    atom meets n - 1 candidates.  Timed, median of `runs`: one list build by
    the oracle's subcell path, and `reps` force evaluations over that list.
    For the sample the build time per atom is scaled to the candidates per
    atom of the full box (3^d of its n_cell^d subcells: 46656 atoms for
    N = 262144 with n_cell = 4) -- the build is one plain loop per candidate.
    Per step the oracle costs N * (force time per atom) + N * (build time per
    atom) / steps_per_build, with the rebuild interval the GPU run measured."""
    from oracle import oracle as O
    from paper_2112_12271_amd import inputs
    sig_full = cfg.diameters()
    L_full = cfg.box(sig_full)
    rlmax = cfg.cutoff * float(sig_full.max()) + cfg.skin
    nc_full = O.ncell(L_full, rlmax)
    cand_full = cfg.n * (min(3, nc_full) / nc_full) ** cfg.d
    whole = cfg.n * cand_full <= full_pairs
    if whole:
        n, sig, L = cfg.n, sig_full, L_full
        x = cfg.positions(L)
    else:
        sig = (inputs.polydisperse(n, cfg.d, cfg.poly_R, 77) if cfg.poly_R > 0
               else inputs.bidisperse(n, cfg.sig_a, cfg.sig_b, 77))
        L = L_full * (n / cfg.n) ** (1.0 / cfg.d)  # the same number density
        x = inputs.uniform_positions(n, cfg.d, L, 78)
        if O.ncell(L, rlmax) != 3:
            log("cpu baseline skipped: the %d-atom sample of %s has %d subcells per axis, not 3"
                % (n, cfg.name, O.ncell(L, rlmax)))
            return None
    O.lib_omp()
    tb, tf = [], []
    for _ in range(runs):
        t0 = time.perf_counter()
        rp, cols = O.nlist_cells(x, sig, L, cfg.cutoff, cfg.skin, omp=True)
        tb.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        for _ in range(reps):
            O.forces(x, sig, L, cfg.potential, cfg.cutoff, 1.0, rp, cols, omp=True)
        tf.append((time.perf_counter() - t0) / reps)
    t_build, t_f = float(np.median(tb)), float(np.median(tf))
    log("cpu baseline: OpenMP oracle list build of %d atoms in %.2f s, force pass %.3f s"
        % (n, t_build, t_f))
    build_per_atom = t_build / n * (1.0 if whole else cand_full / (n - 1))
    step_s = cfg.n * (t_f / n) + cfg.n * build_per_atom / steps_per_build
    host = host_cpu()
    if whole:
        what = ("the workload itself (%d atoms, d=%d, %d subcells per axis, uniform positions)"
                % (n, cfg.d, nc_full))
    else:
        what = ("%d atoms (d=%d, same density, 3 subcells per axis; list build scaled from %d "
                "candidates per atom to the %.0f of N=%d)" % (n, cfg.d, n - 1, cand_full, cfg.n))
    return dict(value=cfg.n / step_s, unit="atom-steps/s", cores=host["omp_threads"],
                kind="oracle",
                sample="oracle FP64 built with -fopenmp, %d threads, on %s: subcell-path list "
                       "build %.3f s and force pass %.4f s (mean row %.1f), medians of %d runs, "
                       "combined at %.2f steps per build"
                       % (host["omp_threads"], what, t_build, t_f, len(cols) / n, runs,
                          steps_per_build),
                build_s_full=cfg.n * build_per_atom, force_s_full=cfg.n * t_f / n, host=host)


def fire_stream(count: int, rate: float, seed: int = 4000):
    """The batched FIRE workload: harmonic soft spheres, 50:50 diameters
    1.0/1.4, d uniform in {3,4,5,6}, N log-uniform in [256, 8192], packing
    fraction uniform in [phi_J - 0.02, phi_J + 0.05] with phi_J per d from the
    committed oracle pilot, Poisson arrivals at `rate` per second."""
    from paper_2112_12271_amd import inputs
    from paper_2112_12271_amd import serve as S
    pj = json.load(open(os.path.join(ROOT, "tests", "golden", "phij.json")))
    phij = {d: float(pj[str(d)]) for d in (3, 4, 5, 6)}
    return [S.Request(r.rid, "fire", r.d, r.n, r.L, r.positions(), r.sig, r.arrival)
            for r in inputs.fire_requests(count, phij, rate, seed=seed)]


def per_instance(H, torch, reqs, prec, f_tol, max_iter):
    """Plain per-instance solves: one hdmd_fire_minimize at a time, in arrival
    order, each with its own workspace (same row-capacity policy as the server:
    estimated, widened by 1.5x + 16 and re-run from the input on overflow)."""
    from paper_2112_12271_amd import serve as S
    params = H.hdmd_fire_defaults(0.05, f_tol, max_iter)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    out = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in sorted(reqs, key=lambda q: q.arrival):
        wait = r.arrival - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        width = S.estimate_width(r.d, r.n, r.box_l, r.cutoff * float(r.sig.max()) + r.skin)
        sig = dev(r.sig)
        while True:
            sysd = H.System(d=r.d, n=r.n, box_l=r.box_l, potential=H.HDMD_HARMONIC,
                            cutoff=1.0, skin=r.skin, sigma_max=float(r.sig.max()),
                            precision=prec, max_neighbors=width)
            ws = H.workspace(sysd)
            X = dev(r.x)
            try:
                res = H.hdmd_fire_minimize(sysd, X, sig, ws, params)
                break
            except H.HdmdError as e:
                if e.status != H.HDMD_ERR_NLIST_OVERFLOW:
                    raise
                width = int(width * 1.5) + 16
        now = time.perf_counter() - t0
        out.append(S.Result(r.rid, "fire", r.d, r.n, r.arrival, now, now, res.iterations,
                            res.fmax, res.energy, res.status, 0, None, res.builds))
    return out, time.perf_counter() - t0


def batched(H, torch, reqs, prec, f_tol, max_iter, slots, budget_gb, chunk):
    from paper_2112_12271_amd import serve as S
    params = H.hdmd_fire_defaults(0.05, f_tol, max_iter)
    ex = S.GpuExecutor(max_slots=slots, max_atoms=slots * 8192, max_cells=slots * 32768,
                       precision=prec, fire_params=params)
    srv = S.Server(ex, max_slots=slots, hbm_budget=int(budget_gb * (1 << 30)), chunk=chunk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = srv.serve(reqs, time_limit=900)
    torch.cuda.synchronize()
    return res, time.perf_counter() - t0, srv


def fire_record(res, wall):
    from paper_2112_12271_amd import serve as S
    rec = S.summarize(res, wall)
    f = np.array([r.fmax for r in res])
    rec.update(converged=int(sum(r.status == 0 for r in res)),
               fmax_final_max=float(f.max()) if len(f) else None,
               iterations_total=int(sum(r.iterations for r in res)),
               iterations_max=int(max((r.iterations for r in res), default=0)),
               builds_total=int(sum(r.builds for r in res)),
               atoms_total=int(sum(r.n for r in res)))
    return rec


def swap_leg(H, torch, cfg, x, sig, L, m):
    """SWAP Monte Carlo (Sec. II.D) on the relaxed MD state: m attempts on
    seeded random pairs at the run's temperature, with the outcome of the
    serial walk the method defines (batches of attempts, settled in order);
    attempts per second."""
    g = np.random.default_rng(7)
    pairs = torch.as_tensor(g.integers(0, cfg.n, size=(m, 2)).astype(np.int32), device="cuda")
    u = torch.as_tensor(g.uniform(size=m), dtype=torch.float64, device="cuda")
    X = torch.as_tensor(x, dtype=torch.float64, device="cuda")
    s = H.System(d=cfg.d, n=cfg.n, box_l=L, potential=cfg.potential, cutoff=cfg.cutoff,
                 skin=cfg.skin, sigma_max=float(sig.max()))
    s, ws = H.build_with_width(s, X, torch.as_tensor(sig, dtype=torch.float64, device="cuda"))
    D = torch.as_tensor(sig, dtype=torch.float64, device="cuda")
    H.hdmd_swap(s, X, D.clone(), ws, pairs[:16], u[:16], cfg.T)   # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, na = H.hdmd_swap(s, X, D, ws, pairs, u, cfg.T)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t
    return {"attempts": m, "accepted": na, "seconds": sec, "attempts_per_s": m / sec,
            "temperature": cfg.T, "note": "wall time of hdmd_swap, including its list build"}


def fire_serving(H, torch, args):
    """Batched mixed-precision FIRE over the whole request stream through the
    continuous-batching server, then the comparison at equal final |F|max on a
    bounded prefix of the same stream: batched mixed vs plain per-instance FP64
    (one minimisation at a time, the only way to serve without batching)."""
    reqs = fire_stream(args.fire_requests, args.fire_rate)
    log("fire stream: %d requests, %d atoms, arrivals over %.2f s"
        % (len(reqs), sum(r.n for r in reqs), reqs[-1].arrival if reqs else 0))
    out = {"f_tol": args.fire_tol, "requests": len(reqs), "arrival_rate_per_s": args.fire_rate}

    def run_batched(rs, prec=H.HDMD_MIXED, f_tol=args.fire_tol):
        res, wall, srv = batched(H, torch, rs, prec, f_tol, args.fire_max_iter,
                                 args.fire_slots, args.fire_budget_gb, args.fire_chunk)
        rec = fire_record(res, wall)
        rec.update(precision="mixed" if prec == H.HDMD_MIXED else "fp64", f_tol=f_tol,
                   slots=args.fire_slots, max_active=srv.max_active,
                   peak_workspace_gb=srv.max_in_use / (1 << 30), budget_gb=args.fire_budget_gb,
                   footprint_gb=stream_footprint(H, rs, prec) / (1 << 30),
                   retries=int(sum(r.retries for r in res)))
        return rec

    out["batched_mixed"] = run_batched(reqs)
    log("batched mixed", json.dumps(out["batched_mixed"]))
    k = min(args.fire_compare, len(reqs))
    if k > 0:
        pre = reqs[:k]
        a = run_batched(pre)
        res, wall = per_instance(H, torch, pre, H.HDMD_FP64, args.fire_tol, args.fire_max_iter)
        b = fire_record(res, wall)
        b.update(precision="fp64")
        out["compare"] = {"requests": k, "batched_mixed": a, "per_instance_fp64": b,
                          "speedup_solves_per_s": a["solves_per_s"] / b["solves_per_s"],
                          "p99_ratio_per_instance_over_batched":
                              b["latency_p99"] / a["latency_p99"]}
        log("compare", json.dumps(out["compare"]))
        if args.fire_tight_tol > 0:
            # the FP64 leg of the workload: |F|max < 1e-10, batched, same prefix
            out["batched_fp64_tight"] = run_batched(pre, H.HDMD_FP64, args.fire_tight_tol)
            log("batched fp64 tight", json.dumps(out["batched_fp64_tight"]))
    return out


def stream_footprint(H, reqs, prec) -> int:
    """Device bytes the whole stream would hold at once (every request's
    workspace at its estimated row capacity, plus its positions): what an
    HBM budget below it has to ration."""
    from paper_2112_12271_amd import serve as S
    tot = 0
    for r in reqs:
        w = S.estimate_width(r.d, r.n, r.box_l, r.cutoff * float(r.sig.max()) + r.skin)
        sysd = H.System(d=r.d, n=r.n, box_l=r.box_l, potential=H.HDMD_HARMONIC, cutoff=1.0,
                        skin=r.skin, sigma_max=float(r.sig.max()), precision=prec,
                        max_neighbors=w)
        tot += H.hdmd_workspace_bytes(sysd) + r.n * (r.d + 1) * 8 * 2
    return tot


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="K: steps of each timed window")
    ap.add_argument("--warmup", type=int, default=50, help="W: untimed steps before the windows")
    ap.add_argument("--windows", type=int, default=3, help="timed windows (median reported)")
    ap.add_argument("--config", default="c3")
    ap.add_argument("--pushoff-iters", type=int, default=1500)
    ap.add_argument("--equil-steps", type=int, default=1000,
                    help="untimed FP64 steps after the pushoff and velocity draw")
    ap.add_argument("--long-steps", type=int, default=10000,
                    help="steps of the production-mode run per precision (0: skip)")
    ap.add_argument("--thermostat-tau", type=float, default=None,
                    help="Berendsen time constant of the MD legs (default: NVE, except 1.0 "
                         "for the paper's state point p6, NVT at its T)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="time with captured graphs and without per-kernel events")
    ap.add_argument("--no-fire", action="store_true", help="skip the batched FIRE serving leg")
    ap.add_argument("--fire-compare", type=int, default=64,
                    help="prefix of the stream run both batched and per instance (0: skip)")
    ap.add_argument("--fire-requests", type=int, default=512)
    ap.add_argument("--fire-rate", type=float, default=200.0, help="Poisson arrivals per second")
    ap.add_argument("--fire-tol", type=float, default=1e-5, help="|F|max target of both legs")
    ap.add_argument("--fire-tight-tol", type=float, default=1e-10,
                    help="|F|max target of the batched FP64 leg on the prefix (0: skip)")
    ap.add_argument("--fire-max-iter", type=int, default=100000)
    ap.add_argument("--fire-slots", type=int, default=512)
    ap.add_argument("--fire-budget-gb", type=float, default=0.5,
                    help="HBM budget of the server's admission (below the stream's footprint)")
    ap.add_argument("--fire-chunk", type=int, default=50)
    ap.add_argument("--no-md", action="store_true", help="skip the MD legs (FIRE serving only)")
    ap.add_argument("--swap-attempts", type=int, default=20000,
                    help="SWAP Monte Carlo attempts timed on the relaxed MD state (0: skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES three times (scales the HBM "
                         "byte counters of a profiler to bytes)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(args.calibrate_copy // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8,
                          "launches": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(the design notes say how it would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2112_12271_amd import hdmd as H
    from paper_2112_12271_amd import inputs

    cfg = inputs.CONFIGS[args.config]
    tau = args.thermostat_tau if args.thermostat_tau is not None else (
        1.0 if args.config == "p6" else 0.0)
    torch.cuda.set_device(0)
    H.lib()
    sig = cfg.diameters()
    L = cfg.box(sig)
    x0 = cfg.positions(L)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")

    out = {}
    setup = {}
    if not args.no_md:
        # untimed set-up: FIRE pushoff of the overlaps on harmonic soft spheres
        t = time.perf_counter()
        sysh = H.System(d=cfg.d, n=cfg.n, box_l=L, potential=H.HDMD_HARMONIC, cutoff=1.0,
                        skin=cfg.skin, sigma_max=float(sig.max()), max_neighbors=64)
        X = dev(x0)
        sysh, res = H.fire_auto(sysh, X, dev(sig),
                                H.hdmd_fire_defaults(0.05, 1e-6, args.pushoff_iters))
        log("pushoff: %d FIRE iterations, %d builds, E/N=%.4g, |F|max=%.3g, %.1fs"
            % (res.iterations, res.builds, res.energy / cfg.n, res.fmax, time.perf_counter() - t))
        SIG = dev(sig)
        V = dev(cfg.velocities())
        setup["pushoff_iterations"] = int(res.iterations)
        if args.equil_steps > 0:
            # untimed equilibration in FP64 (the heating right after the pushoff)
            t = time.perf_counter()
            se = md_system(H, cfg, L, sig, H.HDMD_FP64, tau=tau)
            se, st, _ = H.step_auto(se, X, V, SIG, args.equil_steps, cfg.dt)
            setup.update(equil_steps=args.equil_steps, equil_builds=int(st.builds),
                         T_after_equil=2 * st.ke / (cfg.d * (cfg.n - 1)))
            log("equilibration: %d steps, %d builds, T=%.3f, %.1fs"
                % (args.equil_steps, st.builds, setup["T_after_equil"], time.perf_counter() - t))
        xr = X.cpu().numpy()

        for prec in ([H.HDMD_FP64] + ([] if args.no_mixed else [H.HDMD_MIXED])):
            name = "fp64" if prec == H.HDMD_FP64 else "mixed"
            win, meta = run_windows(H, torch, cfg, X, V, SIG, L, prec, args.steps, args.warmup,
                                    args.windows, 0, not args.no_profile, tau)
            rec = window_record(cfg, prec == H.HDMD_MIXED, win, meta, args.steps)
            if args.long_steps > 0:
                rec["long_run"] = run_long(H, torch, cfg, X, V, SIG, L, prec, args.long_steps,
                                           10, tau)
            out[name] = rec
            log(name, json.dumps(rec))
        if args.swap_attempts > 0:
            out["swap"] = swap_leg(H, torch, cfg, xr, sig, L, args.swap_attempts)
            log("swap", json.dumps(out["swap"]))
    fire = None
    if not args.no_fire:
        fire = fire_serving(H, torch, args)
    f = out.get("fp64", {})
    roof = None
    if "step_kernel_ms" in f:
        roof = {"bound": "hbm", "achieved": f["step_kernel_gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": f["step_kernel_gbs"] / HBM_PEAK_GBS,
                "traffic": committed_traffic("step_kernel_c3_traffic.json"),
                "kernel": "k_step<6,fp64>", "bytes_per_launch": cfg.n * f["step_bytes_per_atom"],
                "launch_ms": f["step_kernel_ms"]}
    # the list build as a candidate rate against the vector ALU peak: every
    # candidate pair of the subcell stencil (Sec. II.C) is priced at the
    # vector prefilter's cost, ceil(d/2) packed int16 dot products and a
    # compare, one VALU lane-operation each; the peak is 256 CUs x 4 SIMDs x
    # 16 lanes x 2.4 GHz lane-operations per second.  (Row culling skips most
    # candidates before any test, and the matrix-core variant runs the tests
    # it does make as f16 products, so this is a rate, not the kernel's own
    # VALU use.)
    roof_build = None
    if f.get("build_ms") and f.get("build_candidates"):
        ops = (cfg.d + 1) // 2 + 1
        ach = f["build_candidates"] * ops / (f["build_ms"] * 1e-3)
        roof_build = {"bound": "alu", "achieved": ach, "peak": VALU_LANE_OPS_PEAK,
                      "unit": "lane-op/s", "frac": ach / VALU_LANE_OPS_PEAK,
                      "kernel": build_kernel_name(cfg.d, f.get("build_variant", 1)),
                      "candidates_per_build": f["build_candidates"],
                      "candidates_per_s": f["build_candidates"] / (f["build_ms"] * 1e-3),
                      "launch_ms": f["build_ms"], "lane_ops_per_candidate": ops}
    cpu = None
    if not args.no_cpu_baseline and not args.no_md:
        spb = f.get("long_run", f)["steps_per_build"]
        cpu = cpu_baseline(cfg, spb)
        log("cpu baseline", json.dumps(cpu))
    lr = {k: out[k].get("long_run") for k in ("fp64", "mixed") if k in out}
    line = {
        "metric": "atom-steps/s at d=6,N=262144; batched FIRE solves/s + p50/p99 latency",
        "value": f.get("value"),
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f.get("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded uniform positions relaxed by harmonic FIRE, Gaussian T=1, "
                "untimed equilibration)",
        "config": {"workload": workload_name(cfg), "precision": "fp64",
                   "ensemble": "NVT Berendsen tau=%g" % tau if tau > 0 else "NVE",
                   "timed": "median of %d windows of K steps, kernels launched one by one with "
                            "HIP events" % args.windows if not args.no_profile else
                            "median of %d windows of K steps, captured graphs" % args.windows},
        "setup": setup,
        "roofline": roof,
        "roofline_build": roof_build,
        "cpu_baseline": cpu,
        "fp64": out.get("fp64"),
        "mixed": out.get("mixed"),
        "mixed_form": "neighbour positions gathered as 32-bit fixed point, stored forces and "
                      "velocities FP32; distances, pair coefficients, force sums, positions and "
                      "energy sums FP64 (FP32 distances and forces exceed 1e-5 F_rms)",
        "drift_difference_mixed_minus_fp64":
            (lr["mixed"]["drift_per_tau"] - lr["fp64"]["drift_per_tau"])
            if lr.get("mixed") and lr.get("fp64") else None,
        "fire_serving": fire,
        "swap": out.get("swap"),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
