#!/usr/bin/env python
"""Throughput of the hdMD hot path on one MI355X.

One step = one pass of the whole hot path over the system: the fused
velocity-Verlet kernel (forces, kicks, drift, rebuild trigger) and, when the
largest displacement since the last build exceeds skin/2, the subcell binning,
counting sort and Verlet-list rebuild.

Workload (default): d=6, N=262144, 50:50 WCA mixture sigma 1.0/1.2 at packing
fraction 0.42, dt=0.002, skin 0.25, T=1.0.  Seeded uniform positions are relaxed
by FIRE on harmonic soft spheres (on the GPU, untimed), Gaussian velocities at
T=1 are drawn, then W warm-up steps and K timed steps run, in FP64 and in the
mixed form (FP32 forces/velocities, FP64 positions and sums).

Prints one JSON line.  `value` is atom-steps/s of the FP64 run with inputs
resident in HBM.  `roofline` is the fused-step kernel's algorithmic bytes per
launch (SURVEY-defined per-atom bytes times N) over its mean
duration measured with HIP events inside the timed region.  `cpu_baseline` is
the plain oracle on the host, on a bounded sample described in the line.
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def step_bytes_per_atom(d: int, mean_row: float, mixed: bool) -> float:
    """Compulsory bytes of one fused step per atom: read x (8d), write x (8d),
    read x_ref (8d), read+write v (2 b_v d), the row (4 per entry), row length
    (4) and own diameter (8).  Gathered neighbour data is not counted."""
    bv = 4 if mixed else 8
    return 8 * d * 3 + 2 * bv * d + 4 * mean_row + 4 + 8


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


def run_md(H, torch, cfg, x0, v0, sig, L, prec, steps, warmup, every, profile):
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    sysd = H.System(d=cfg.d, n=cfg.n, box_l=L, cutoff=cfg.cutoff, skin=cfg.skin,
                    sigma_max=float(sig.max()), precision=prec, max_neighbors=64)
    X, V, SIG = dev(x0), dev(v0), dev(sig)
    sysd, _, _ = H.step_auto(sysd, X, V, SIG, max(warmup, 1), cfg.dt)   # warm-up (sizes the rows)
    ws = H.workspace(sysd)
    if profile:
        os.environ["HDMD_PROFILE"] = "1"
    else:
        os.environ.pop("HDMD_PROFILE", None)
    for attempt in range(4):
        Xs, Vs = X.clone(), V.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            st, th = H.hdmd_step(sysd, Xs, Vs, SIG, ws, steps, cfg.dt, every)
        except H.HdmdError as e:
            if e.status != H.HDMD_ERR_NLIST_OVERFLOW:
                raise
            sysd.max_neighbors = int(sysd.max_neighbors * 1.5) + 16
            ws = H.workspace(sysd)
            continue
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        break
    os.environ.pop("HDMD_PROFILE", None)
    rp, cols = H.hdmd_nlist_export(sysd, ws)
    mean_row = cols.numel() / cfg.n
    return dict(seconds=t1 - t0, stats=st, thermo=th.cpu().numpy(), mean_row=mean_row,
                width=sysd.max_neighbors)


def cpu_baseline(cfg, steps: int = 10):
    """Oracle (single thread) on a bounded sample of the same workload: d=6,
    phi=0.42, 50:50 sigma 1.0/1.2, dt, skin, T as the GPU run, but 6^6 = 46656
    atoms in a box of exactly 3 subcells per axis, so that every atom meets the
    same number of candidates (its 3^6 linked subcells at the same density)
    and has the same list length as in the 262144-atom box; one list build and
    `steps` velocity-Verlet steps from a jittered lattice."""
    from oracle import oracle as O
    from paper_2112_12271_amd import inputs
    m = 6
    n = m ** cfg.d
    sig = inputs.bidisperse(n, cfg.sig_a, cfg.sig_b, 77)
    L = inputs.box_for_packing(cfg.d, sig, cfg.phi)
    x, Lq = inputs.jittered_lattice(cfg.d, m, L / m, 0.15 * L / m, 78)
    v = inputs.gaussian_velocities(n, cfg.d, cfg.T, 79)
    O.lib()
    t0 = time.perf_counter()
    _, _, th, builds = O.vv(x, v, sig, Lq, O.WCA, cfg.cutoff, cfg.skin, 1.0, steps, cfg.dt)
    t1 = time.perf_counter()
    return dict(value=n * steps / (t1 - t0), unit="atom-steps/s", cores=1, kind="oracle",
                sample="oracle FP64, 1 thread: %d atoms, d=%d, phi=%.2f, box of 3 subcells per axis "
                       "(same candidates per atom as N=%d), %d list build(s) + %d VV steps in %.1f s"
                       % (n, cfg.d, cfg.phi, cfg.n, builds, steps, t1 - t0),
                steps_per_build=steps / max(builds, 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--pushoff-iters", type=int, default=1500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="time with captured graphs and without per-kernel events")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(see DESIGN.md for how it would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2112_12271_amd import hdmd as H
    from paper_2112_12271_amd import inputs

    cfg = inputs.CONFIGS[args.config]
    torch.cuda.set_device(0)
    H.lib()
    sig = cfg.diameters()
    L = cfg.box(sig)
    x0 = cfg.positions(L)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")

    # untimed set-up: FIRE pushoff of the overlaps on harmonic soft spheres
    t = time.perf_counter()
    sysh = H.System(d=cfg.d, n=cfg.n, box_l=L, potential=H.HDMD_HARMONIC, cutoff=1.0,
                    skin=cfg.skin, sigma_max=float(sig.max()), max_neighbors=64)
    X = dev(x0)
    sysh, res = H.fire_auto(sysh, X, dev(sig),
                            H.hdmd_fire_defaults(0.05, 1e-6, args.pushoff_iters))
    xr = X.cpu().numpy()
    log("pushoff: %d FIRE iterations, %d builds, E/N=%.4g, |F|max=%.3g, %.1fs"
        % (res.iterations, res.builds, res.energy / cfg.n, res.fmax, time.perf_counter() - t))
    v0 = cfg.velocities()

    out = {}
    for prec in ([H.HDMD_FP64] + ([] if args.no_mixed else [H.HDMD_MIXED])):
        name = "fp64" if prec == H.HDMD_FP64 else "mixed"
        r = run_md(H, torch, cfg, xr, v0, sig, L, prec, args.steps, args.warmup, 10,
                   not args.no_profile)
        st = r["stats"]
        sl, fl = drift(r["thermo"], cfg.n, cfg.dt)
        rate = cfg.n * args.steps / r["seconds"]
        rec = dict(value=rate, ms_per_step=1e3 * r["seconds"] / args.steps, builds=int(st.builds),
                   steps_per_build=args.steps / max(st.builds, 1), mean_row=r["mean_row"],
                   max_row=int(st.max_row), width=r["width"], drift_per_tau=sl, rms_fluct=fl,
                   T_end=2 * st.ke / (cfg.d * (cfg.n - 1)))
        if st.step_kernels > 0:
            avg_ms = st.step_kernel_ms / st.step_kernels
            bpa = step_bytes_per_atom(cfg.d, r["mean_row"], prec == H.HDMD_MIXED)
            ach = cfg.n * bpa / (avg_ms * 1e-3) / 1e9
            rec.update(step_kernel_ms=avg_ms, step_kernel_gbs=ach, step_bytes_per_atom=bpa,
                       build_ms=(st.build_kernel_ms / st.build_kernels if st.build_kernels else None),
                       share_step_kernel=st.step_kernel_ms / (1e3 * r["seconds"]),
                       share_build_kernel=st.build_kernel_ms / (1e3 * r["seconds"]))
        out[name] = rec
        log(name, json.dumps(rec))

    f = out["fp64"]
    roof = None
    if "step_kernel_ms" in f:
        roof = {"bound": "hbm", "achieved": f["step_kernel_gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": f["step_kernel_gbs"] / HBM_PEAK_GBS,
                "traffic": committed_traffic("step_kernel_c3_traffic.json"),
                "kernel": "k_step<6,fp64>", "bytes_per_launch": cfg.n * f["step_bytes_per_atom"],
                "launch_ms": f["step_kernel_ms"]}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg)
        log("cpu baseline", json.dumps(cpu))
    line = {
        "metric": "atom-steps/s at d=6,N=262144",
        "value": f["value"],
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded uniform positions relaxed by harmonic FIRE, Gaussian T=1)",
        "config": {"workload": "%s: d=%d N=%d 50:50 WCA sigma %.1f/%.1f phi=%.2f dt=%g skin=%g T=%g"
                               % (cfg.name, cfg.d, cfg.n, cfg.sig_a, cfg.sig_b, cfg.phi, cfg.dt,
                                  cfg.skin, cfg.T),
                   "precision": "fp64", "timed_with_events": not args.no_profile},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64": out.get("fp64"),
        "mixed": out.get("mixed"),
        "drift_difference_mixed_minus_fp64": (out["mixed"]["drift_per_tau"] - f["drift_per_tau"])
        if "mixed" in out else None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
