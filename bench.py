#!/usr/bin/env python3
"""Benchmark: SSP-RK3 steps of the five-equation finite-volume solver on one
MI355X, 256^3 Mach-2 shock-droplet workload, FP64 path.

One step = three right-hand-side evaluations (x, y, z sweeps each) plus the
stage updates and the CFL reduction, on a state already resident in HBM.
Prints one JSON line:
  value        grind time, ns per cell per RK stage (lower is better)
  roofline     the dominant kernel's algorithmic bytes per launch over its
               mean HIP-event duration, against 8 TB/s HBM
  cpu_baseline the FP64 CPU oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grind time (ns/cell/RK-stage) + %HBM peak; FP32/learned vs FP64 at fixed L1"
HBM_PEAK_GBS = 8000.0
STATE_BYTES = 56  # 7 float64 per cell
KERNEL_NAMES = {0: "sweep_fp64<0>", 1: "sweep_fp64<1>", 2: "sweep_fp64<2>"}


def sweep_bytes_per_cell(first: int, mode: int) -> int:
    """Algorithmic HBM bytes per cell of one sweep launch: read the stage state
    (stencil and, for the stage update, the same cells again: counted once),
    read the partial RHS unless first, write the partial RHS / caller RHS /
    new state, and read the step's initial state in stages 2 and 3."""
    b = STATE_BYTES  # stage state
    if not first:
        b += STATE_BYTES  # partial RHS in
    b += STATE_BYTES  # output
    if mode in (3, 4):
        b += STATE_BYTES  # q^n for the RK combination
    return b


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2409_10729_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != source_hash():
        return None
    return t.get("kernels", {}).get(kernel)


def cpu_baseline(P, q0_np, budget_s: float):
    """Oracle (plain FP64 C, OpenMP) timed on the host: one SSP-RK3 step of
    the same state, on an x-slab of the grid sized to the time budget."""
    import numpy as np

    import oracle

    nx, ny, nz = P["spec"]["n"]
    threads = oracle.max_threads()
    # probe on a thin slab to size the sample
    def slab(k):
        spec = dict(P["spec"])
        spec["n"] = (nx, ny, k)
        spec["bc"] = (P["spec"]["bc"][0], P["spec"]["bc"][1], (0, 0))
        g = oracle.make_grid(spec)
        q = np.ascontiguousarray(q0_np[:, :k])
        return g, q

    g, q = slab(4)
    t0 = time.perf_counter()
    oracle.rk3_step(g, q)
    per_cell = (time.perf_counter() - t0) / (nx * ny * 4 * 3)
    k = int(max(4, min(nz, budget_s / max(per_cell * nx * ny * 3, 1e-12))))
    g, q = slab(k)
    t0 = time.perf_counter()
    oracle.rk3_step(g, q)
    dt = time.perf_counter() - t0
    cells = nx * ny * k
    return {
        "value": dt * 1e9 / (cells * 3),
        "unit": "ns/cell/RK-stage",
        "cores": threads,
        "kind": "oracle",
        "sample": f"one SSP-RK3 step of the first {k} z-planes ({nx}x{ny}x{k} = {cells} cells, "
                  f"z periodic) of the same initial state; {dt:.1f} s wall",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256, help="cells per direction")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device-to-device copy of 7 * n^3 float64 (known bytes), five times, "
                         "to scale rocprofv3 FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU halo exchange is a design note, not code)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2409_10729_amd import Solver
    from paper_2409_10729_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.ones(7 * args.n ** 3, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 8, "launches": 5}), flush=True)
        return
    print(f"[bench] generating shock_droplet n={args.n} seed={args.seed}", file=sys.stderr, flush=True)
    P = wl.shock_droplet(n=args.n, seed=args.seed)
    N = args.n ** 3
    w_dev = torch.from_numpy(P["w"]).cuda()
    s = Solver(P["spec"])
    s.set_primitive(w_dev)
    del w_dev
    stream = s.stream

    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        s.rk3_step()
    torch.cuda.synchronize()

    s.profile(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        s.rk3_step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    prof = s.profile_read()
    s.profile(False)
    st = s.stats()
    if st["status"] != 0:
        raise RuntimeError(f"solver flagged a non-physical state: {st}")
    ms_step = ms_total / args.steps
    grind = ms_step * 1e6 / (N * 3)
    print(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step, {grind:.4f} ns/cell/stage", file=sys.stderr,
          flush=True)

    # per-kernel: algorithmic bytes / mean event duration
    per_dir = {}
    for (d, first, mode), (ms, cnt) in prof.items():
        b = sweep_bytes_per_cell(first, mode) * N
        e = per_dir.setdefault(d, {"ms": 0.0, "launches": 0, "bytes": 0})
        e["ms"] += ms
        e["launches"] += cnt
        e["bytes"] += b * cnt
    kernels = {}
    for d, e in sorted(per_dir.items()):
        mean_ms = e["ms"] / e["launches"]
        bytes_per_launch = e["bytes"] / e["launches"]
        kernels[KERNEL_NAMES[d]] = {
            "mean_us": mean_ms * 1e3,
            "launches": e["launches"],
            "share": e["ms"] / ms_total,
            "alg_bytes_per_launch": bytes_per_launch,
            "achieved_GBs": bytes_per_launch / (mean_ms * 1e-3) / 1e9,
        }
    dom = max(kernels, key=lambda k: kernels[k]["mean_us"] * kernels[k]["launches"])
    kd = kernels[dom]
    traffic = load_traffic(dom)
    step_bytes = sum(e["bytes"] for e in per_dir.values()) / args.steps
    roofline = {
        "bound": "hbm",
        "achieved": round(kd["achieved_GBs"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(kd["achieved_GBs"] / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": dom,
        "mean_us": round(kd["mean_us"], 2),
        "alg_bytes_per_launch": kd["alg_bytes_per_launch"],
    }

    out = {
        "metric": METRIC,
        "value": round(grind, 5),
        "unit": "ns/cell/RK-stage",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"shock_droplet {args.n}^3: Mach-2 air shock on a water droplet (R=0.15), 1% density "
                        f"noise, x transmissive / y,z periodic, CFL 0.4, WENO5-JS + HLLC + SSP-RK3, FP64",
            "cells": N,
            "seed": args.seed,
            "precision": "fp64",
        },
        "grind_ns_per_cell_pde_rhs": round(grind / 7, 6),
        "step_alg_bytes_hbm_frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "kernels": kernels,
        "roofline": roofline,
    }
    if not args.no_cpu:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        import oracle

        q_ic = oracle.prim_to_cons(oracle.make_grid(P["spec"]), P["w"])
        cb = cpu_baseline(P, q_ic, args.cpu_budget)
        out["cpu_baseline"] = cb
        out["gpu_over_cpu"] = round(cb["value"] / grind, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
