#!/usr/bin/env python3
"""Benchmark: SSP-RK3 steps of the five-equation finite-volume solver on one
MI355X, 256^3 Mach-2 shock-droplet workload, FP64 path (other synthetic
workloads with --workload).

One step = three right-hand-side evaluations (each a fused x-y pass and a z
pass) plus the stage updates and the CFL reduction, on a state already
resident in HBM.  Prints one JSON line:
  value        grind time, ns per cell per RK stage (lower is better)
  roofline     the dominant kernel against the roof its arithmetic intensity
               selects: algorithmic float64 flops per launch over its mean
               HIP-event duration against 78.6 TFLOP/s, or algorithmic bytes
               against 8 TB/s HBM
  cpu_baseline the FP64 CPU oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grind time (ns/cell/RK-stage) + %HBM peak; FP32/learned vs FP64 at fixed L1"
HBM_PEAK_GBS = 8000.0
STATE_BYTES = 56  # 7 float64 per cell
KERNEL_NAMES = {0: "sweep_x", 1: "sweep_y", 2: "sweep_z", 3: "sweep_xy"}
# synthetic workloads: description, default cells per direction
WORKLOADS = {
    "shock_droplet": ("Mach-2 air shock on a water droplet (R=0.15), 1% density noise, x transmissive / y,z "
                      "periodic", 256),
    "bubble_cloud": ("Mach-1.5 water shock on 4-16 seeded air bubbles (R 0.05-0.15), x transmissive / y,z "
                     "periodic", 192),
    "droplet_cloud": ("Mach-2 air shock on 32 seeded water droplets (R log-uniform 0.02-0.1), 1% density noise, "
                      "x transmissive / y,z periodic", 384),
    "advected_bubble": ("air bubble advected through water at u=(1,0.5,0.25), periodic", 128),
    "shock_droplet_walls": ("Mach-2 air shock on a water droplet (R=0.15), 1% density noise, x inflow at the "
                            "post-shock state / transmissive, y,z reflective walls", 256),
    "droplet_bubble": ("three fluids: Mach-2 air shock on a water droplet (R=0.15) and a helium bubble "
                       "(R=0.08), 1% density noise, x transmissive / y,z periodic", 256),
    "shock_droplet_stretched": ("Mach-2 air shock on a water droplet (R=0.15), 1% density noise, on cells refined "
                                "around the droplet (tanh stretching, up to 2x finer), x transmissive / y,z "
                                "periodic", 256),
}


def sweep_bytes_per_cell(first: int, mode: int, rhs_bytes: int = STATE_BYTES, state_bytes: int = STATE_BYTES) -> int:
    """Algorithmic HBM bytes per cell of one sweep launch: read the stage state
    (stencil and, for the stage update, the same cells again: counted once),
    read the partial RHS unless first, write the partial RHS / caller RHS /
    new state, and read the step's initial state in stages 2 and 3.
    rhs_bytes is the partial-RHS size per cell (56 in FP64, 28 in FP32 for
    two fluids); state_bytes the state's (8 per variable)."""
    b = state_bytes  # stage state
    if not first:
        b += rhs_bytes  # partial RHS in
    b += rhs_bytes if mode == 0 else state_bytes  # output
    if mode in (3, 4):
        b += state_bytes  # q^n for the RK combination
    return b


# Algorithmic float64 operations per cell (+, -, *, /, sqrt, min, max each
# one; constants such as 13/12 and the per-fluid 1/(gamma-1) precomputed;
# a value the formulas use twice counted once), from the definitions:
# conserved -> primitive 21; WENO5 with Jiang-Shu weights, both edges of one
# variable: indicators 33, right edge 35, left edge 29 (its (eps + beta)^2
# shared) = 97; HLLC with Davis speeds, one face: 120; flux difference,
# alpha1 source and accumulation 25; the RK stage combination 2 (stage 1) or
# 5 (stages 2, 3) per variable.  WENO3 (Jiang-Shu), one variable, both
# edges: indicators 4, right edge 18, left edge 14 = 36.
FLOPS_CONV = 21
FLOPS_WENO_VAR = 97
FLOPS_WENO3_VAR = 36
FLOPS_HLLC = 120
FLOPS_FLUXDIFF = 25
FLOPS_RK = {0: 0, 1: 0, 2: 14, 3: 35, 4: 35}
FP64_PEAK_TFLOPS = 78.6  # MI355X float64 vector peak (FMA = 2 flops)


def sweep_flops_per_cell(d: int, mode: int, order: int = 5) -> int:
    """Algorithmic float64 flops per cell of one launch of pass d (3 = the
    fused x-y pass: both directions, one conversion)."""
    ndir = 2 if d == 3 else 1
    weno = FLOPS_WENO_VAR if order == 5 else FLOPS_WENO3_VAR
    return FLOPS_CONV + ndir * (7 * weno + FLOPS_HLLC + FLOPS_FLUXDIFF) + FLOPS_RK[mode]


def code_of(text: str) -> str:
    """C++ source without comments and blank lines."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def source_hash() -> str:
    """Hash of the kernel sources' code (comments and blank lines left out:
    a comment edit does not change what the counters measured)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2409_10729_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            h.update(name.encode())
            h.update(code_of(f.read()).encode())
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


def _host_cpus():
    """Logical CPUs of the host, the ones this process may run on, and the
    CPU model (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = None
    return os.cpu_count(), allowed, model


def cpu_baseline(P, q0_np, budget_s: float):
    """Oracle (plain FP64 C, OpenMP over pencils) timed on the host: one
    SSP-RK3 step of the same state, on an x-slab of the grid sized to the
    time budget, with every thread OpenMP runs and again on one thread (a
    smaller slab)."""
    import numpy as np

    import oracle

    nx, ny, nz = P["spec"]["n"]

    def slab(k):
        spec = dict(P["spec"])
        spec["n"] = (nx, ny, k)
        spec["bc"] = (P["spec"]["bc"][0], P["spec"]["bc"][1], (0, 0))
        if spec.get("faces") is not None and spec["faces"][2] is not None:  # unequal cells: the slab's z faces
            spec["faces"] = (spec["faces"][0], spec["faces"][1], np.asarray(spec["faces"][2])[:k + 1])
        g = oracle.make_grid(spec)
        q = np.ascontiguousarray(q0_np[:, :k])
        return g, q

    def timed(budget):
        # probe on a thin slab to size the sample
        g, q = slab(4)
        t0 = time.perf_counter()
        oracle.rk3_step(g, q)
        per_cell = (time.perf_counter() - t0) / (nx * ny * 4 * 3)
        k = int(max(4, min(nz, budget / max(per_cell * nx * ny * 3, 1e-12))))
        g, q = slab(k)
        t0 = time.perf_counter()
        oracle.rk3_step(g, q)
        dt = time.perf_counter() - t0
        return dt, k

    cpus, allowed, model = _host_cpus()
    threads = oracle.team_size()
    dt, k = timed(budget_s)
    cells = nx * ny * k
    oracle.set_threads(1)
    try:
        dt1, k1 = timed(max(2.0, budget_s / 3))
    finally:
        oracle.set_threads(threads)
    cells1 = nx * ny * k1
    return {
        "value": dt * 1e9 / (cells * 3),
        "unit": "ns/cell/RK-stage",
        "cores": threads,
        "kind": "oracle",
        "sample": f"one SSP-RK3 step of the first {k} z-planes ({nx}x{ny}x{k} = {cells} cells, "
                  f"z periodic) of the same initial state on {threads} OpenMP threads; {dt:.1f} s wall",
        "host_cpus": cpus,
        "cpus_allowed": allowed,
        "cpu_model": model,
        "single_thread": {
            "value": dt1 * 1e9 / (cells1 * 3),
            "unit": "ns/cell/RK-stage",
            "sample": f"one SSP-RK3 step of the first {k1} z-planes ({cells1} cells) on 1 thread; "
                      f"{dt1:.1f} s wall",
        },
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="shock_droplet",
                    help="synthetic 3D problem (the headline line is shock_droplet at 256^3)")
    ap.add_argument("--n", type=int, default=None, help="cells per direction (default: the workload's size)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--compare-steps", type=int, default=200,
                    help="steps of the FP64 run whose time steps the FP32 and learned forms replay for their L1 "
                         "error (0: time the forms at the first CFL step without the comparison; negative: skip "
                         "the forms)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-weights form")
    ap.add_argument("--forms", default="all",
                    help="comma-separated forms to compare after the FP64 run (fp32_mixed, fp64_weno3, fp64_wenoz, "
                         "learned, learned_edge; default all), e.g. to profile one form's kernels")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain device-to-device copy of 7 * n^3 float64 (known bytes), five times, "
                         "to scale rocprofv3 FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.n is None:
        args.n = WORKLOADS[args.workload][1]

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU halo exchange is a design note, not code)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2409_10729_amd import (MFX_FP32_MIXED, MFX_FP64, MFX_WENO5_JS, MFX_WENO5_LEARNED,
                                      MFX_WENO5_LEARNED_EDGE, MFX_WENO5_Z, Solver)
    from paper_2409_10729_amd import learned
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
    print(f"[bench] generating {args.workload} n={args.n} seed={args.seed}", file=sys.stderr, flush=True)
    P = getattr(wl, args.workload)(n=args.n, seed=args.seed)
    if "inflow_prim" in P:
        from paper_2409_10729_amd import inflow_states

        P["spec"] = dict(P["spec"], inflow=inflow_states(P["spec"], P["inflow_prim"]))
    N = args.n ** 3
    w_dev = torch.from_numpy(P["w"]).cuda()
    nv = P["w"].shape[0]  # variables: 7 for two fluids, 9 for three
    stretched = any(f is not None for f in P["spec"].get("faces") or ())
    # the byte count per cell follows the variable count; the flop count and
    # the learned weights are defined for two fluids on equal cells
    two_fluid_uniform = nv == 7 and not stretched
    state_bytes = 8 * nv
    nf = (nv - 3) // 2  # fluids: nf partial densities, 3 momenta, energy, nf - 1 fractions

    nets = {}
    if not args.no_learned and two_fluid_uniform:
        for wmode, path in ((MFX_WENO5_LEARNED, learned.DEFAULT_PARAMS), (MFX_WENO5_LEARNED_EDGE, learned.EDGE_PARAMS)):
            if os.path.exists(path):
                nets[wmode] = (torch.from_numpy(learned.load_params(path)).cuda(), path)

    def new_solver(precision, weights=MFX_WENO5_JS, order=5):
        s = Solver(dict(P["spec"], weno_order=order), precision=precision, weights=weights)
        if weights in (MFX_WENO5_LEARNED, MFX_WENO5_LEARNED_EDGE):
            s.set_mlp(nets[weights][0])
        s.set_primitive(w_dev)
        return s

    def time_form(precision, dt, weights=MFX_WENO5_JS, order=5):
        """Warm-up, then `steps` timed steps with HIP events on the solver's
        stream; per-kernel event times from the library.  dt <= 0 uses the
        device CFL step (FP64 headline run)."""
        s = new_solver(precision, weights, order)
        for _ in range(args.warmup):
            s.rk3_step(dt)
        torch.cuda.synchronize()
        s.profile(True)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(s.stream)
        for _ in range(args.steps):
            s.rk3_step(dt)
        ev1.record(s.stream)
        torch.cuda.synchronize()
        ms_total = ev0.elapsed_time(ev1)
        prof = s.profile_read()
        s.profile(False)
        st = s.stats()
        if st["error"] != 0:
            raise RuntimeError(f"solver flagged a non-physical state: {st}")
        s.destroy()
        return ms_total, prof

    def replay(precision, dts, weights=MFX_WENO5_JS, order=5):
        """Final state (host, [7, N]) and fallback count after replaying dts."""
        s = new_solver(precision, weights, order)
        for dt in dts:
            s.rk3_step(dt)
        q = s.get_state().cpu().numpy().reshape(nv, -1)
        fb = s.stats()["fallback_faces"]
        s.destroy()
        return q, fb

    def l1_vs(q, q64):
        den = np.abs(q64).sum(axis=1)
        den[nf:nf + 3] = den[nf:nf + 3].max()  # the momenta share one scale
        l1 = (np.abs(q - q64).sum(axis=1) / den).tolist()
        rho64 = q64[:nf].sum(axis=0)
        rho_l1 = float(np.abs(q[:nf].sum(axis=0) - rho64).sum() / np.abs(rho64).sum())
        return [float(f"{x:.3e}") for x in l1], float(f"{rho_l1:.3e}")

    def kernel_table(prof, ms_total, rhs_bytes, order=5):
        per_dir = {}
        for (d, first, mode), (ms, cnt) in prof.items():
            b = sweep_bytes_per_cell(first, mode, rhs_bytes, state_bytes) * N
            e = per_dir.setdefault(d, {"ms": 0.0, "launches": 0, "bytes": 0, "flops": 0})
            e["ms"] += ms
            e["launches"] += cnt
            e["bytes"] += b * cnt
            e["flops"] += sweep_flops_per_cell(d, mode, order) * N * cnt if two_fluid_uniform else 0
        kernels = {}
        for d, e in sorted(per_dir.items()):
            mean_ms = e["ms"] / e["launches"]
            bpl = e["bytes"] / e["launches"]
            fpl = e["flops"] / e["launches"]
            kernels[KERNEL_NAMES[d]] = {
                "mean_us": round(mean_ms * 1e3, 2),
                "launches": e["launches"],
                "share": round(e["ms"] / ms_total, 4),
                "alg_bytes_per_launch": bpl,
                "achieved_GBs": round(bpl / (mean_ms * 1e-3) / 1e9, 1),
            }
            if two_fluid_uniform:
                kernels[KERNEL_NAMES[d]].update({
                    "alg_flops_per_launch": fpl,
                    "achieved_TFLOPs": round(fpl / (mean_ms * 1e-3) / 1e12, 2),
                    "flop_per_byte": round(fpl / bpl, 2),
                })
        step_bytes = sum(e["bytes"] for e in per_dir.values()) / args.steps
        return kernels, step_bytes

    # ---- FP64 headline run
    print(f"[bench] fp64: warmup {args.warmup}, {args.steps} timed steps", file=sys.stderr, flush=True)
    ms_total, prof = time_form(MFX_FP64, 0.0)
    ms_step = ms_total / args.steps
    grind = ms_step * 1e6 / (N * 3)
    kernels, step_bytes = kernel_table(prof, ms_total, state_bytes)
    print(f"[bench] fp64: {ms_step:.3f} ms/step, {grind:.4f} ns/cell/stage", file=sys.stderr, flush=True)
    dom = max(kernels, key=lambda k: kernels[k]["mean_us"] * kernels[k]["launches"])
    kd = kernels[dom]
    if two_fluid_uniform:
        # the dominant kernel's bound by its arithmetic intensity against the
        # ridge point of the float64 vector peak and HBM bandwidth
        ridge = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
        if kd["flop_per_byte"] >= ridge:
            roofline = {"bound": "alu", "achieved": kd["achieved_TFLOPs"], "peak": FP64_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(kd["achieved_TFLOPs"] / FP64_PEAK_TFLOPS, 4)}
        else:
            roofline = {"bound": "hbm", "achieved": kd["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(kd["achieved_GBs"] / HBM_PEAK_GBS, 4)}
        roofline.update({
            "traffic": load_traffic(dom),
            "kernel": dom,
            "mean_us": kd["mean_us"],
            "alg_bytes_per_launch": kd["alg_bytes_per_launch"],
            "alg_flops_per_launch": kd["alg_flops_per_launch"],
            "flop_per_byte": kd["flop_per_byte"],
            "ridge_flop_per_byte": round(ridge, 2),
            "hbm_frac": round(kd["achieved_GBs"] / HBM_PEAK_GBS, 4),
        })
    else:
        # (the flop count per cell is written for two fluids on equal cells)
        roofline = {"bound": "hbm", "achieved": kd["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(kd["achieved_GBs"] / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                    "mean_us": kd["mean_us"], "alg_bytes_per_launch": kd["alg_bytes_per_launch"],
                    "note": "algorithmic bytes only: the flop model covers two fluids on equal cells"}

    forms = {"fp64": {"ms_per_step": round(ms_step, 4), "grind": round(grind, 5), "kernels": kernels,
                      "step_alg_bytes_hbm_frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}

    # ---- FP32 mixed and learned forms: accuracy against FP64 on replayed
    # time steps, then timing at a fixed step
    if args.compare_steps >= 0:
        print(f"[bench] accuracy: fp64 reference over {args.compare_steps} steps", file=sys.stderr, flush=True)
        s64 = new_solver(MFX_FP64)
        if args.compare_steps > 0:
            dts = [s64.rk3_step(sync=True) for _ in range(args.compare_steps)]
            q64 = s64.get_state().cpu().numpy().reshape(nv, -1)
        else:
            # timing only (e.g. under a profiler): the forms run at the first
            # CFL step, with no accuracy comparison
            dts, q64 = [s64.rk3_step(sync=True)], None
        s64.destroy()
        del s64
        dt_fixed = dts[0]
        # (name, precision, weights, WENO order); fp64_weno3 (third order) and
        # fp64_wenoz (WENO-Z weights) are different schemes: their L1
        # distance to the fifth-order Jiang-Shu run is a scheme difference
        variants = [("fp32_mixed", MFX_FP32_MIXED, MFX_WENO5_JS, 5)]
        if not stretched:  # (unequal cells take WENO5 with Jiang-Shu weights)
            variants += [("fp64_weno3", MFX_FP64, MFX_WENO5_JS, 3), ("fp64_wenoz", MFX_FP64, MFX_WENO5_Z, 5)]
        if MFX_WENO5_LEARNED in nets:
            variants.append(("learned", MFX_FP32_MIXED, MFX_WENO5_LEARNED, 5))
        if MFX_WENO5_LEARNED_EDGE in nets:
            variants.append(("learned_edge", MFX_FP32_MIXED, MFX_WENO5_LEARNED_EDGE, 5))
        if args.forms != "all":
            keep = set(args.forms.split(","))
            unknown = keep - {v[0] for v in variants}
            if unknown:
                raise SystemExit(f"bench.py: unknown or unavailable forms {sorted(unknown)}")
            variants = [v for v in variants if v[0] in keep]
        for name, prec, weights, order in variants:
            l1 = rho_l1 = fb = None
            if q64 is not None:
                print(f"[bench] {name}: replaying {len(dts)} steps", file=sys.stderr, flush=True)
                q, fb = replay(prec, dts, weights, order)
                l1, rho_l1 = l1_vs(q, q64)
                del q
            print(f"[bench] {name}: timing {args.steps} steps", file=sys.stderr, flush=True)
            ms_f, prof_f = time_form(prec, dt_fixed, weights, order)
            msf_step = ms_f / args.steps
            kf, _ = kernel_table(prof_f, ms_f, state_bytes if prec == MFX_FP64 else 4 * nv, order)
            forms[name] = {
                "ms_per_step": round(msf_step, 4),
                "grind": round(msf_step * 1e6 / (N * 3), 5),
                "speedup_vs_fp64": round(ms_step / msf_step, 3),
                "compare_steps": args.compare_steps,
                "l1_rel_vs_fp64": l1,
                "density_l1_rel_vs_fp64": rho_l1,
                "kernels": kf,
            }
            if weights in nets and fb is not None:
                edges = 2 * N * sum(1 for k in P["spec"]["n"] if k > 1) * 3 * len(dts)
                forms[name]["fallback_edges"] = fb
                forms[name]["fallback_fraction"] = float(f"{fb / max(edges, 1):.3e}")
                forms[name]["network"] = os.path.relpath(nets[weights][1], os.path.dirname(os.path.abspath(__file__)))
            acc = f", density L1 {rho_l1:.2e}" if rho_l1 is not None else ""
            print(f"[bench] {name}: {msf_step:.3f} ms/step (x{ms_step / msf_step:.2f}){acc}", file=sys.stderr,
                  flush=True)
        del q64
    del w_dev

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
            "workload": f"{args.workload} {args.n}^3: {WORKLOADS[args.workload][0]}, CFL 0.4, WENO5-JS + HLLC + "
                        f"SSP-RK3, FP64",
            "cells": N,
            "seed": args.seed,
            "precision": "fp64",
        },
        "grind_ns_per_cell_pde_rhs": round(grind / nv, 6),
        "roofline": roofline,
        "forms": forms,
    }
    if not args.no_cpu:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        import oracle

        P_cpu = dict(P)
        if "inflow_prim" in P:  # the oracle converts the inflow states itself
            one = {k: v for k, v in P["spec"].items() if k != "inflow"}
            g1 = oracle.make_grid(dict(one, n=(1, 1, 1), bc=((0, 0),) * 3))
            conv = [[oracle.prim_to_cons(g1, np.asarray(w7, dtype=np.float64).reshape(7, 1, 1, 1)).reshape(7)
                     for w7 in pair] for pair in P["inflow_prim"]]
            P_cpu["spec"] = dict(one, inflow=np.array(conv))
        q_ic = oracle.prim_to_cons(oracle.make_grid(P_cpu["spec"]), P["w"])
        cb = cpu_baseline(P_cpu, q_ic, args.cpu_budget)
        out["cpu_baseline"] = cb
        out["gpu_over_cpu"] = round(cb["value"] / grind, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
