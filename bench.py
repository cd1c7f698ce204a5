"""Throughput of the hard-sphere lattice Boltzmann step on one MI355X.

Workload: the 64x64x136 slit (128 fluid layers), sigma 8, tau 0.8, g 2e-6
along x, FP32 populations with FP64 arithmetic, exact shell-sum force: the
plain path of the benchmark metric.  The slit is specified at packing fraction
0.35, where the scheme diverges a few hundred steps after the uniform start;
the timed run uses packing fraction 0.25 (same grid, stencil and cost per
step; 0.30 and above diverge on this grid), and the 0.35 slit is timed
separately over 250 steps.  Inputs are seeded and synthetic (paper_0712_2247_amd.workloads).

A step is one pass of the whole hot path: moments, coarse-grained density,
midpoint contact values, hard-sphere force plus external field, BGK collision,
streaming with bounce-back.  The state stays resident in HBM; the timed region
is K steps replayed from the library's HIP graphs, bracketed by stream
synchronisation.  A second pass of K steps launches kernel by kernel with HIP
events on the library's stream to time each kernel (roofline).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
# Algorithmic bytes per fluid-node update (FP32 populations, FP32 moments):
#   whole step: 19 populations read + written (152 B) + n, j written and read
#   once (32 B) = 184 B; the fused force/collide/stream kernel alone: 152 B of
#   populations + n, j read once (16 B) = 168 B.
STEP_BYTES = 184.0
COLLIDE_BYTES = 168.0
# The same counts on the 39-velocity lattice (FP64 populations, FP64 moments):
#   step 39 x 8 x 2 = 624 B + n, j written and read (64 B) = 688 B; its collide
#   kernel 624 B + n, j read once (32 B) = 656 B.
STEP39_BYTES = 688.0
COLLIDE39_BYTES = 656.0
# With the non-isothermal terms the temperature field adds 8 B written and read
# once to the step and 8 B read to the collide kernel.
STEP39T_BYTES = 704.0
COLLIDE39T_BYTES = 664.0
DOMINANT = "collide"


def _kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("hslb_kernels.hip", "hslb_internal.hpp"):
        with open(os.path.join(ROOT, "paper_0712_2247_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_collide_slit64x64x136_s8.txt")
TRAFFIC39_FILE = os.path.join(ROOT, "profiles", "traffic_collide39_slit64x64x136_s8.txt")
TRAFFIC39T_FILE = os.path.join(ROOT, "profiles", "traffic_collide39_thermal_slit64x64x136_s8.txt")
TRAFFIC_BULK_FILE = os.path.join(ROOT, "profiles", "traffic_collide_bulk256_s6.txt")


def _traffic(workload: str, path: str = TRAFFIC_FILE):
    """HBM bytes per launch of a collide kernel, from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary (key = value lines), if it was
    taken on the current kernel source and workload; else None."""
    try:
        rec = {}
        for line in open(path):
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                rec[k.strip()] = v.strip()
    except OSError:
        return None
    if rec.get("kernel_source_hash") != _kernel_source_hash() or rec.get("workload") != workload:
        return None
    return float(rec["bytes_per_launch"])


def ensemble_throughput(hslb, workloads, steps: int):
    """The 512-slit ragged ensemble advanced by the batched persistent path
    (autotuned launch shape, graph replay): MLUPS over `steps` steps."""
    wls = workloads.ensemble()
    b = hslb.Batch(wls)
    b.init_all()
    choice, us = b.autotune(steps=10)
    b.step(20)
    b.sync()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    dt = time.perf_counter() - t0
    fin = int(b.finite().sum())
    out = {"workload": f"{len(wls)} slits 16x16x(H+walls), H 10..60, sigma 3..8, packing 0.10..0.40",
           "fluid_nodes": b.fluid_nodes, "steps": steps,
           "value": round(b.fluid_nodes * steps / dt / 1e6, 1), "unit": "MLUPS",
           "ms_per_step": round(dt / steps * 1e3, 5),
           "autotune_choice": int(choice), "finite_slits": fin}
    b.close()
    return out


PEAK_BF16_TFLOPS = 2500.0


def surrogate_leg(hslb, workloads, wl, steps: int, epochs: int):
    """The learned force on the benchmark slit: snapshots of the 40 training
    slits (64x64xnz, sigma 4..8, stable runs only), Adam on the GPU, then the
    surrogate path (exact judge every 50 steps, residual threshold 1e-3) with
    the network plus frozen correction and without the network (frozen exact
    force: the ablation), each against the exact path's profiles."""
    from paper_0712_2247_amd import surrogate
    runs = workloads.surrogate_training_runs()
    tr = hslb.Trainer(sum(w.nodes for w in runs) * 100 + 1, max(w.nodes for w in runs))
    t0 = time.perf_counter()
    recs = surrogate.collect(tr, runs, 20, 2000)
    snaps = [k for r in recs for k in r["snapshots"]]
    t_collect = time.perf_counter() - t0
    res = surrogate.train(tr, workloads.cnn_init_weights(), snaps, epochs, 1e-3)
    w = res["weights"]
    tr.close()
    ref = surrogate.exact_profiles(wl, steps)
    out = {"training": {"runs": len(runs), "stable_runs": sum(r["stable"] for r in recs),
                        "snapshots": len(snaps), "epochs": epochs, "adam_steps": res["steps"],
                        "mean_loss_per_epoch": [float(v) for v in res["losses"]],
                        "collect_s": round(t_collect, 1), "train_s": round(res["seconds"], 1)}}
    for mode in (hslb.HSLB_SURR_CORRECTED, hslb.HSLB_SURR_FROZEN):
        r = surrogate.evaluate(wl, w, steps, 50, 1e-3, mode, reference=ref)
        out[r["mode"]] = r
        print(f"bench: surrogate {r['mode']}: {r}", file=sys.stderr, flush=True)
    # network kernel times on the benchmark slit (eager, HIP events)
    s = hslb.Sim.from_workload(wl, force_mode=hslb.HSLB_FORCE_SURROGATE, surr_check_every=50, surr_tol=1e-3)
    hslb.hslb_surrogate_set_weights(s.ctx, w)
    n, u = wl.fields()
    s.init(n, u)
    hslb.hslb_set_kernel_timing(s.ctx, True)
    s.step(100)
    s.sync()
    kt = {k: v[0] / v[1] * 1e3 for k, v in hslb.hslb_kernel_times(s.ctx).items()}
    s.close()
    out["kernels_us"] = {k: round(v, 2) for k, v in kt.items()}
    flops = 2.0 * 125 * 32 * 32 * wl.nodes   # layer 2: 32 -> 32 channels, 5^3 taps, every node
    ach = flops / (kt["cnn_l2"] * 1e-6) / 1e12
    out["roofline_cnn_l2"] = {"bound": "mfma", "achieved": round(ach, 1), "peak": PEAK_BF16_TFLOPS,
                              "unit": "TFLOP/s", "frac": round(ach / PEAK_BF16_TFLOPS, 4),
                              "algorithmic_flop_per_launch": flops}
    return out


def attraction_leg(hslb, wl, n, u, steps: int):
    """The benchmark slit with the mean-field attraction on (range sigma / 2,
    a 25-point cube side, depth 1e-3): throughput over `steps` graph-replayed
    steps, then the three potential passes and the collide timed per kernel."""
    lam = wl.sigma / 2.0
    s = hslb.Sim.from_workload(wl, att_eps=1e-3, att_range=lam)
    s.init(n, u)
    s.step(20)
    s.sync()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    dt = time.perf_counter() - t0
    hslb.hslb_set_kernel_timing(s.ctx, True)
    s.step(min(steps, 200))
    s.sync()
    kt = hslb.hslb_kernel_times(s.ctx)
    s.close()
    return {"workload": f"{wl.name} + attraction (range {lam:g}, cube side {2 * math.ceil(3 * lam) + 1})",
            "steps": steps, "value": round(wl.fluid_nodes * steps / dt / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(dt / steps * 1e3, 5),
            "kernels_us": {k: round(v[0] / v[1] * 1e3, 2) for k, v in kt.items()}}


def obstacle_leg(hslb, np, wl, n, u, steps: int):
    """The benchmark slit with a solid cylinder of radius sigma across y at its
    centre (solid mask, per-node wall factor): throughput over the fluid nodes
    that remain, graph-replayed steps."""
    z, x = np.meshgrid(np.arange(wl.nz), np.arange(wl.nx), indexing="ij")
    cyl = (z - wl.nz / 2) ** 2 + (x - wl.nx / 2) ** 2 <= wl.sigma ** 2
    m = np.broadcast_to(cyl[:, None, :], (wl.nz, wl.ny, wl.nx)).astype(np.uint8)
    fluid = wl.fluid_nodes - int(m.sum())
    s = hslb.Sim.from_workload(wl)
    s.set_solid(m)
    s.init(n, u)
    s.step(20)
    s.sync()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    dt = time.perf_counter() - t0
    finite = bool(np.isfinite(s.moments()[0]).all())
    s.close()
    return {"workload": f"{wl.name} + solid cylinder (radius {wl.sigma}, axis along y)",
            "fluid_nodes": fluid, "steps": steps, "value": round(fluid * steps / dt / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(dt / steps * 1e3, 5), "state_finite_after": finite}


def d3q39_leg(hslb, np, wl, n, u, steps: int, thermal: bool = False):
    """The benchmark slit on the third-order 39-velocity lattice (FP64
    populations and moments, regularised collision): throughput over `steps`
    graph-replayed steps, then the kernels timed one by one, with the collide
    kernel's achieved bandwidth on its algorithmic bytes.  thermal: with the
    non-isothermal terms, from a temperature 2 % above and below the lattice
    temperature across the slit."""
    s = hslb.Sim.from_workload(wl, precision="f64", lattice=hslb.HSLB_D3Q39, thermal=int(thermal))
    if thermal:
        T0 = 2.0 / 3.0
        zz = np.arange(wl.nz)
        T = np.broadcast_to((T0 * (1.0 + 0.02 * np.sin(2.0 * np.pi * zz / wl.nz)))[:, None, None],
                            (wl.nz, wl.ny, wl.nx)).copy()
        s.init(n, u, T)
    else:
        s.init(n, u)
    s.step(20)
    s.sync()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    dt = time.perf_counter() - t0
    hslb.hslb_set_kernel_timing(s.ctx, True)
    s.step(min(steps, 200))
    s.sync()
    kt = hslb.hslb_kernel_times(s.ctx)
    finite = bool(np.isfinite(s.moments()[0]).all())
    s.close()
    mlups = wl.fluid_nodes * steps / dt / 1e6
    col_s = kt["collide"][0] / kt["collide"][1] * 1e-3
    cb = COLLIDE39T_BYTES if thermal else COLLIDE39_BYTES
    col_gbps = cb * wl.fluid_nodes / col_s / 1e9
    return {"workload": f"{wl.name} on the 39-velocity lattice, FP64" + (", non-isothermal" if thermal else ""),
            "steps": steps,
            "value": round(mlups, 1), "unit": "MLUPS", "ms_per_step": round(dt / steps * 1e3, 5),
            "step_algorithmic_GBps": round(mlups * 1e6 * (STEP39T_BYTES if thermal else STEP39_BYTES) / 1e9, 1),
            "collide_us": round(col_s * 1e6, 2), "collide_GBps": round(col_gbps, 1),
            "collide_hbm_frac": round(col_gbps / PEAK_HBM_GBPS, 4),
            "collide_algorithmic_bytes": cb * wl.fluid_nodes,
            "collide_traffic": _traffic(wl.name, TRAFFIC39T_FILE if thermal else TRAFFIC39_FILE),
            "kernels_us": {k: round(v[0] / v[1] * 1e3, 2) for k, v in kt.items()},
            "state_finite_after": finite}


def fp64_leg(hslb, wl, n, u, steps: int):
    """The benchmark slit with FP64 population storage (all else equal):
    throughput over `steps` graph-replayed steps and the collide kernel's time.
    Two FP64 population copies (2 x 85 MB) exceed the 128 MiB threshold of the
    non-temporal collide instance."""
    s = hslb.Sim.from_workload(wl, precision="f64")
    s.init(n, u)
    s.step(20)
    s.sync()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    dt = time.perf_counter() - t0
    hslb.hslb_set_kernel_timing(s.ctx, True)
    s.step(min(steps, 200))
    s.sync()
    kt = hslb.hslb_kernel_times(s.ctx)
    s.close()
    return {"workload": f"{wl.name} with FP64 storage", "steps": steps,
            "value": round(wl.fluid_nodes * steps / dt / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(dt / steps * 1e3, 5),
            "kernels_us": {k: round(v[0] / v[1] * 1e3, 2) for k, v in kt.items()}}


def bulk_leg(hslb, workloads, steps: int):
    """The 256^3 periodic bulk (sigma 6, packing 0.25, FP32 storage, shear wave
    and density noise as its recipe states): throughput over `steps`
    graph-replayed steps and the per-kernel times.  Its two population copies
    (2 x 1.27 GB) overflow the last-level cache, so the collide runs the
    non-temporal instance."""
    wl = workloads.bulk_256_f32()
    n, u = wl.fields()
    s = hslb.Sim.from_workload(wl)
    s.init(n, u)
    del n, u
    s.step(20)
    s.sync()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    dt = time.perf_counter() - t0
    hslb.hslb_set_kernel_timing(s.ctx, True)
    s.step(min(steps, 100))
    s.sync()
    kt = hslb.hslb_kernel_times(s.ctx)
    s.close()
    col_s = kt["collide"][0] / kt["collide"][1] * 1e-3
    col_gbps = COLLIDE_BYTES * wl.fluid_nodes / col_s / 1e9
    return {"workload": wl.name, "steps": steps,
            "value": round(wl.fluid_nodes * steps / dt / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(dt / steps * 1e3, 5),
            "collide_us": round(col_s * 1e6, 2), "collide_GBps": round(col_gbps, 1),
            "collide_hbm_frac": round(col_gbps / PEAK_HBM_GBPS, 4),
            "collide_algorithmic_bytes": int(COLLIDE_BYTES * wl.fluid_nodes),
            "collide_traffic": _traffic(wl.name, TRAFFIC_BULK_FILE),
            "kernels_us": {k: round(v[0] / v[1] * 1e3, 2) for k, v in kt.items()}}


def cpu_baseline(wl, n, u, budget_s: float):
    import oracle
    o = oracle.Oracle(**wl.params())
    o.init(n, u)
    o.step(1)  # first-touch
    steps = 0
    t0 = time.perf_counter()
    while True:
        o.step(1)
        steps += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s and steps >= 2:
            break
    return {"value": wl.fluid_nodes * steps / dt / 1e6, "unit": "MLUPS",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{steps} full steps of the {wl.nx}x{wl.ny}x{wl.nz} slit, FP64 C oracle, "
                      f"OpenMP, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-pass", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-attraction", action="store_true")
    ap.add_argument("--no-obstacle", action="store_true")
    ap.add_argument("--no-d3q39", action="store_true")
    ap.add_argument("--no-thermal", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-bulk", action="store_true")
    ap.add_argument("--surrogate-epochs", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0712_2247_amd import hslb, workloads

    wl = workloads.slit_64_f32_stable()
    n, u = wl.fields()
    sim = hslb.Sim.from_workload(wl)
    sim.init(n, u)
    print(f"bench: {wl.name} warmup {args.warmup}", file=sys.stderr, flush=True)
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    sim.step(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    mlups = wl.fluid_nodes * args.steps / dt / 1e6
    print(f"bench: timed {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)

    # the slit as specified (eta 0.35), timed before it diverges
    spec = workloads.slit_64_f32()
    sn, su = spec.fields()
    ssim = hslb.Sim.from_workload(spec)
    ssim.init(sn, su)
    ssim.step(20)
    ssim.sync()
    k_spec = min(args.steps, 250)
    t1 = time.perf_counter()
    ssim.step(k_spec)
    ssim.sync()
    dt_spec = time.perf_counter() - t1
    spec_finite = bool(np.isfinite(ssim.moments()[0]).all())
    ssim.close()
    as_specified = {"workload": spec.name, "steps": k_spec,
                    "value": round(spec.fluid_nodes * k_spec / dt_spec / 1e6, 1),
                    "ms_per_step": round(dt_spec / k_spec * 1e3, 5),
                    "state_finite_after": spec_finite,
                    "note": "diverges under the scheme within ~15 steps of the noisy "
                            "uniform start (FP64 oracle: density x1e13 by step 15); timed over "
                            "steps 20-270 on the diverged state: work and traffic per step do "
                            "not depend on the values"}

    roof = None
    kernels = {}
    if not args.no_kernel_pass:
        hslb.hslb_set_kernel_timing(sim.ctx, True)
        sim.step(args.steps)
        sim.sync()
        kt = hslb.hslb_kernel_times(sim.ctx)
        hslb.hslb_set_kernel_timing(sim.ctx, False)
        kernels = {k: {"avg_us": v[0] / v[1] * 1e3, "launches": v[1]} for k, v in kt.items()}
        avg_s = kt[DOMINANT][0] / kt[DOMINANT][1] * 1e-3
        per_launch = COLLIDE_BYTES * wl.fluid_nodes
        achieved = per_launch / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBPS, 4),
                "traffic": _traffic(wl.name), "kernel": "k_collide",
                "algorithmic_bytes_per_launch": per_launch,
                "avg_launch_us": round(avg_s * 1e6, 2)}
        print(f"bench: kernel pass {kernels}", file=sys.stderr, flush=True)

    gn, gu = sim.moments()
    assert np.isfinite(gn).all(), "non-finite state"
    sim.close()

    copy_gbps = hslb.hslb_copy_bandwidth(1 << 30, 20)
    print(f"bench: device copy {copy_gbps:.0f} GB/s", file=sys.stderr, flush=True)

    ens = None
    if not args.no_ensemble:
        print("bench: ensemble", file=sys.stderr, flush=True)
        ens = ensemble_throughput(hslb, workloads, min(args.steps, 500))

    surr = None
    if not args.no_surrogate:
        print("bench: surrogate", file=sys.stderr, flush=True)
        surr = surrogate_leg(hslb, workloads, wl, args.steps, args.surrogate_epochs)

    att = None
    if not args.no_attraction:
        print("bench: attraction", file=sys.stderr, flush=True)
        att = attraction_leg(hslb, wl, n, u, args.steps)

    obst = None
    if not args.no_obstacle:
        print("bench: obstacle", file=sys.stderr, flush=True)
        obst = obstacle_leg(hslb, np, wl, n, u, args.steps)

    f64 = None
    if not args.no_fp64:
        print("bench: FP64 storage", file=sys.stderr, flush=True)
        f64 = fp64_leg(hslb, wl, n, u, min(args.steps, 1000))

    bulk = None
    if not args.no_bulk:
        print("bench: 256^3 bulk", file=sys.stderr, flush=True)
        bulk = bulk_leg(hslb, workloads, min(args.steps, 300))

    q39 = None
    if not args.no_d3q39:
        print("bench: 39-velocity lattice", file=sys.stderr, flush=True)
        q39 = d3q39_leg(hslb, np, wl, n, u, min(args.steps, 1000))

    q39t = None
    if not args.no_thermal:
        print("bench: 39-velocity lattice, non-isothermal", file=sys.stderr, flush=True)
        q39t = d3q39_leg(hslb, np, wl, n, u, min(args.steps, 500), thermal=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(wl, n, u, args.cpu_seconds)

    out = {
        "metric": "MLUPS incl. HS force: plain FP32 vs surrogate at <=1e-3 profile err; % HBM BW",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": [wl.nx, wl.ny, wl.nz],
                   "fluid_nodes": wl.fluid_nodes, "sigma": wl.sigma, "eta": wl.eta,
                   "tau": wl.tau, "storage": "f32 populations, f32 moments",
                   "force": "exact shell sum", "parallelism": "single GPU"},
        "step_algorithmic_GBps": round(mlups * 1e6 * STEP_BYTES / 1e9, 1),
        "step_hbm_frac": round(mlups * 1e6 * STEP_BYTES / 1e9 / PEAK_HBM_GBPS, 4),
        "copy_GBps": round(copy_gbps, 1),
        "step_copy_frac": round(mlups * 1e6 * STEP_BYTES / 1e9 / copy_gbps, 4),
        "as_specified": as_specified,
        "ensemble": ens,
        "surrogate": surr,
        "attraction": att,
        "obstacle": obst,
        "fp64_storage": f64,
        "bulk": bulk,
        "d3q39": q39,
        "d3q39_thermal": q39t,
        "roofline": roof,
        "kernels_us": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
