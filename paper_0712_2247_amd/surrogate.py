"""Workflow of the learned force: training data from plain runs, training, and
evaluation of the surrogate path against the exact one.

Host orchestration only: every step, snapshot, forward/backward pass and Adam
update runs in libhslb.so (``hslb.Sim``, ``hslb.Trainer``).

Training data: slits driven by the exact force; every ``every`` steps the
trainer stores the state's network input and its exact force (C1 without the
external field).  A run that the watchdog flags as unstable (the scheme
diverges above a packing that depends on sigma and tau) contributes nothing,
so that diverging states never enter the data.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import hslb, workloads


def is_stable(wl: workloads.Workload, steps: int, precision: str = "f32") -> bool:
    """Runs the plain path for `steps` steps under the watchdog (every 50
    steps: finite state, mass within 1e-3)."""
    s = hslb.Sim.from_workload(wl, precision=precision)
    n, u = wl.fields()
    s.init(n, u)
    hslb.hslb_set_watchdog(s.ctx, 50, 1e-3)
    try:
        s.step(steps)
        return True
    except hslb.HslbError as e:
        if e.code == hslb.HSLB_EUNSTABLE:
            return False
        raise
    finally:
        s.close()


def collect(trainer: hslb.Trainer, wls: Sequence[workloads.Workload], every: int, steps: int,
            precision: str = "f32", log=None) -> List[Dict]:
    """Snapshots every `every` steps (from step `every` on) of each stable run;
    returns one record per run."""
    out = []
    for k, wl in enumerate(wls):
        rec = {"run": k, "name": wl.name, "sigma": wl.sigma, "eta": wl.eta, "nz": wl.nz,
               "stable": is_stable(wl, steps, precision), "snapshots": []}
        if rec["stable"]:
            s = hslb.Sim.from_workload(wl, precision=precision)
            n, u = wl.fields()
            s.init(n, u)
            for _ in range(steps // every):
                s.step(every)
                rec["snapshots"].append(trainer.add(s))
            s.close()
        if log:
            log(f"run {k}: sigma {wl.sigma} eta {wl.eta:.3f} nz {wl.nz} "
                f"{'stable' if rec['stable'] else 'unstable'}, {len(rec['snapshots'])} snapshots")
        out.append(rec)
    return out


def train(trainer: hslb.Trainer, w0: np.ndarray, snapshots: Sequence[int], epochs: int, lr: float,
          seed: int = 1008, lr_decay: float = 0.5, log=None) -> Dict:
    """Adam over the given snapshots in a seeded random order per epoch; the
    learning rate is multiplied by lr_decay after each epoch."""
    trainer.set_weights(w0)
    rng = np.random.default_rng(seed)
    losses = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(np.asarray(snapshots, dtype=np.int32))
        L = trainer.train(order, lr * lr_decay ** ep)
        losses.append(L)
        if log:
            log(f"epoch {ep}: mean loss {L:.4e} ({time.perf_counter() - t0:.1f} s)")
    return {"weights": trainer.weights(), "losses": losses, "seconds": time.perf_counter() - t0,
            "steps": epochs * len(snapshots)}


def evaluate(wl: workloads.Workload, w: Optional[np.ndarray], steps: int, K: int, tol: float,
             mode: int = hslb.HSLB_SURR_CORRECTED, precision: str = "f32",
             reference: Optional[tuple] = None, components: int = 7) -> Dict:
    """Runs the surrogate path for `steps` steps and returns its throughput
    (every step, checks included), judge statistics and profile errors
    against `reference` = (n_z, u_z) of the exact path (relative L2 of n(z)
    and u_x(z) over the fluid layers).  `components`: the force components
    the network drives (bits x, y, z; 4 = wall-normal only)."""
    s = hslb.Sim.from_workload(wl, precision=precision, force_mode=hslb.HSLB_FORCE_SURROGATE,
                               surr_check_every=K, surr_tol=tol)
    hslb.hslb_surrogate_set_weights(s.ctx, w if w is not None else
                                    np.zeros(hslb.HSLB_CNN_NWEIGHTS, dtype=np.float32))
    hslb.hslb_surrogate_set_mode(s.ctx, mode)
    hslb.hslb_surrogate_set_components(s.ctx, components)
    n, u = wl.fields()
    s.init(n, u)
    # the watchdog (every K steps: finite state, mass within 1e-3) stops a run
    # that the learned force destabilises
    hslb.hslb_set_watchdog(s.ctx, K, 1e-3)
    s.sync()
    diverged_at = None
    t0 = time.perf_counter()
    try:
        s.step(steps)
        s.sync()
    except hslb.HslbError as e:
        if e.code != hslb.HSLB_EUNSTABLE:
            raise
        diverged_at = hslb.hslb_step_count(s.ctx)
    dt = time.perf_counter() - t0
    done = hslb.hslb_step_count(s.ctx)
    checks, fallback, last_r, max_r = hslb.hslb_surrogate_stats(s.ctx)
    pn, pu = s.profiles()
    s.close()
    fin = lambda v: float(v) if np.isfinite(v) else None  # noqa: E731
    out = {"steps": steps, "K": K, "tol": tol, "mode": {0: "corrected", 1: "plain", 2: "frozen"}[mode],
           "components": components,
           "mlups": wl.fluid_nodes * done / dt / 1e6, "ms_per_step": dt / max(done, 1) * 1e3,
           "checks": checks, "fallback_steps": fallback, "last_residual": fin(last_r),
           "max_residual": fin(max_r), "diverged_at_step": diverged_at}
    if reference is not None and diverged_at is None:
        fl = slice(wl.wall_lo, wl.nz - wl.wall_hi)
        rn, ru = reference
        out["profile_err_n"] = float(np.linalg.norm(pn[fl] - rn[fl]) / np.linalg.norm(rn[fl]))
        out["profile_err_ux"] = float(np.linalg.norm(pu[0][fl] - ru[0][fl]) / np.linalg.norm(ru[0][fl]))
    return out


def exact_profiles(wl: workloads.Workload, steps: int, precision: str = "f32"):
    s = hslb.Sim.from_workload(wl, precision=precision)
    n, u = wl.fields()
    s.init(n, u)
    s.step(steps)
    p = s.profiles()
    s.close()
    return p
