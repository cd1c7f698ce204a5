"""The learned force on the held-out 128x128x264 slit (sigma 8, packing 0.28,
tau 1, g 1e-6; the specified packing 0.38 is linearly unstable under the
scheme): the surrogate path's profiles after 3000 steps against the FP64
oracle's run of the same slit (tests/golden, written by make_golden.py from
the oracle alone; 3000 steps of the oracle took 2.4 hours on 6 threads, so
the comparison is made in the transient, where the force changes fastest,
rather than at the steady state some 10^5 steps later), and what the trained
network gains over the method without it, on every force component and on
the wall-normal one only.

The network is trained here on the first 12 of the 40 seeded training slits
(64x64xnz, sigma 4..8, packing 0.1..0.4; slits the watchdog flags as unstable
contribute nothing), 100 snapshots each over 2000 steps, 2 epochs of Adam.
The path checks the exact force every K = 50 steps with the residual
threshold 1e-3 and falls back to exact steps above it."""
import json
import os

import numpy as np
import pytest

from paper_0712_2247_amd import hslb, surrogate, workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "slit_128x128x264_eta0.28_profiles.json")
STEPS = 3000
K, TOL = 50, 1e-3


def _golden(step):
    with open(GOLDEN) as fh:
        snap = json.load(fh)["snapshots"][str(step)]
    return np.array(snap["n_z"]), np.array(snap["u_z"])


@pytest.fixture(scope="module")
def trained():
    runs = workloads.surrogate_training_runs()[:12]
    tr = hslb.Trainer(sum(w.nodes for w in runs) * 100 + 1, max(w.nodes for w in runs))
    recs = surrogate.collect(tr, runs, 20, 2000)
    snaps = [k for r in recs for k in r["snapshots"]]
    assert len(snaps) >= 300
    res = surrogate.train(tr, workloads.cnn_init_weights(), snaps, 2, 1e-3)
    tr.close()
    print(f"training: {len(snaps)} snapshots, mean loss per epoch {res['losses']}", flush=True)
    return res["weights"]


def _errors(r):
    return r.get("profile_err_n"), r.get("profile_err_ux")


def test_frozen_surrogate_path_meets_the_profile_bar_on_the_held_out_slit(trained):
    """The surrogate path without the network (the frozen exact force of the
    last check between checks): n(z), u_x(z) within 1e-3 relative L2 of the
    oracle after 3000 steps, with frozen-force steps actually taken."""
    wl = workloads.slit_128_f32_stable()
    r = surrogate.evaluate(wl, trained, STEPS, K, TOL, hslb.HSLB_SURR_FROZEN, reference=_golden(STEPS))
    frozen = r["steps"] - r["checks"] - r["fallback_steps"]
    print(f"frozen: {r}; steps on the frozen force {frozen}", flush=True)
    assert r["diverged_at_step"] is None
    en, eu = _errors(r)
    assert en <= 1e-3 and eu <= 1e-3
    assert frozen > 0


def test_exact_path_against_the_oracle_on_the_held_out_slit():
    """The plain FP32 path on the same slit: profiles within 1e-5 of the oracle
    at every stored step (the bar of the plain path)."""
    wl = workloads.slit_128_f32_stable()
    n, u = wl.fields()
    g = hslb.Sim.from_workload(wl)
    g.init(n, u)
    fl = slice(wl.wall_lo, wl.nz - wl.wall_hi)
    done = 0
    for t in (500, 1000, 2000, 3000):
        g.step(t - done)
        done = t
        pn, pu = g.profiles()
        on, ou = _golden(t)
        en = np.linalg.norm(pn[fl] - on[fl]) / np.linalg.norm(on[fl])
        eu = np.linalg.norm(pu[0][fl] - ou[0][fl]) / np.linalg.norm(ou[0][fl])
        print(f"exact path, step {t}: n_z {en:.2e}, u_x {eu:.2e}", flush=True)
        assert en <= 1e-5 and eu <= 1e-5


def test_what_the_network_gains_over_the_ablation(trained):
    """The network plus the frozen correction against the no-network ablation
    on the held-out slit, on every force component and on the wall-normal
    component only (components = 4: the in-plane components keep the exact
    force of the last check).  Measured relations, asserted as they stand:

    - On every component the network fails the bar on u_x (measured: 45-66 %
      off after acting on 49 of 3000 steps).  In the slit the in-plane force
      balances the driving field, g n ~ 1e-9 per node, while the network's
      output error is of the order of the layering force it learns (~1e-5):
      between checks its in-plane outputs move the flow.
    - Wall-normal only, it meets the bar (measured: n 2.8e-4 - 4.3e-4, u_x
      1.1e-4 - 1.2e-4), as does the ablation (8.6e-4, 3.3e-4), whose profiles
      it beats here.  It takes the surrogate force on 49 steps against the
      ablation's 147 (the judge rejects more of its checks in the transient)
      and so runs slower (about 7300 against 8400 MLUPS): the gain is in
      accuracy at fewer approximate steps, not in throughput.
    The trained weights, and with them these figures, move with the rounding
    of the network kernels (the ranges span two kernel versions)."""
    wl = workloads.slit_128_f32_stable()
    ref = _golden(STEPS)
    net = surrogate.evaluate(wl, trained, STEPS, K, TOL, hslb.HSLB_SURR_CORRECTED, reference=ref)
    wn = surrogate.evaluate(wl, trained, STEPS, K, TOL, hslb.HSLB_SURR_CORRECTED, reference=ref,
                            components=4)
    abl = surrogate.evaluate(wl, trained, STEPS, K, TOL, hslb.HSLB_SURR_FROZEN, reference=ref)
    print(f"network + correction: {net}", flush=True)
    print(f"wall-normal network + correction: {wn}", flush=True)
    print(f"ablation (frozen exact force): {abl}", flush=True)
    ea = max(_errors(abl))
    assert ea <= 1e-3
    if net["diverged_at_step"] is None:
        assert max(_errors(net)) > ea
    assert wn["diverged_at_step"] is None
    assert max(_errors(wn)) <= 1e-3
    assert wn["steps"] - wn["checks"] - wn["fallback_steps"] > 0   # the network did act
    # checks happen on schedule in every run
    assert abl["checks"] == wn["checks"] == STEPS // K


GOLDEN_BENCH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "slit_64x64x136_eta0.25_profiles.json")


def test_wall_normal_network_on_the_benchmark_slit():
    """The benchmark's surrogate leg as a test: the network trained on all 40
    training slits (27 stable, 2700 snapshots, 2 epochs), then 5000 steps of
    the 64x64x136 slit (sigma 8, packing 0.25, tau 0.8) with K = 50, against
    the oracle's FP64 run of the same slit (tests/golden).  The wall-normal
    variant and the ablation meet the 1e-3 bar, and the network acts on some
    of the steps.  Measured: wall-normal n 7.6e-6 - 4.9e-5, u_x 3.5e-5 -
    3.6e-5 on 245-343 network steps (two versions of the network kernels);
    ablation 4.0e-4 and 2.5e-4 on 784 frozen steps."""
    runs = workloads.surrogate_training_runs()
    tr = hslb.Trainer(sum(w.nodes for w in runs) * 100 + 1, max(w.nodes for w in runs))
    recs = surrogate.collect(tr, runs, 20, 2000)
    snaps = [k for r in recs for k in r["snapshots"]]
    w = surrogate.train(tr, workloads.cnn_init_weights(), snaps, 2, 1e-3)["weights"]
    tr.close()
    steps = 5000
    with open(GOLDEN_BENCH) as fh:
        snap = json.load(fh)["snapshots"][str(steps)]
    ref = (np.array(snap["n_z"]), np.array(snap["u_z"]))
    wl = workloads.slit_64_f32_stable()
    wn = surrogate.evaluate(wl, w, steps, K, TOL, hslb.HSLB_SURR_CORRECTED, reference=ref, components=4)
    abl = surrogate.evaluate(wl, w, steps, K, TOL, hslb.HSLB_SURR_FROZEN, reference=ref)
    print(f"{len(snaps)} snapshots; wall-normal: {wn}; ablation: {abl}", flush=True)
    assert wn["diverged_at_step"] is None and abl["diverged_at_step"] is None
    assert max(_errors(wn)) <= 1e-3 and max(_errors(abl)) <= 1e-3
    assert wn["steps"] - wn["checks"] - wn["fallback_steps"] > 0
