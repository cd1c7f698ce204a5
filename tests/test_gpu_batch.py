"""Batched ensemble of slits on the GPU: the persistent, graph-replayed batch
path against the single-lattice path and against the FP64 oracle, slit by
slit.

The ensemble starts from laterally uniform density and rest, so every slit
stays uniform in x and y: the oracle runs it as a 1 x 1 x nz column, which by
the definitions (periodic wrapping of every lateral offset) computes exactly
the same profiles as the 16 x 16 x nz slit.
"""
import os

import numpy as np
import pytest

from paper_0712_2247_amd import hslb, workloads

pytestmark = pytest.mark.gpu


def rel(a, b):
    b = np.asarray(b)
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ensemble_columns.npz")


def _oracle_columns(run):
    """The oracle's profiles of the ensemble slits run as laterally uniform
    columns (tests/golden/ensemble_columns.npz, written by make_golden.py
    from the oracle alone): {slit: (n_z, u_z with u_x filled, divergence step
    or None)}.  run: "small" (12 slits, 1000 steps, plain start), "eps1" /
    "eps2" (every slit, 10000 steps, start perturbed by 1e-9 / 2e-9 sin z)."""
    g = np.load(GOLDEN)
    idx = g["small_index"] if run == "small" else np.arange(len(g["nz"]))
    out = {}
    for i, k in enumerate(idx):
        nz = int(g["nz"][k])
        pn = g[f"{run}_n"][i, :nz]
        pu = np.zeros((3, nz))
        pu[0] = g[f"{run}_ux"][i, :nz]
        d = int(g[f"{run}_div"][i])
        out[int(k)] = (pn, pu, None if d < 0 else d)
    return out


SMALL = [0, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144]   # the stored "small" run


def test_batch_matches_single_lattice_and_oracle():
    steps = 1000
    wls = [workloads.ensemble()[k].with_size(steps=steps) for k in SMALL]
    print("sigmas", [w.sigma for w in wls], "nz", [w.nz for w in wls], flush=True)
    b = hslb.Batch(wls)
    b.init_all()
    b.step(steps)
    fin = b.finite()
    ref = _oracle_columns("small")
    assert sorted(ref) == SMALL
    for i, k in enumerate(SMALL):
        pn, pu = b.profiles(i)
        on, ou, _ = ref[k]
        o_fin = bool(np.isfinite(on).all() and np.isfinite(ou).all())
        assert bool(fin[i]) == o_fin, (k, fin[i], o_fin)
        if o_fin:
            assert rel(pn, on) <= 1e-5 and rel(pu[0], ou[0]) <= 1e-5, k
    # the same slits one by one through the single-lattice path
    for i in (0, 3, 7):
        w = wls[i]
        g = hslb.Sim.from_workload(w)
        hslb.hslb_set_watchdog(g.ctx, 0, 0.0)   # slit 3 diverges; only finite slits are compared
        n, u = w.fields()
        g.init(n, u)
        g.step(steps)
        sn, su = g.profiles()
        pn, pu = b.profiles(i)
        if fin[i]:
            assert rel(pn, sn) <= 1e-12 and rel(pu[0], su[0]) <= 1e-12


def test_batch_ragged_planes_match_single_lattice():
    """Cross sections whose planes are not multiples of 256 nodes (10x12:
    one partial chunk per layer; 24x20: one full and one partial) and lateral
    noise: the batch reproduces the single-lattice path node for node."""
    base = [workloads.ensemble()[k] for k in (1, 2, 5)]
    wls = [base[0].with_size(nx=10, ny=12, noise=0.01, steps=50),
           base[1].with_size(nx=24, ny=20, noise=0.01, steps=50),
           base[2].with_size(nx=16, ny=16, noise=0.01, steps=50)]
    b = hslb.Batch(wls)
    b.init_all()
    b.step(50)
    for i, w in enumerate(wls):
        g = hslb.Sim.from_workload(w)
        n, u = w.fields()
        g.init(n, u)
        g.step(50)
        sn, su = g.profiles()
        pn, pu = b.profiles(i)
        assert np.isfinite(sn).all()
        assert rel(pn, sn) <= 1e-12 and rel(pu[0], su[0]) <= 1e-12, (i, rel(pn, sn), rel(pu[0], su[0]))


def test_lane_shared_shell_reads_match_loaded_ones():
    """Where x-rows are whole 16-lane rows (a batch whose slits are all 16 wide)
    or whole waves (a 64-wide single lattice), lanes take shell reads that
    another lane of the row loads from that lane; the other path loads every
    read.  16-wide slits whose planes are not multiples of 64 nodes (waves
    straddle layers) against the single-lattice path, and a 64 x 18 single
    lattice (a partial last chunk of 128 nodes per layer) against the batch
    path, which loads every read for a 64-wide slit."""
    base = [workloads.ensemble()[k] for k in (1, 2, 5)]   # sigma 4, 3, 8
    wls = [base[0].with_size(nx=16, ny=12, noise=0.01, steps=40),
           base[1].with_size(nx=16, ny=20, noise=0.01, steps=40),
           base[2].with_size(nx=16, ny=12, noise=0.01, steps=40)]
    print("16-wide batch", [(w.ny, w.sigma) for w in wls], flush=True)
    b = hslb.Batch(wls)
    b.init_all()
    b.step(40)
    for i, w in enumerate(wls):
        g = hslb.Sim.from_workload(w)
        n, u = w.fields()
        g.init(n, u)
        g.step(40)
        sn, su = g.profiles()
        pn, pu = b.profiles(i)
        assert np.isfinite(sn).all()
        assert rel(pn, sn) <= 1e-12 and rel(pu[0], su[0]) <= 1e-12, (i, rel(pn, sn), rel(pu[0], su[0]))
    for w in (base[0].with_size(nx=64, ny=18, noise=0.01, steps=40),
              base[2].with_size(nx=64, ny=18, noise=0.01, steps=40)):
        print("64-wide single lattice", w.ny, w.sigma, flush=True)
        b = hslb.Batch([w])
        b.init_all()
        b.step(40)
        g = hslb.Sim.from_workload(w)
        n, u = w.fields()
        g.init(n, u)
        g.step(40)
        sn, su = g.profiles()
        pn, pu = b.profiles(0)
        assert np.isfinite(sn).all()
        assert rel(pn, sn) <= 1e-12 and rel(pu[0], su[0]) <= 1e-12, (rel(pn, sn), rel(pu[0], su[0]))


def test_batch_graph_and_eager_agree_and_autotune_restores_state():
    wls = [workloads.ensemble()[k].with_size(steps=60) for k in SMALL[:6]]
    a = hslb.Batch(wls)
    a.init_all()
    a.step(40)
    before = [a.profiles(i) for i in range(len(wls))]
    choice, us = a.autotune(steps=10)
    assert 0 <= choice < 12 and (us > 0).all()
    after = [a.profiles(i) for i in range(len(wls))]
    for (p0, u0), (p1, u1) in zip(before, after):
        assert np.array_equal(p0, p1) and np.array_equal(u0, u1)
    b = hslb.Batch(wls)
    hslb.hslb_set_graph(b.ctx, False)
    b.init_all()
    for _ in range(40):
        b.step(1)
    for i in range(len(wls)):
        assert np.array_equal(a.profiles(i)[0], b.profiles(i)[0])


def test_autotune_cache_round_trip(tmp_path, monkeypatch):
    """With HSLB_TUNE_CACHE set, the first autotune times the 12 launch
    configurations and stores the fastest; a second batch of the same slits
    applies it without timing; a different slit list is timed again."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("HSLB_TUNE_CACHE", str(cache))
    wls = [workloads.ensemble()[k].with_size(steps=60) for k in SMALL[:6]]
    a = hslb.Batch(wls)
    a.init_all()
    choice, us = a.autotune(steps=4)
    assert 0 <= choice < 12 and (us > 0).all()
    launch = hslb.hslb_batch_get_launch(a.ctx)
    text = cache.read_text()
    assert text.startswith("{") and "hslb-batch-v1|" in text and '"collide_grid": %d' % launch[1] in text
    b = hslb.Batch(wls)
    b.init_all()
    choice2, us2 = b.autotune(steps=4)
    assert choice2 == -1 and us2[0] == pytest.approx(us[choice], rel=1e-3)
    assert hslb.hslb_batch_get_launch(b.ctx) == launch
    c = hslb.Batch(wls[:5])
    c.init_all()
    choice3, _ = c.autotune(steps=4)
    assert choice3 >= 0 and text != cache.read_text()
    # the state after a cached or timed tuning steps as an untuned batch
    ref = hslb.Batch(wls)
    ref.init_all()
    for bb in (a, b, ref):
        bb.step(20)
    for i in range(len(wls)):
        assert np.array_equal(a.profiles(i)[0], ref.profiles(i)[0])
        assert np.array_equal(b.profiles(i)[0], ref.profiles(i)[0])


# Both sides start from the ensemble's uniform density times 1 + EPS sin(z):
# the paired shell sum of the GPU path is exactly antisymmetric under the
# mirror z -> nz-1-z, so without a common seed an unstable mirror-antisymmetric
# mode would grow on the oracle (whose summation order breaks the symmetry at
# the level of rounding) but never on the GPU.
EPS = 1e-9


def test_ensemble_512_slits_against_oracle():
    """The full ensemble: 512 slits, 16x16 cross section, H in 10..60,
    sigma in {3,4,5,6,8}, packing in [0.10, 0.40], 10000 steps in one batch.

    A slit the oracle sees diverge within 5000 steps (from the seeded start and
    from one seeded twice as strongly) diverges on the GPU too.  Slower divergence grows
    from rounding noise, so its timing -- and the verdict at 10000 steps --
    depends on the noise and is only reported.  A slit that stays finite and
    whose final state is unique (doubling the seed moves the oracle's
    profiles by at most 1e-6) agrees with the oracle to 1e-5.  Beyond the bulk
    stability limit of the closure some finite slits settle into layered
    states that the noise selects (the second oracle run lands elsewhere);
    those are reported, not compared."""
    wls = workloads.ensemble()
    b = hslb.Batch(wls)
    for k, w in enumerate(wls):
        n, u = w.fields()
        b.init(k, n * (1.0 + EPS * np.sin(np.arange(w.nz)))[:, None, None], u)
    choice, us = b.autotune(steps=10)
    print(f"autotune choice {choice}: {np.round(us, 1)} us/step", flush=True)
    b.step(10000)
    fin = b.finite()
    print(f"{fin.sum()} of {len(wls)} slits finite", flush=True)
    ref = _oracle_columns("eps1")      # start perturbed by EPS sin z
    pert = _oracle_columns("eps2")     # by 2 EPS sin z
    worst, compared, selected, marginal, diverged = 0.0, 0, [], [], 0
    for k, w in enumerate(wls):
        on, ou, div = ref[k]
        pn2, pu2, div2 = pert[k]
        if div is not None and div2 is not None and max(div, div2) <= 5000:
            # a fast instability: it must show on the GPU as well
            assert not fin[k], (k, w.sigma, w.eta, div)
            diverged += 1
            continue
        if div is not None or div2 is not None:
            marginal.append(k)  # slow growth from noise: the verdict depends on it
            continue
        assert fin[k], (k, w.sigma, w.eta)
        if max(rel(pn2, on), rel(pu2[0], ou[0])) > 1e-6:
            selected.append(k)
            continue
        pn, pu = b.profiles(k)
        e = max(rel(pn, on), rel(pu[0], ou[0]))
        worst = max(worst, e)
        compared += 1
        assert e <= 1e-5, (k, w.sigma, w.eta, e)
    print(f"{compared} slits compared to 1e-5 (worst {worst:.2e}); {diverged} diverge fast in both; "
          f"{len(selected)} finite slits with noise-selected states: {selected}; "
          f"{len(marginal)} diverging slowly from noise: {marginal}", flush=True)
    assert compared >= 300
