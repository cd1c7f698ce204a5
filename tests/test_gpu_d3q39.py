"""The third-order 39-velocity lattice on the GPU against the oracle: FP64
steps (periodic boxes and slits, the hard-sphere force, the attraction, force
off with a driving field, the narrowest slit and the smallest periodic box),
the force and moment readouts, population and checkpoint round trips, and at
the benchmarked 64x64x136 slit's size two steps against two oracle steps, and
the graph-replayed and eager steps (isothermal and thermal) bit for bit."""
import numpy as np
import pytest

import oracle
from paper_0712_2247_amd import hslb, workloads

pytestmark = pytest.mark.gpu

# (nx, ny, nz, sigma, walls, force_mode, att_range)
CASES = [
    (10, 9, 12, 4, 0, hslb.HSLB_FORCE_EXACT, 0.0),     # periodic box
    (12, 11, 16, 3, 2, hslb.HSLB_FORCE_EXACT, 0.0),    # slit
    (8, 8, 7, 2, 2, hslb.HSLB_FORCE_EXACT, 0.0),       # 3 fluid layers: links of length 3 reach the far wall plane
    (12, 12, 18, 4, 3, hslb.HSLB_FORCE_EXACT, 1.5),    # with the attraction
    (6, 5, 12, 4, 1, hslb.HSLB_FORCE_OFF, 0.0),        # force off, driven
    (3, 3, 5, 2, 0, hslb.HSLB_FORCE_OFF, 0.0),         # smallest periodic box
    (16, 16, 24, 6, 3, hslb.HSLB_FORCE_EXACT, 0.0),    # 256 nodes per layer
    (14, 13, 20, 5, 3, hslb.HSLB_FORCE_EXACT, 0.0),    # odd sigma: half-integer axis midpoints
    (16, 16, 22, 7, 0, hslb.HSLB_FORCE_EXACT, 0.0),    # sigma 7, periodic, fused row sums
]
TOL = 1e-12   # FP64 against the FP64 oracle


def _ids(c):
    return "x".join(map(str, c[:5])) + ("-off" if c[5] == hslb.HSLB_FORCE_OFF else "") + \
        (f"-att{c[6]}" if c[6] else "")


def _pair(case, accel=(2e-5, 0.0, 0.0)):
    nx, ny, nz, sigma, walls, fm, lam = case
    kw = dict(accel=accel, wall_lo=walls, wall_hi=walls, force_mode=fm,
              att_eps=0.05 if lam else 0.0, att_range=lam)
    g = hslb.Sim(nx, ny, nz, sigma, 0.9, precision="f64", lattice=hslb.HSLB_D3Q39, **kw)
    o = oracle.Oracle(nx, ny, nz, sigma=sigma, tau=0.9, lattice=39, **kw)
    return g, o


def _state(case, seed):
    nx, ny, nz, sigma, walls, fm, lam = case
    nb = workloads.number_density(0.2, max(sigma, 2))
    return workloads.random_state((nz, ny, nx), nb, 0.05, 5e-3, seed=seed, solid_lo=walls, solid_hi=walls)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_steps_fp64(case):
    print(f"case {case}", flush=True)
    n, u = _state(case, seed=31)
    g, o = _pair(case)
    g.init(n, u)
    o.init(n, u)
    assert _rel(g.get_populations(), o.get_populations()) <= 1e-15
    g.step(30)
    o.step(30)
    fg, fo = g.get_populations(), o.get_populations()
    err = _rel(fg, fo)
    print(f"30 steps: relative difference {err:.3e}", flush=True)
    assert err <= TOL
    gn, gu = g.moments()
    on, ou = o.moments()
    assert np.abs(gn - on).max() <= TOL * on.max()
    assert np.abs(gu - ou).max() <= 1e-10 * max(np.abs(ou).max(), 1e-12)
    gp, gv = g.profiles()
    op, ov = o.profiles()
    assert np.abs(gp - op).max() <= TOL * op.max()


@pytest.mark.parametrize("case", [CASES[0], CASES[1], CASES[3]], ids=_ids)
def test_force_readout(case):
    n, u = _state(case, seed=32)
    g, o = _pair(case)
    g.init(n, u)
    o.init(n, u)
    Fg, Fo = g.force(), o.force()
    assert np.abs(Fg - Fo).max() <= 1e-13 * np.abs(Fo).max()


def test_population_and_checkpoint_round_trips():
    case = CASES[1]
    nx, ny, nz, sigma, walls, fm, lam = case
    n, u = _state(case, seed=33)
    g, _ = _pair(case)
    g.init(n, u)
    g.step(5)
    f = g.get_populations()
    assert f.shape == (39, nz, ny, nx)
    assert np.all(f[:, :walls] == 0.0) and np.all(f[:, nz - walls:] == 0.0)
    # set_populations zeroes the wall layers and keeps the rest as given
    f2 = f.copy()
    f2[:, 0] = 1.0
    g.set_populations(f2)
    assert np.array_equal(g.get_populations(), f)
    blob = hslb.hslb_checkpoint_save(g.ctx)
    g.step(7)
    a = g.get_populations()
    hslb.hslb_checkpoint_load(g.ctx, blob)
    g.step(7)
    assert np.array_equal(g.get_populations(), a)
    # a 19-velocity context of the same grid refuses the checkpoint
    h = hslb.Sim(nx, ny, nz, sigma, 0.9, wall_lo=walls, wall_hi=walls, precision="f64")
    h.init(n, u)
    with pytest.raises(hslb.HslbError) as ei:
        hslb.hslb_checkpoint_load(h.ctx, blob)
    assert ei.value.code == hslb.HSLB_EINVAL


def test_mask_rejected():
    g = hslb.Sim(12, 12, 16, 4, 1.0, wall_lo=2, wall_hi=2, lattice=hslb.HSLB_D3Q39)
    with pytest.raises(hslb.HslbError) as ei:
        g.set_solid(np.zeros((16, 12, 12)))
    assert ei.value.code == hslb.HSLB_EINVAL


def test_full_size_two_steps():
    """The benchmarked 64x64x136 slit (sigma 8, packing 0.25, tau 0.8) on the
    39-velocity lattice in FP64: two GPU steps from the workload's initial state
    against two oracle steps, every population."""
    wl = workloads.slit_64_f32_stable()
    n, u = wl.fields()
    g = hslb.Sim.from_workload(wl, precision="f64", lattice=hslb.HSLB_D3Q39)
    g.init(n, u)
    g.step(2)
    o = oracle.Oracle(**wl.params(), lattice=39)
    o.init(n, u)
    o.step(2)
    fg, fo = g.get_populations(), o.get_populations()
    err = _rel(fg, fo)
    print(f"64x64x136, 2 steps: relative difference {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.parametrize("thermal", [0, 1])
def test_graph_and_eager_steps_agree_and_watchdog_passes(thermal):
    """The captured graphs (16-step and 2-step) and the eager launches run the
    same kernels in the same order: 11 steps with the watchdog on (mass and
    finiteness every 4 steps, through the 39-velocity profile kernel), then 35
    without it, give populations identical to eager stepping."""
    case = CASES[6]
    nx, ny, nz, sigma, walls, fm, lam = case
    n, u = _state(case, seed=34)
    kw = dict(accel=(2e-5, 0.0, 0.0), wall_lo=walls, wall_hi=walls, precision="f64",
              lattice=hslb.HSLB_D3Q39, thermal=thermal)
    T = None
    if thermal:
        T = (2.0 / 3.0) * (1.0 + 0.03 * np.random.default_rng(35).uniform(-1, 1, size=(nz, ny, nx)))
    a = hslb.Sim(nx, ny, nz, sigma, 0.9, **kw)
    b = hslb.Sim(nx, ny, nz, sigma, 0.9, **kw)
    hslb.hslb_set_graph(b.ctx, False)
    hslb.hslb_set_watchdog(a.ctx, 4, 1e-10)
    for s in (a, b):
        s.init(n, u, T)
        s.step(11)
    assert hslb.hslb_step_count(a.ctx) == 11
    assert np.array_equal(a.get_populations(), b.get_populations())
    # without the watchdog's 4-step chunks: 16-step graphs, a 2-step graph and
    # an eager step (35 = 2 x 16 + 2 + 1)
    hslb.hslb_set_watchdog(a.ctx, 0, 1e-10)
    a.step(35)
    b.step(35)
    assert np.array_equal(a.get_populations(), b.get_populations())
