"""Solid masks on the GPU: equivalences that hold bit for bit (an empty mask,
solid layers as a mask), obstacle flows against the oracle at FP64 and FP32,
a square duct, and one step of the benchmarked slit with an obstacle against
one oracle step."""
import numpy as np
import pytest

import oracle
from paper_0712_2247_amd import hslb, workloads

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def test_empty_mask_and_mask_layers_reproduce_the_slit_fp64():
    shape = (20, 16, 16)
    nb = workloads.number_density(0.2, 4)
    n, u = workloads.random_state(shape, nb, 0.05, 1e-3, seed=1, solid_lo=2, solid_hi=2)
    kw = dict(accel=(1e-5, 0.0, 0.0), precision="f64")
    slit = hslb.Sim(16, 16, 20, 4, 0.9, wall_lo=2, wall_hi=2, **kw)
    slit.init(n, u)
    empty = hslb.Sim(16, 16, 20, 4, 0.9, wall_lo=2, wall_hi=2, **kw)
    empty.set_solid(np.zeros(shape))
    empty.init(n, u)
    m = np.zeros(shape, dtype=np.uint8)
    m[:2] = 1
    m[-2:] = 1
    box = hslb.Sim(16, 16, 20, 4, 0.9, **kw)
    box.set_solid(m)
    box.init(n, u)
    for s in (slit, empty, box):
        s.step(20)
    f = slit.get_populations()
    assert np.array_equal(empty.get_populations(), f)
    fb = box.get_populations()
    print(f"mask layers vs walls: max difference {np.abs(fb - f).max():.3e}", flush=True)
    assert np.array_equal(fb, f)


CASES = [  # (nx, ny, nz, sigma, walls, solid fraction, precision-independent seed)
    (14, 12, 16, 4, 0, 0.06, 3),
    (16, 16, 24, 6, 3, 0.04, 4),     # whole x-rows per block
    (12, 13, 18, 3, 2, 0.10, 5),
]


def _obstacles(case):
    nx, ny, nz, sigma, walls, frac, seed = case
    rng = np.random.default_rng(seed)
    m = (rng.uniform(size=(nz, ny, nx)) < frac).astype(np.uint8)
    n, u = workloads.random_state((nz, ny, nx), workloads.number_density(0.2, sigma), 0.05, 1e-3,
                                  seed=seed + 10, solid_lo=walls, solid_hi=walls)
    n[m == 1] = 0.0
    u[:, m == 1] = 0.0
    return m, n, u


def _pair(case, precision, **kw):
    nx, ny, nz, sigma, walls, frac, seed = case
    g = hslb.Sim(nx, ny, nz, sigma, 0.9, accel=(2e-5, 0.0, 0.0), wall_lo=walls, wall_hi=walls,
                 precision=precision, **kw)
    o = oracle.Oracle(nx, ny, nz, sigma=sigma, tau=0.9, accel=(2e-5, 0.0, 0.0), wall_lo=walls,
                      wall_hi=walls, **kw)
    return g, o


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:5])))
def test_obstacles_fp64(case):
    print(f"case {case}", flush=True)
    m, n, u = _obstacles(case)
    g, o = _pair(case, "f64")
    g.set_solid(m)
    o.set_solid(m)
    g.init(n, u)
    o.init(n, u)
    Fg, Fo = g.force(), o.force()
    assert np.abs(Fg - Fo).max() <= 1e-13 * np.abs(Fo).max()
    g.step(30)
    o.step(30)
    assert _rel(g.get_populations(), o.get_populations()) <= 1e-13
    gn, _ = g.moments()
    assert np.all(gn[m == 1] == 0.0)


@pytest.mark.parametrize("case", CASES[:2], ids=lambda c: "x".join(map(str, c[:5])))
def test_obstacles_fp32(case):
    """FP32 storage: solid nodes hold exact zeros (FP32-representable
    references) and 300 steps stay within 1e-5 of the FP64 oracle."""
    m, n, u = _obstacles(case)
    g, o = _pair(case, "f32")
    g.set_solid(m)
    o.set_solid(m)
    g.init(n, u)
    o.init(n, u)
    g.step(300)
    o.step(300)
    gn, gu = g.moments()
    on, ou = o.moments()
    assert np.all(gn[m == 1] == 0.0) and np.all(gu[:, m == 1] == 0.0)
    assert _rel(gn, on) <= 1e-5 and _rel(gu, ou) <= 1e-5
    assert abs(gn.sum() - n.sum()) <= 1e-6 * n.sum()


def test_square_duct_against_oracle():
    """Stokes flow in a square duct whose side walls are mask nodes (force
    off, 4 x 22 x 22, 500 steps), FP64 against the oracle."""
    H = 20
    m = np.zeros((H + 2, H + 2, 4), dtype=np.uint8)
    m[0], m[-1], m[:, 0], m[:, -1] = 1, 1, 1, 1
    n = np.full(m.shape, 0.01)
    n[m == 1] = 0.0
    kw = dict(accel=(1e-6, 0.0, 0.0), force_mode=hslb.HSLB_FORCE_OFF)
    g = hslb.Sim(4, H + 2, H + 2, 4, 1.0, precision="f64", **kw)
    o = oracle.Oracle(4, H + 2, H + 2, 4, 1.0, **kw)
    g.set_solid(m)
    o.set_solid(m)
    g.init(n)
    o.init(n)
    g.step(500)
    o.step(500)
    assert _rel(g.get_populations(), o.get_populations()) <= 1e-13


def test_full_size_obstacle_one_step():
    """The benchmarked 64x64x136 slit (sigma 8, FP32) with a cylinder of radius
    8 across y and the wall factor off (the oracle's wall factor is a brute
    force search): one GPU step from a developed state against one oracle step
    from the same populations."""
    wl = workloads.slit_64_f32_stable()
    n, u = wl.fields()
    z, x = np.meshgrid(np.arange(wl.nz), np.arange(wl.nx), indexing="ij")
    cyl = ((z - wl.nz / 2) ** 2 + (x - wl.nx / 2) ** 2 <= 64)
    m = np.broadcast_to(cyl[:, None, :], (wl.nz, wl.ny, wl.nx)).astype(np.uint8)
    g = hslb.Sim.from_workload(wl, wall_reg=0)
    g.set_solid(m)
    g.init(n, u)
    g.step(200)
    f = g.get_populations()
    o = oracle.Oracle(**wl.params(), wall_reg=0)
    o.set_solid(m)
    o.init(n, u)
    o.set_populations(f)
    g2 = hslb.Sim.from_workload(wl, wall_reg=0)
    g2.set_solid(m)
    g2.init(n, u)
    g2.set_populations(f)
    g2.step(1)
    o.step(1)
    fg, fo = g2.get_populations(), o.get_populations()
    assert np.all(np.isfinite(fg))
    assert _rel(fg, fo) <= 1e-6
    gn, _ = g2.moments()
    assert np.all(gn[m == 1] == 0.0)


def test_set_solid_errors():
    g = hslb.Sim(12, 12, 16, 4, 1.0, wall_lo=2, wall_hi=2)
    g.init(np.full((16, 12, 12), 0.005))
    with pytest.raises(hslb.HslbError) as ei:
        g.set_solid(np.zeros((16, 12, 12)))
    assert ei.value.code == hslb.HSLB_ESTATE
    s = hslb.Sim(32, 32, 16, 4, 1.0, wall_lo=2, wall_hi=2, force_mode=hslb.HSLB_FORCE_SURROGATE)
    with pytest.raises(hslb.HslbError) as ei:
        s.set_solid(np.zeros((16, 32, 32)))
    assert ei.value.code == hslb.HSLB_EINVAL


def test_obstacles_with_attraction_fp64():
    """Obstacles and the mean-field attraction together (12 x 13 x 18 slit,
    sigma 3, 10 % solid, attraction range 1.5): 30 FP64 steps against the
    oracle."""
    case = CASES[2]
    m, n, u = _obstacles(case)
    g, o = _pair(case, "f64", att_eps=0.05, att_range=1.5)
    g.set_solid(m)
    o.set_solid(m)
    g.init(n, u)
    o.init(n, u)
    g.step(30)
    o.step(30)
    assert _rel(g.get_populations(), o.get_populations()) <= 1e-13
    gn, _ = g.moments()
    assert np.all(gn[m == 1] == 0.0)
