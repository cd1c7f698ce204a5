"""The non-isothermal terms on the GPU (39-velocity lattice, FP64) against the
oracle: the temperature and energy-source readouts, 30 steps on periodic boxes
and slits (with the attraction, and with the force off under a driving field),
two steps of the benchmarked 64x64x136 slit, and the error paths."""
import math

import numpy as np
import pytest

import oracle
from paper_0712_2247_amd import hslb, workloads

pytestmark = pytest.mark.gpu

T0 = 2.0 / 3.0
TOL = 1e-12

# (nx, ny, nz, sigma, walls, force_mode, att_range)
CASES = [
    (10, 9, 12, 4, 0, hslb.HSLB_FORCE_EXACT, 0.0),
    (12, 11, 16, 3, 2, hslb.HSLB_FORCE_EXACT, 0.0),
    (12, 12, 18, 4, 3, hslb.HSLB_FORCE_EXACT, 1.5),
    (6, 5, 12, 4, 1, hslb.HSLB_FORCE_OFF, 0.0),
    (16, 16, 24, 6, 3, hslb.HSLB_FORCE_EXACT, 0.0),
    (14, 13, 20, 5, 3, hslb.HSLB_FORCE_EXACT, 0.0),
    (16, 16, 22, 7, 0, hslb.HSLB_FORCE_EXACT, 0.0),
]


def _ids(c):
    return "x".join(map(str, c[:5])) + ("-off" if c[5] == hslb.HSLB_FORCE_OFF else "") + \
        (f"-att{c[6]}" if c[6] else "")


def _pair(case, accel=(2e-5, 0.0, 0.0)):
    nx, ny, nz, sigma, walls, fm, lam = case
    kw = dict(accel=accel, wall_lo=walls, wall_hi=walls, force_mode=fm,
              att_eps=0.05 if lam else 0.0, att_range=lam)
    g = hslb.Sim(nx, ny, nz, sigma, 0.9, precision="f64", lattice=hslb.HSLB_D3Q39, thermal=1, **kw)
    o = oracle.Oracle(nx, ny, nz, sigma=sigma, tau=0.9, lattice=39, thermal=1, **kw)
    return g, o


def _state(case, seed):
    nx, ny, nz, sigma, walls, fm, lam = case
    n, u = workloads.random_state((nz, ny, nx), workloads.number_density(0.2, max(sigma, 2)), 0.05, 5e-3,
                                  seed=seed, solid_lo=walls, solid_hi=walls)
    rng = np.random.default_rng(seed + 100)
    T = T0 * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, size=(nz, ny, nx)))
    return n, u, T


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_thermal_fields_at_init(case):
    n, u, T = _state(case, seed=41)
    g, o = _pair(case)
    g.init(n, u, T)
    o.init(n, u, T)
    Tg, Qg = g.thermal_fields()
    To, Qo = o.thermal_fields()
    walls = case[4]
    fl = np.s_[walls:case[2] - walls] if walls else np.s_[:]
    assert np.abs(Tg[fl] - T[fl]).max() <= 1e-14
    assert np.abs(Tg - To).max() <= 1e-14
    if case[5] != hslb.HSLB_FORCE_OFF:
        assert np.abs(Qg - Qo).max() <= 1e-13 * np.abs(Qo).max()
    assert np.abs(g.force() - o.force()).max() <= 1e-13 * np.abs(o.force()).max()


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_thermal_steps_fp64(case):
    print(f"case {case}", flush=True)
    n, u, T = _state(case, seed=42)
    g, o = _pair(case)
    g.init(n, u, T)
    o.init(n, u, T)
    g.step(30)
    o.step(30)
    err = _rel(g.get_populations(), o.get_populations())
    print(f"30 thermal steps: relative difference {err:.3e}", flush=True)
    assert err <= TOL
    Tg, Qg = g.thermal_fields()
    To, Qo = o.thermal_fields()
    assert np.abs(Tg - To).max() <= TOL * To.max()
    if case[5] != hslb.HSLB_FORCE_OFF:
        # After 30 steps the temperature has nearly levelled out and C^(2) is a
        # small difference of terms of size sigma^2 4 pi n^2 g2 T0^(3/2)/sqrt(pi)
        # times relative temperature differences: its error is bounded by that
        # scale times the temperature's relative error, not by its own size.
        sigma = case[3]
        nmax = float(np.max(n))
        scale = sigma ** 2 * 4 * math.pi * nmax ** 2 * oracle.g2(math.pi * sigma ** 3 * nmax / 6) \
            * T0 ** 1.5 / math.sqrt(math.pi)
        assert np.abs(Qg - Qo).max() <= TOL * scale


def test_full_size_two_thermal_steps():
    """The benchmarked 64x64x136 slit (sigma 8, packing 0.25, tau 0.8) with a
    temperature varying by 2 % across the slit, two GPU steps against two
    oracle steps."""
    wl = workloads.slit_64_f32_stable()
    n, u = wl.fields()
    z = np.arange(wl.nz)
    T = np.broadcast_to((T0 * (1.0 + 0.02 * np.sin(2 * math.pi * z / wl.nz)))[:, None, None],
                        (wl.nz, wl.ny, wl.nx)).copy()
    g = hslb.Sim.from_workload(wl, precision="f64", lattice=hslb.HSLB_D3Q39, thermal=1)
    g.init(n, u, T)
    g.step(2)
    o = oracle.Oracle(**wl.params(), lattice=39, thermal=1)
    o.init(n, u, T)
    o.step(2)
    err = _rel(g.get_populations(), o.get_populations())
    print(f"64x64x136 thermal, 2 steps: relative difference {err:.3e}", flush=True)
    assert err <= TOL


def test_thermal_error_paths():
    g = hslb.Sim(12, 12, 16, 4, 1.0, wall_lo=2, wall_hi=2, lattice=hslb.HSLB_D3Q39)
    n = np.full((16, 12, 12), 0.005)
    with pytest.raises(hslb.HslbError) as ei:
        g.init(n, None, np.full((16, 12, 12), T0))
    assert ei.value.code == hslb.HSLB_ESTATE
    g.init(n)
    with pytest.raises(hslb.HslbError) as ei:
        g.thermal_fields()
    assert ei.value.code == hslb.HSLB_ESTATE
    t = hslb.Sim(12, 12, 16, 4, 1.0, wall_lo=2, wall_hi=2, lattice=hslb.HSLB_D3Q39, thermal=1)
    bad = np.full((16, 12, 12), T0)
    bad[5, 3, 3] = -0.1
    with pytest.raises(hslb.HslbError) as ei:
        t.init(n, None, bad)
    assert ei.value.code == hslb.HSLB_EINVAL
    # hslb_init on a thermal context starts at the lattice temperature
    t.init(n)
    Tg, Qg = t.thermal_fields()
    assert np.abs(Tg[2:14] - T0).max() <= 1e-14 and np.abs(Qg).max() <= 1e-15
