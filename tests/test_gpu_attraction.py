"""The optional mean-field attraction on the GPU against the oracle: the
potential (three separable passes on the GPU, a plain triple sum in the
oracle), the total force, FP64 and FP32 steps, and at the benchmarked slit's
size the potential at sampled nodes against direct sums."""
import math

import numpy as np
import pytest

import oracle
from paper_0712_2247_amd import hslb, workloads

pytestmark = pytest.mark.gpu

# (nx, ny, nz, sigma, walls, att_range, force_mode)
CASES = [
    (12, 11, 14, 2, 0, 1.5, hslb.HSLB_FORCE_EXACT),
    (10, 9, 20, 4, 2, 2.0, hslb.HSLB_FORCE_EXACT),
    (6, 8, 9, 3, 0, 2.5, hslb.HSLB_FORCE_EXACT),      # cube wider than the box: offsets wrap twice
    (16, 16, 24, 6, 3, 1.2, hslb.HSLB_FORCE_EXACT),   # whole x-rows per block (fused moments)
    (12, 12, 16, 4, 2, 2.0, hslb.HSLB_FORCE_OFF),     # attraction without the hard-sphere term
]
EPS = 0.05


def _pair(case, precision="f64", accel=(0.0, 0.0, 0.0)):
    nx, ny, nz, sigma, walls, lam, fm = case
    g = hslb.Sim(nx, ny, nz, sigma, 0.9, accel=accel, wall_lo=walls, wall_hi=walls, precision=precision,
                 force_mode=fm, att_eps=EPS, att_range=lam)
    o = oracle.Oracle(nx, ny, nz, sigma=sigma, tau=0.9, accel=accel, wall_lo=walls, wall_hi=walls,
                      force_mode=fm, att_eps=EPS, att_range=lam)
    return g, o


def _state(case, seed):
    nx, ny, nz, sigma, walls, lam, fm = case
    nb = workloads.number_density(0.2, max(sigma, 2))
    return workloads.random_state((nz, ny, nx), nb, 0.05, 2e-3, seed=seed, solid_lo=walls, solid_hi=walls)


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:6])))
def test_potential_and_force_fp64(case):
    print(f"case {case}", flush=True)
    n, u = _state(case, seed=11)
    g, o = _pair(case)
    g.init(n, u)
    o.init(n, u)
    pg, po = g.attraction_potential(), o.attraction_potential()
    # sums of up to 17^3 = 4913 terms in different orders: rounding reaches ~1e-14
    assert np.abs(pg - po).max() <= 1e-13 * np.abs(po).max()
    Fg, Fo = g.force(), o.force()
    # the attraction is a difference of two potentials: rounding of those
    # bounds its absolute error
    bound = 1e-13 * np.abs(Fo).max() + 1e-14 * n.max() * np.abs(po).max()
    assert np.abs(Fg - Fo).max() <= bound


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:6])))
def test_steps_fp64(case):
    print(f"case {case}", flush=True)
    n, u = _state(case, seed=12)
    g, o = _pair(case, accel=(1e-5, 0.0, 0.0))
    g.init(n, u)
    o.init(n, u)
    g.step(30)
    o.step(30)
    fg, fo = g.get_populations(), o.get_populations()
    assert np.linalg.norm(fg - fo) <= 1e-13 * np.linalg.norm(fo)


def test_slit_fp32_against_oracle():
    """FP32 storage, a 32x32x40 slit (sigma 8, packing 0.2, tau 0.9, +-5 %
    noise) with the attraction (range 3, eps 0.05), 300 steps: profiles and
    velocity field within 1e-5 of the FP64 oracle."""
    case = (32, 32, 40, 8, 4, 3.0, hslb.HSLB_FORCE_EXACT)
    n, u = _state(case, seed=13)
    g, o = _pair(case, precision="f32", accel=(2e-6, 0.0, 0.0))
    g.init(n, u)
    o.init(n, u)
    g.step(300)
    o.step(300)
    gp, gv = g.profiles()
    op, ov = o.profiles()
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)  # noqa: E731
    assert rel(gp, op) <= 1e-5 and rel(gv, ov) <= 1e-5
    gn, gu = g.moments()
    on, ou = o.moments()
    assert rel(gn, on) <= 1e-5 and rel(gu, ou) <= 1e-5


def test_full_size_potential_at_sampled_nodes():
    """The benchmarked 64x64x136 slit (sigma 8, FP32) with an attraction of
    range sigma (a 49^3 cube): the potential at 40 seeded nodes, fluid and
    wall layers, against direct sums over the FP32 density field the GPU
    reads."""
    wl = workloads.slit_64_f32_stable()
    lam = float(wl.sigma)
    n, u = wl.fields()
    g = hslb.Sim.from_workload(wl, att_eps=1e-3, att_range=lam)
    g.init(n, u)
    g.step(20)
    gn, _ = g.moments()
    phi = g.attraction_potential()
    n32 = gn.astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(21)
    nodes = [(int(rng.integers(0, wl.nz)), int(rng.integers(0, wl.ny)), int(rng.integers(0, wl.nx)))
             for _ in range(40)]
    ref = oracle.attraction_potential_at(n32, nodes, 1e-3, lam, zperiodic=False)
    got = np.array([phi[z, y, x] for z, y, x in nodes])
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()
    assert math.isfinite(float(np.abs(phi).max()))


def test_quench_against_oracle_column():
    """The coexistence run's box (16 x 16 x 128 periodic, sigma 4, tau 1,
    attraction range 4 at 1.05 times the critical depth), 300 steps into the
    separation, against a 1 x 1 x 128 oracle column (laterally uniform)."""
    from paper_0712_2247_amd import experiments as ex
    sigma, L, lam = 4, 128, 4.0
    eta_c, A_c = ex.mean_field_critical()
    eps = 1.05 * A_c * 2.0 * ex.VT2 * math.pi * sigma ** 3 / 6.0 / ex.att_lattice_sum(lam)
    n_c = workloads.number_density(eta_c, sigma)
    z = np.arange(L)
    col = n_c * (1.0 + 0.02 * np.cos(2.0 * math.pi * z / L))
    g = hslb.Sim(16, 16, L, sigma, 1.0, att_eps=eps, att_range=lam)
    g.init(np.broadcast_to(col[:, None, None], (L, 16, 16)).copy())
    o = oracle.Oracle(1, 1, L, sigma, 1.0, att_eps=eps, att_range=lam)
    o.init(col[:, None, None])
    g.step(300)
    o.step(300)
    gn, gu = g.profiles()
    on, ou = o.profiles()
    print(f"density contrast after 300 steps: {gn.max() / gn.min():.3f}", flush=True)
    assert gn.max() / gn.min() > 1.1      # well into the separation
    assert np.abs(gn - on).max() <= 1e-11 * on.max()
    assert np.abs(gu - ou).max() <= 1e-9 * np.abs(ou).max()


def test_phase_separation_reaches_mean_field_binodal():
    """Below the critical attraction the perturbed uniform state relaxes; above
    it the box separates into liquid and vapour slabs whose packings match the
    Maxwell construction of the mean-field EOS (hard-sphere Z of the printed
    closure minus the attraction's A eta^2) within 2 %."""
    from paper_0712_2247_amd import experiments as ex
    res = ex.coexistence((0.9, 1.05, 1.1))
    for r in res["rows"]:
        print(f"quench {r['quench']}: {r['steps']} steps, vapour {r['eta_vapour']:.4f}, liquid "
              f"{r['eta_liquid']:.4f}, binodal {r['binodal']}", flush=True)
    sub = res["rows"][0]
    assert sub["binodal"] is None and sub["eta_liquid"] - sub["eta_vapour"] < 1e-6
    for r in res["rows"][1:]:
        assert r["last_change"] < 1e-10
        v, l = r["binodal"]
        assert r["eta_vapour"] == pytest.approx(v, rel=0.02)
        assert r["eta_liquid"] == pytest.approx(l, rel=0.02)
