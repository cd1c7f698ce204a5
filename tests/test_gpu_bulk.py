"""The 256^3 periodic bulk (sigma 6, packing 0.25, tau 1, shear wave
u_x = 1e-3 sin(2 pi z / 256), Gaussian density noise 1e-3) on the GPU: its
layer-averaged modes against the oracle and the linear symbol.

The initial velocity depends on z only, so the layer means of the initial
equilibrium populations are the equilibrium of the layer-mean density: the
modes along z of the 3-D run evolve (to linear order, the lateral noise does
not feed them) as a 1 x 1 x 256 column of the oracle started from the layer
means.  The shear mode gives the viscosity the method predicts (symbol:
nu = (tau - 1/2)/3 + the discrete collisional part).

The noise leaves the layer-averaged density modes at ~1e-7 of the mean, below
what FP32 moment fields (6e-8 relative per node) and the second-order coupling
of the 3-D noise leave intact, so sound is measured on a deterministic wave of
amplitude 1e-4 (second test)."""
import math

import numpy as np
import pytest

import oracle
from oracle import symbol as sy
from paper_0712_2247_amd import hslb, workloads

pytestmark = pytest.mark.gpu


def modes(prof_n, prof_u, ms):
    nz = prof_n.size
    z = np.arange(nz)
    j = prof_u * prof_n[None]
    out = {}
    for m in ms:
        ph = np.exp(-2j * math.pi * m * z / nz)
        out[m] = ((prof_n * ph).sum() / nz, (j[0] * ph).sum() / nz, (j[2] * ph).sum() / nz)
    return out


def test_bulk_256_shear_mode_against_oracle_column_and_symbol():
    """The recipe's full 5000 steps.  The shear mode matches the oracle column
    to 1e-5 relative while it holds more than 5 % of its initial amplitude
    (steps 200, 600, 2000); by step 5000 it has decayed to 0.4 %, and there the
    bar is 1e-7 of the initial amplitude, the resolution of FP32 populations
    and fields (2^-24 per value, over thousands of steps).  The viscosity it
    decays with (200 -> 600, 600 -> 5000 steps) equals the oracle column's to
    1e-5 and the symbol's to 1e-4."""
    wl = workloads.bulk_256_f32()
    n, u = wl.fields()
    g = hslb.Sim.from_workload(wl)
    g.init(n, u)
    nl = n.mean(axis=(1, 2))
    o = oracle.Oracle(1, 1, wl.nz, sigma=wl.sigma, tau=wl.tau)
    o.init(nl[:, None, None], u[:, :, :1, :1])
    k = 2 * math.pi / wl.nz
    ms = (1, 3, 4)
    done = 0
    shear, oshear = {}, {}
    for t in (0, 200, 600, 2000, wl.steps):
        g.step(t - done)
        o.step(t - done)
        done = t
        gm = modes(*g.profiles(), ms)
        on, ou = o.profiles()
        om = modes(on, ou, ms)
        shear[t], oshear[t] = gm[1][1], om[1][1]
        e_shear = abs(gm[1][1] - om[1][1]) / abs(om[1][1])
        print(f"t {t}: shear mode {e_shear:.2e}, amplitude {abs(om[1][1]) / abs(oshear[0]):.2e} of the "
              f"initial (noise-level density mode |n_1| / n_b = {abs(om[1][0]) / wl.n_bulk:.1e})", flush=True)
        if abs(om[1][1]) >= 0.05 * abs(oshear[0]):
            assert e_shear <= 1e-5
        else:
            assert abs(gm[1][1] - om[1][1]) <= 1e-7 * abs(oshear[0])
    nu = -math.log(abs(shear[600] / shear[200])) / (400 * k * k)
    nu_late = -math.log(abs(shear[wl.steps] / shear[600])) / ((wl.steps - 600) * k * k)
    onu_late = -math.log(abs(oshear[wl.steps] / oshear[600])) / ((wl.steps - 600) * k * k)
    assert nu_late == pytest.approx(onu_late, rel=1e-5)
    nu_sym = sy.shear_nu(wl.nz, wl.sigma, wl.eta, wl.tau)
    c, gam = sy.sound(wl.nz, wl.sigma, wl.eta, wl.tau)
    print(f"bulk 256^3: nu measured {nu:.6f} (steps 200-600), {nu_late:.6f} (600-{wl.steps}), "
          f"symbol {nu_sym:.6f}; sound speed {c:.5f}, damping {gam:.3e} per step at k = 2 pi / 256",
          flush=True)
    assert nu == pytest.approx(nu_sym, rel=1e-4)
    assert nu_late == pytest.approx(nu_sym, rel=1e-4)


@pytest.mark.parametrize("steps", [3, 100])
def test_bulk_256_force_at_sampled_nodes_against_definition(steps):
    """The full-size 256^3 state after 3 and 100 steps: the GPU's hard-sphere
    force at 48 seeded nodes against a direct evaluation of equation (12) from
    its definition (tests/_bruteforce.py: distance tests for the smearing ball,
    each quadrature point placed at r + sigma s and spread bilinearly) on the
    same moments rounded to FP32.  The GPU also holds the coarse-grained
    density and the contact values in FP32, and in this nearly uniform state
    the force is 1e-3 to 1e-6 of the sum of the magnitudes of its terms: the
    difference stays within 2e-6 of that sum (a few dozen roundings of 2^-24)
    and below a twentieth of the largest sampled force."""
    from tests import _bruteforce as bf
    wl = workloads.bulk_256_f32()
    n, u = wl.fields()
    g = hslb.Sim.from_workload(wl)
    g.init(n, u)
    del n, u
    g.step(steps)
    F = g.force()
    n, u = g.moments()
    g.close()
    n32 = n.astype(np.float32).astype(np.float64)
    j32 = (u * n[None]).astype(np.float32).astype(np.float64)
    del u
    grid = bf.Grid(n32, j32, wl.sigma)
    rng = np.random.default_rng(4242)
    nodes = [tuple(int(v) for v in rng.integers(0, 256, 3)) for _ in range(48)]
    Fb, A = grid.force_at(nodes)
    Fg = np.array([[F[a, z, y, x] for (x, y, z) in nodes] for a in range(3)])
    err = np.abs(Fg - Fb)
    print(f"sampled force after {steps} steps: max |F| {np.abs(Fb).max():.3e}, max err {err.max():.3e}, "
          f"max err / term scale {(err / A).max():.3e}, max |F| / term scale {(np.abs(Fb) / A).max():.3e}",
          flush=True)
    assert np.all(err <= 2e-6 * A)
    assert err.max() <= 0.05 * np.abs(Fb).max()


def test_sound_wave_against_oracle_column_and_symbol():
    """64 x 64 x 128 periodic bulk, sigma 6, packing 0.25, tau 1, FP32, density
    n_b (1 + 1e-4 cos(2 pi z / 128)) plus +-1e-4 uniform noise: the density
    mode along z against the oracle column and the linear symbol, and the
    sound speed and damping it implies."""
    sigma, eta, tau, L = 6, 0.25, 1.0, 128
    nb = workloads.number_density(eta, sigma)
    n, u = workloads.random_state((L, 64, 64), nb, 1e-4, 0.0, seed=91)
    z = np.arange(L)
    n *= (1 + 1e-4 * np.cos(2 * math.pi * z / L))[:, None, None]
    g = hslb.Sim(64, 64, L, sigma, tau, precision="f32")
    g.init(n, u)
    nl = n.mean(axis=(1, 2))
    o = oracle.Oracle(1, 1, L, sigma=sigma, tau=tau)
    o.init(nl[:, None, None], np.zeros((3, L, 1, 1)))
    k = 2 * math.pi / L
    A = sy.amplification(np.array([0.0, 0.0, k]), sigma, eta, tau)
    f0 = nb * sy.W
    a0 = (o.get_populations()[:, :, 0, 0] - f0[:, None]) @ np.exp(-1j * k * z) / L
    done = 0
    series = []
    for t in (10, 20, 40, 80, 120):
        g.step(t - done)
        o.step(t - done)
        done = t
        gn = modes(*g.profiles(), (1,))[1][0]
        on = modes(*o.profiles(), (1,))[1][0]
        pred = (np.linalg.matrix_power(A, t) @ a0).sum()
        series.append((t, gn))
        e_o, e_s = abs(gn - on) / abs(on), abs(on - pred) / abs(pred)
        print(f"t {t}: density mode GPU vs oracle {e_o:.2e}, oracle vs symbol {e_s:.2e}", flush=True)
        assert e_o <= 1e-4 and e_s <= 1e-4
    c, gam = sy.sound(L, sigma, eta, tau)
    print(f"sound at k = 2 pi / {L}: speed {c:.5f}, amplitude damping {gam:.3e} per step "
          f"(continuum speed {math.sqrt(sy.VT2 * (1 + 2 * eta) ** 2 / (1 - eta) ** 4):.5f})", flush=True)
