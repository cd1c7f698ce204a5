"""Pins of the oracle's non-isothermal terms (the temperature term of C^(1) and
the energy source C^(2), on the 39-velocity lattice) against what the
mathematics and kinetic theory fix, independent of the oracle's own code:

  - the thermal equilibrium has the Maxwellian's moments through third order at
    (n, u, T), and the temperature read back is the one put in;
  - C^(1) and C^(2) on a small slit against the brute-force evaluator of
    tests/_bruteforce.py (its own geometry, no tables);
  - a uniform state at any temperature feels no force and no energy source;
    at rest, the density and temperature terms of C^(1) conserve momentum;
  - long waves: C^(1) = -grad p_c and C^(2) = lambda_c lap T for a temperature
    wave, C^(2) = -p_c div u for a compression, with Enskog's collisional
    pressure p_c = (2 pi / 3) sigma^3 n^2 g2 T and collisional conductivity
    lambda_c = (2/3) sqrt(pi) n^2 sigma^4 g2 v_T;
  - energy: a step adds exactly sum (F.u + C^(2)); with the force off a closed
    box keeps its energy; a temperature wave at uniform pressure decays at the
    BGK diffusivity T0 (tau - 1/2)."""
import math

import numpy as np
import pytest

import oracle
from paper_0712_2247_amd import workloads

from tests import _bruteforce as bf

T0 = 2.0 / 3.0


def _energy(o):
    c, _ = oracle.lattice_q(39)
    return 0.5 * float(np.tensordot((c ** 2).sum(1).astype(float), o.get_populations(), axes=(0, 0)).sum())


def test_thermal_equilibrium_moments():
    rng = np.random.default_rng(1)
    shape = (3, 2, 3)
    n = rng.uniform(0.5, 1.5, size=shape)
    u = rng.uniform(-0.1, 0.1, size=(3,) + shape)
    T = T0 * rng.uniform(0.8, 1.2, size=shape)
    o = oracle.Oracle(3, 2, 3, 4, 0.8, force_mode=oracle.FORCE_OFF, lattice=39, thermal=1)
    o.init(n, u, T)
    f = o.get_populations()
    c = oracle.lattice_q(39)[0].astype(float)
    d = np.eye(3)
    for idx in np.ndindex(shape):
        fi = f[(slice(None),) + idx]
        ui, Ti, ni = u[(slice(None),) + idx], T[idx], n[idx]
        assert fi.sum() == pytest.approx(ni, rel=1e-14)
        assert np.abs(c.T @ fi - ni * ui).max() < 1e-14
        P = np.einsum("ia,ib,i->ab", c, c, fi)
        assert np.abs(P - ni * (Ti * d + np.outer(ui, ui))).max() < 1e-14
        Q = np.einsum("ia,ib,ig,i->abg", c, c, c, fi)
        Qm = ni * (Ti * (np.einsum("a,bg->abg", ui, d) + np.einsum("b,ag->abg", ui, d) + np.einsum("g,ab->abg", ui, d))
                   + np.einsum("a,b,g->abg", ui, ui, ui))
        assert np.abs(Q - Qm).max() < 1e-14
    Tb, _ = o.thermal_fields()
    assert np.abs(Tb - T).max() < 1e-14


def test_force_and_energy_source_against_brute_force():
    nx, ny, nz, sig = 6, 5, 10, 2
    rng = np.random.default_rng(1)
    n, u = workloads.random_state((nz, ny, nx), workloads.number_density(0.2, sig), 0.1, 5e-3, seed=2,
                                  solid_lo=2, solid_hi=2)
    T = T0 * (1 + 0.1 * rng.uniform(-1, 1, size=(nz, ny, nx)))
    o = oracle.Oracle(nx, ny, nz, sig, 0.9, wall_lo=2, wall_hi=2, lattice=39, thermal=1)
    o.init(n, u, T)
    To, Qo = o.thermal_fields()
    Fo = o.force()
    nn, uu = o.moments()
    Fb, Qb = bf.thermal_force(bf.Grid(nn, nn[None] * uu, sig, wall_lo=2, wall_hi=2), To)
    assert np.abs(Fo - Fb).max() <= 1e-13 * np.abs(Fb).max()
    assert np.abs(Qo - Qb).max() <= 1e-13 * np.abs(Qb).max()


def test_uniform_state_and_momentum_at_rest():
    o = oracle.Oracle(8, 8, 8, 3, 0.9, lattice=39, thermal=1)
    o.init(np.full((8, 8, 8), workloads.number_density(0.3, 3)), None, np.full((8, 8, 8), 0.8))
    T, Q = o.thermal_fields()
    assert np.abs(o.force()).max() <= 1e-15 and np.abs(Q).max() <= 1e-15
    nx, ny, nz, sig = 10, 9, 12, 4
    rng = np.random.default_rng(4)
    n, _ = workloads.random_state((nz, ny, nx), workloads.number_density(0.2, sig), 0.05, 0.0, seed=3)
    T = T0 * (1 + 0.05 * rng.uniform(-1, 1, size=(nz, ny, nx)))
    o = oracle.Oracle(nx, ny, nz, sig, 0.9, lattice=39, thermal=1)
    o.init(n, None, T)
    F = o.force()
    assert np.abs(F.sum(axis=(1, 2, 3))).max() <= 1e-13 * np.abs(F).max()


def _long_wave(sig=4, L=128, eta=0.25):
    nb = workloads.number_density(eta, sig)
    G = oracle.g2(math.pi * sig ** 3 * nb / 6)
    z = np.arange(L)
    return nb, G, z, 2 * math.pi / L


def test_long_wave_temperature_gradient():
    sig = 4
    nb, G, z, k = _long_wave(sig)
    eps = 1e-3
    Tz = T0 * (1 + eps * np.cos(k * z))
    o = oracle.Oracle(4, 4, len(z), sig, 1.0, lattice=39, thermal=1)
    o.init(np.full((len(z), 4, 4), nb), None, np.broadcast_to(Tz[:, None, None], (len(z), 4, 4)).copy())
    _, Q = o.thermal_fields()
    F = o.force()
    lam = 2.0 / 3.0 * math.sqrt(math.pi) * nb ** 2 * sig ** 4 * G * math.sqrt(T0)
    want_Q = -lam * k * k * T0 * eps * np.cos(k * z)               # lambda_c d2T/dz2
    want_F = (2 * math.pi / 3) * sig ** 3 * nb ** 2 * G * T0 * eps * k * np.sin(k * z)   # -d p_c / dz
    proj = lambda a, b: float(a @ b) / float(b @ b)  # noqa: E731
    # the face-diagonal points are interpolated between lattice corners: ~1 % at sigma 4
    assert proj(Q[:, 0, 0], want_Q) == pytest.approx(1.0, abs=0.02)
    assert proj(F[2, :, 0, 0], want_F) == pytest.approx(1.0, abs=0.01)
    assert np.abs(F[:2]).max() <= 1e-12 * np.abs(F[2]).max()


def test_long_wave_compression_work():
    sig = 4
    nb, G, z, k = _long_wave(sig)
    L = len(z)
    u = np.zeros((3, L, 4, 4))
    u[2] = 1e-4 * np.sin(k * z)[:, None, None]
    o = oracle.Oracle(4, 4, L, sig, 1.0, lattice=39, thermal=1)
    o.init(np.full((L, 4, 4), nb), u)
    _, Q = o.thermal_fields()
    pc = 2 * math.pi / 3 * sig ** 3 * nb ** 2 * G * T0
    want = -pc * 1e-4 * k * np.cos(k * z)                        # -p_c du_z/dz
    assert float(Q[:, 0, 0] @ want) / float(want @ want) == pytest.approx(1.0, abs=0.01)


def test_energy_bookkeeping():
    nx, ny, nz, sig = 10, 9, 12, 4
    rng = np.random.default_rng(5)
    n, u = workloads.random_state((nz, ny, nx), workloads.number_density(0.2, sig), 0.05, 5e-3, seed=3)
    T = T0 * (1 + 0.05 * rng.uniform(-1, 1, size=(nz, ny, nx)))
    o = oracle.Oracle(nx, ny, nz, sig, 0.9, lattice=39, thermal=1, accel=(1e-5, 0, 0))
    o.init(n, u, T)
    E0 = _energy(o)
    _, Q = o.thermal_fields()
    F = o.force()
    _, uu = o.moments()
    gain = float(np.sum(F * uu) + Q.sum())
    o.step(1)
    assert _energy(o) - E0 == pytest.approx(gain, rel=1e-11)
    c = oracle.Oracle(nx, ny, nz, sig, 0.9, lattice=39, thermal=1, force_mode=oracle.FORCE_OFF)
    c.init(n, u, T)
    E0 = _energy(c)
    c.step(20)
    assert abs(_energy(c) - E0) <= 1e-14 * E0


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_temperature_wave_decays_at_the_bgk_diffusivity(tau):
    L, steps, eps = 64, 300, 1e-3
    k = 2 * math.pi / L
    z = np.arange(L)
    Tz = T0 * (1 + eps * np.cos(k * z))
    nz_ = 1.0 / (1 + eps * np.cos(k * z))                      # uniform pressure n T
    o = oracle.Oracle(3, 3, L, 4, tau, lattice=39, thermal=1, force_mode=oracle.FORCE_OFF)
    o.init(np.broadcast_to(nz_[:, None, None], (L, 3, 3)).copy(), None,
           np.broadcast_to(Tz[:, None, None], (L, 3, 3)).copy())
    o.step(steps)
    T, _ = o.thermal_fields()
    amp = (T[:, 0, 0] - T[:, 0, 0].mean()) @ np.cos(k * z) * 2 / L / (T0 * eps)
    assert -math.log(amp) / steps / (T0 * (tau - 0.5) * k * k) == pytest.approx(1.0, abs=0.02)


def test_rejections():
    with pytest.raises(ValueError):
        oracle.Oracle(6, 6, 8, 2, 0.9, thermal=1)                  # needs the 39-velocity lattice
    o = oracle.Oracle(6, 6, 8, 2, 0.9, wall_lo=1, wall_hi=1, lattice=39, thermal=1)
    with pytest.raises(ValueError):
        o.init(np.full((8, 6, 6), 0.01), None, np.full((8, 6, 6), -1.0))


@pytest.mark.parametrize("thermal,gamma", [(0, 1.0), (1, 5.0 / 3.0)])
def test_sound_speed_isothermal_and_adiabatic(thermal, gamma):
    """A density wave (force off, uniform T0 start) on the 39-velocity lattice:
    its velocity mode oscillates at c k with c^2 = T0 on the isothermal lattice
    and c^2 = 5 T0 / 3, the adiabatic value of a monatomic gas, once the energy
    equation is coupled.  (The density mode of the thermal lattice also carries
    the non-propagating entropy mode; the velocity mode does not.)"""
    L, eps = 64, 1e-4
    k = 2 * math.pi / L
    z = np.arange(L)
    o = oracle.Oracle(1, 1, L, 4, 0.8, lattice=39, thermal=thermal, force_mode=oracle.FORCE_OFF)
    o.init((1 + eps * np.cos(k * z))[:, None, None])
    v = []
    for _ in range(400):
        v.append(float(o.moments()[1][2, :, 0, 0] @ np.sin(k * z)))
        o.step(1)
    a = np.array(v)
    zc = [i + a[i] / (a[i] - a[i + 1]) for i in range(1, len(a) - 1) if a[i] * a[i + 1] < 0]
    assert len(zc) >= 8
    c = math.pi / ((zc[-1] - zc[0]) / (len(zc) - 1)) / k
    assert c == pytest.approx(math.sqrt(gamma * T0), rel=3e-3)
