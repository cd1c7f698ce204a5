"""Pins of the oracle's mean-field attraction (the optional attractive term,
Phi = -eps (g * n) with Gaussian weights g and C1_att = -n grad Phi by
central differences), against what the definition fixes independently of
the oracle's triple sum:

  - a single density mode has the closed-form force -n(r) eps delta
    g_hat(k) sin(k_a) sin(k.r), with g_hat the product of three 1-D cosine
    sums (the Gaussian factorises over the axes);
  - a uniform periodic fluid feels no force, and the total force on any
    periodic state vanishes (g is even, so the pair sums cancel);
  - next to a wall the attraction pulls the fluid away from the wall, with
    mirror-symmetric layers in a symmetric slit;
  - the linear symbol with the attraction predicts the oracle's evolution of
    a small mode, and its sound speed tends to v_T^2 d(eta Z)/d eta minus
    eps n0 g_hat(0), the van der Waals term of the mean-field pressure
    -(eps g_hat(0)/2) n^2; the uniform state turns unstable once that speed
    squared is negative."""
import math

import numpy as np
import pytest

import oracle
from oracle import symbol as sy
from paper_0712_2247_amd import workloads


def _grid(shape):
    nz, ny, nx = shape
    return np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")


@pytest.mark.parametrize("shape,m,lam", [((8, 10, 12), (1, 2, 1), 1.5),
                                         ((6, 6, 20), (2, 1, 3), 2.0),
                                         ((4, 5, 7), (1, 1, 2), 1.2)])
def test_single_mode_closed_form(shape, m, lam):
    nz, ny, nx = shape
    k = 2 * math.pi * np.array([m[0] / nx, m[1] / ny, m[2] / nz])  # (kx, ky, kz)
    n0, delta, eps = 0.01, 0.002, 3e-3
    Z, Y, X = _grid(shape)
    phase = k[0] * X + k[1] * Y + k[2] * Z
    n = n0 + delta * np.cos(phase)
    o = oracle.Oracle(nx, ny, nz, 4, 1.0, force_mode=oracle.FORCE_OFF, att_eps=eps, att_range=lam)
    o.init(n)
    F = o.force()
    R = math.ceil(3 * lam)
    mm = np.arange(-R, R + 1)
    g1 = np.exp(-mm * mm / lam ** 2)
    ghat = np.prod([np.sum(g1 * np.cos(ka * mm)) for ka in k])
    # the force is a difference of two potentials of size eps n g_hat(0):
    # rounding of those sums bounds the absolute error
    round_bound = 1e-14 * n.max() * eps * n.max() * g1.sum() ** 3
    for a in range(3):
        ref = -n * eps * delta * ghat * math.sin(k[a]) * np.sin(phase)
        assert np.abs(F[a] - ref).max() <= 1e-12 * np.abs(ref).max() + round_bound, a
        if abs(math.sin(k[a])) > 0.1:
            assert np.abs(ref).max() > 1e3 * round_bound


def test_uniform_fluid_and_momentum_conservation():
    o = oracle.Oracle(9, 7, 8, 4, 1.0, force_mode=oracle.FORCE_OFF, att_eps=1e-2, att_range=1.7)
    o.init(np.full((8, 7, 9), 0.02))
    assert np.abs(o.force()).max() <= 1e-18
    n, _ = workloads.random_state((8, 7, 9), 0.02, 0.3, 0.0, seed=5)
    o.init(n)
    F = o.force()
    for a in range(3):
        assert abs(F[a].sum()) <= 1e-13 * np.abs(F[a]).sum()


def test_wall_pulls_fluid_into_the_slit():
    nz, w = 20, 2
    o = oracle.Oracle(6, 6, nz, 4, 1.0, wall_lo=w, wall_hi=w, force_mode=oracle.FORCE_OFF,
                      att_eps=1e-2, att_range=1.5)
    n = np.full((nz, 6, 6), 0.02)
    n[:w] = 0.0
    n[nz - w:] = 0.0
    o.init(n)
    F = o.force()
    fz = F[2, :, 0, 0]
    assert np.abs(F[0]).max() <= 1e-18 and np.abs(F[1]).max() <= 1e-18
    # away from the walls, toward the middle
    assert fz[w] > 0 and fz[nz - w - 1] < 0
    assert np.abs(fz + fz[::-1]).max() <= 1e-13 * np.abs(fz).max()
    # the middle of a wide enough slit is bulk-like: no force
    assert abs(fz[nz // 2 - 1]) <= 1e-3 * abs(fz[w])


def test_symbol_predicts_oracle_evolution_with_attraction():
    """A small density-and-current perturbation of a uniform periodic fluid
    (hard spheres and attraction on) evolves as A(k)^T a0 in the oracle."""
    sigma, eta, tau, lam, eps = 4, 0.2, 0.9, 1.5, 2.0
    shape = (10, 6, 8)
    nz, ny, nx = shape
    mvec = (1, 1, 1)
    k = 2 * math.pi * np.array([mvec[0] / nx, mvec[1] / ny, mvec[2] / nz])
    n0 = workloads.number_density(eta, sigma)
    Z, Y, X = _grid(shape)
    phase = k[0] * X + k[1] * Y + k[2] * Z
    n = n0 * (1 + 1e-6 * np.cos(phase))
    u = np.zeros((3,) + shape)
    u[0] = 1e-6 * np.sin(phase)
    o = oracle.Oracle(nx, ny, nz, sigma, tau, att_eps=eps, att_range=lam)
    o.init(n, u)
    _, w = oracle.lattice()
    f0 = (n0 * w)[:, None, None, None]
    ph = np.exp(-1j * phase)

    def fourier(f):
        return ((f - f0) * ph[None]).reshape(19, -1).sum(axis=1) / phase.size

    a0 = fourier(o.get_populations())
    A = sy.amplification(k, sigma, eta, tau, att_eps=eps, att_range=lam)
    # the mode decays by ~0.6 per step: after 10 steps it is still far above
    # the second-order terms of the 1e-6 perturbation
    T = 10
    o.step(T)
    pred = np.linalg.matrix_power(A, T) @ a0
    got = fourier(o.get_populations())
    assert np.linalg.norm(got - pred) <= 1e-6 * np.linalg.norm(pred)
    # and the attraction is visible at that level: without it the symbol is off
    A0 = sy.amplification(k, sigma, eta, tau)
    assert np.linalg.norm(got - np.linalg.matrix_power(A0, T) @ a0) > 1e-3 * np.linalg.norm(pred)


def test_symbol_sound_speed_and_spinodal():
    sigma, eta, tau, lam = 4, 0.2, 1.0, 2.0
    n0 = workloads.number_density(eta, sigma)
    c2_hs = sy.VT2 * (1 + 2 * eta) ** 2 / (1 - eta) ** 4      # printed closure (PY compressibility)
    g0 = sy.att_ghat([0.0, 0.0, 0.0], lam)
    eps_s = c2_hs / (n0 * g0)
    for frac in (0.25, 0.5, 0.75):
        c, _ = sy.sound(1024, sigma, eta, tau, att_eps=frac * eps_s, att_range=lam)
        assert c * c == pytest.approx(c2_hs - frac * eps_s * n0 * g0, rel=2e-4)
    assert sy.max_growth(64, sigma, eta, tau, axes="z", att_eps=0.5 * eps_s, att_range=lam) <= 1 + 1e-12
    assert sy.max_growth(64, sigma, eta, tau, axes="z", att_eps=1.1 * eps_s, att_range=lam) > 1.05
