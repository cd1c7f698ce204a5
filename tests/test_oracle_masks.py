"""Pins of the oracle's solid masks against what their definition fixes:

  - an empty mask changes nothing, and solid layers given as a mask in a
    periodic box reproduce the wall layers of a slit (the same bounce-back,
    the same wall factor from the distance to the nearest solid node centre
    minus half a spacing), bit for bit;
  - an obstacle conserves mass;
  - pressure-driven flow through a square duct whose side walls are mask
    nodes (hard-sphere force off) approaches the series solution of the
    Stokes problem in a rectangle, u = sum over odd n of
    (16 g a^2 / (nu pi^3 n^3)) (-1)^((n-1)/2) [1 - cosh(n pi z / 2a) /
    cosh(n pi b / 2a)] cos(n pi y / 2a), with the walls halfway between the
    last fluid and the first solid node."""
import math

import numpy as np

import oracle
from paper_0712_2247_amd import workloads


def test_empty_mask_and_mask_walls_reproduce_the_slit():
    shape = (20, 10, 12)
    nb = workloads.number_density(0.2, 4)
    n, u = workloads.random_state(shape, nb, 0.05, 1e-3, seed=1, solid_lo=2, solid_hi=2)
    kw = dict(accel=(1e-5, 0.0, 0.0))
    slit = oracle.Oracle(12, 10, 20, 4, 0.9, wall_lo=2, wall_hi=2, **kw)
    slit.init(n, u)
    empty = oracle.Oracle(12, 10, 20, 4, 0.9, wall_lo=2, wall_hi=2, **kw)
    empty.set_solid(np.zeros(shape))
    empty.init(n, u)
    m = np.zeros(shape, dtype=np.uint8)
    m[:2] = 1
    m[-2:] = 1
    box = oracle.Oracle(12, 10, 20, 4, 0.9, **kw)
    box.set_solid(m)
    box.init(n, u)
    for o in (slit, empty, box):
        o.step(20)
    f = slit.get_populations()
    assert np.array_equal(empty.get_populations(), f)
    assert np.array_equal(box.get_populations(), f)


def test_obstacle_conserves_mass():
    shape = (16, 12, 14)
    rng = np.random.default_rng(3)
    m = (rng.uniform(size=shape) < 0.08).astype(np.uint8)
    n, u = workloads.random_state(shape, workloads.number_density(0.2, 4), 0.05, 1e-3, seed=2)
    n[m == 1] = 0.0
    o = oracle.Oracle(14, 12, 16, 4, 0.9, accel=(2e-5, 0.0, 0.0))
    o.set_solid(m)
    o.init(n, u)
    m0 = o.moments()[0].sum()
    o.step(40)
    nn, uu = o.moments()
    assert abs(nn.sum() - m0) <= 1e-13 * m0
    assert np.all(nn[m == 1] == 0.0) and np.all(uu[:, m == 1] == 0.0)
    assert np.abs(uu).max() < 0.05        # a bounded flow around the obstacles


def test_square_duct_flow_matches_the_series_solution():
    H, tau, g = 20, 1.0, 1e-6
    ny = nz = H + 2
    m = np.zeros((nz, ny, 1), dtype=np.uint8)
    m[0], m[-1], m[:, 0], m[:, -1] = 1, 1, 1, 1
    n0 = 0.01
    n = np.full((nz, ny, 1), n0)
    n[m == 1] = 0.0
    o = oracle.Oracle(1, ny, nz, 4, tau, accel=(g, 0.0, 0.0), force_mode=oracle.FORCE_OFF)
    o.set_solid(m)
    o.init(n)
    o.step(6000)
    _, u = o.moments()
    ux = u[0, 1:-1, 1:-1, 0]
    nu = (tau - 0.5) / 3.0
    a = b = H / 2.0
    c = np.arange(H) + 0.5 - H / 2.0            # node positions from the duct axis
    Y, Z = np.meshgrid(c, c, indexing="xy")
    ref = np.zeros_like(Y)
    for k in range(1, 80, 2):
        ref += ((-1) ** ((k - 1) // 2) / k ** 3 * (1 - np.cosh(k * math.pi * Z / (2 * a)) / np.cosh(k * math.pi * b / (2 * a)))
                * np.cos(k * math.pi * Y / (2 * a)))
    ref *= 16 * g * a * a / (nu * math.pi ** 3)
    err = np.abs(ux - ref).max() / ref.max()
    assert err < 5e-3, err
    # the profile is symmetric under the duct's reflections
    assert np.abs(ux - ux.T).max() <= 1e-12 * ux.max()
