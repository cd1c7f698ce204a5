"""The collide kernel with shell fields staged through LDS (hslb_set_collide_tiles)
against the default kernel with direct reads: both sum the same pair elements
in the same order with the same arithmetic, so the populations after several
steps must agree bit for bit.  Cases cover one tile row (ny = 4), odd and even
sigma, walls and periodic z, the non-temporal instance of lattices whose
populations exceed the last-level cache (with x-rows of 128 and 256 nodes,
whose direct kernel exchanges row-edge reads between waves), and a lattice the
staged kernel does not take (nx not a multiple of 64), where the switch must
change nothing."""
import numpy as np
import pytest

from paper_0712_2247_amd import hslb, workloads

pytestmark = pytest.mark.gpu


def _run(nx, ny, nz, sigma, walls, steps, tiles, seed, eta=0.25, att=0.0):
    nb = workloads.number_density(eta, sigma)
    n, u = workloads.random_state((nz, ny, nx), nb, 0.01, 2e-3, seed=seed, solid_lo=walls, solid_hi=walls)
    g = hslb.Sim(nx, ny, nz, sigma, 0.9, accel=(1e-5, -3e-6, 0.0), wall_lo=walls, wall_hi=walls, precision="f32",
                 att_eps=att, att_range=3.0 if att else 0.0)
    hslb.hslb_set_watchdog(g.ctx, 0, 0.0)
    hslb.hslb_set_collide_tiles(g.ctx, tiles)
    g.init(n, u)
    g.step(steps)
    f = g.get_populations()
    g.close()
    return f


@pytest.mark.parametrize("nx,ny,nz,sigma,walls,steps", [
    (64, 64, 136, 8, 4, 30),     # the benchmark slit's shape
    (128, 8, 24, 5, 0, 20),      # periodic, odd sigma
    (64, 4, 20, 2, 1, 20),       # one tile row, walls
    (64, 12, 18, 3, 2, 20),      # odd sigma, walls
    (128, 128, 136, 6, 0, 4),    # populations beyond the last-level cache
    (256, 64, 60, 5, 3, 3),      # beyond the cache, x-rows over four waves
    (48, 16, 20, 4, 2, 10),      # not tiled: the switch changes nothing
])
def test_staged_collide_is_bitwise_the_direct_one(nx, ny, nz, sigma, walls, steps):
    print(f"collide tiles case {nx}x{ny}x{nz} sigma {sigma} walls {walls}", flush=True)
    a = _run(nx, ny, nz, sigma, walls, steps, 1, seed=nx + ny + nz + sigma)
    b = _run(nx, ny, nz, sigma, walls, steps, 0, seed=nx + ny + nz + sigma)
    assert np.isfinite(a).all()
    assert np.array_equal(a, b), float(np.abs(a - b).max())


def test_staged_collide_with_the_attraction_is_bitwise_the_direct_one():
    """The mean-field attraction adds its force at the node after the shell
    sum; with it on, the staged and direct kernels still agree bit for bit."""
    a = _run(64, 8, 24, 6, 3, 20, 1, seed=77, att=2e-3)
    b = _run(64, 8, 24, 6, 3, 20, 0, seed=77, att=2e-3)
    assert np.isfinite(a).all()
    assert np.array_equal(a, b), float(np.abs(a - b).max())
