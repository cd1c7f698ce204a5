"""Host-side logic of the validation reruns (no GPU): the closed forms of the
Fig. 1 caption and the reduction of a velocity profile to its near-wall
drop."""
import math

import numpy as np
import pytest

from paper_0712_2247_amd import experiments as ex


def test_viscosity_closed_forms_limits():
    # low density: g2 -> 1, LHP ~ (4/15) n*^2, Enskog's collisional part
    # ~ (5/16) pi^(-1/2) 0.8 (2 pi / 3) n*
    ns = 1e-4
    r = ex.viscosity_closed_forms(ns)
    assert r["lhp_printed"] == pytest.approx(4 / 15 * ns ** 2, rel=1e-3)
    assert r["enskog"] == pytest.approx(5 / 16 / math.sqrt(math.pi) * 0.8 * 2 * math.pi / 3 * ns, rel=1e-3)
    for ns in (0.064, 0.256, 0.512, 0.609, 0.8):
        r = ex.viscosity_closed_forms(ns)
        assert r["lhp_sqrt_pi"] / r["lhp_printed"] == pytest.approx(math.sqrt(math.pi), rel=1e-15)
        # the ordering the Fig. 1 caption describes
        assert r["lhp_sqrt_pi"] < r["enskog"]
    # the closure at packing 0 and the paper's density map
    assert ex.g2_paper(0.0) == 1.0
    assert ex.eta_of(0.512) == pytest.approx(0.2680825731, rel=1e-9)


def test_near_wall_drop():
    z = np.arange(40) + 0.5
    par = z * (40 - z)
    assert ex.near_wall_drop(par) == 0.0
    bump = par.copy()
    bump[3] = par[10]      # a local maximum at layer 3, then a fall to par[4]
    assert ex.near_wall_drop(bump) == pytest.approx((par[10] - par[4]) / par.max())
    # the same bump at the other wall counts the same
    assert ex.near_wall_drop(bump[::-1]) == pytest.approx(ex.near_wall_drop(bump))


def test_mean_field_eos_and_binodal():
    """The closed-form excess chemical potential of the printed closure's EOS
    against quadrature of (Z - 1)/eta, the critical point (dP = d2P = 0), and
    the binodal's equal pressure and chemical potential."""
    from scipy.integrate import quad
    for eta in (0.05, 0.2, 0.35):
        ex_mu = quad(lambda e: (ex.compressibility_Z(e) - 1.0) / e, 0.0, eta)[0]
        closed = ex.mean_field_betamu(eta, 0.0) - math.log(eta) - ex.compressibility_Z(eta) + 1.0
        assert closed == pytest.approx(ex_mu, rel=1e-10)
    ec, Ac = ex.mean_field_critical()
    h = 1e-4
    P = lambda e: ex.mean_field_pressure(e, Ac)  # noqa: E731
    assert abs((P(ec + h) - P(ec - h)) / (2 * h)) < 1e-6
    assert abs((P(ec + h) - 2 * P(ec) + P(ec - h)) / h ** 2) < 1e-3
    assert ex.mean_field_binodal(0.95 * Ac) is None
    for q in (1.02, 1.1, 1.5):
        v, l = ex.mean_field_binodal(q * Ac)
        assert v < ec < l
        A = q * Ac
        assert ex.mean_field_pressure(v, A) == pytest.approx(ex.mean_field_pressure(l, A), rel=1e-8, abs=1e-12)
        assert ex.mean_field_betamu(v, A) == pytest.approx(ex.mean_field_betamu(l, A), rel=1e-8, abs=1e-10)
    # the attraction's A from its depth and lattice sum
    assert ex.mean_field_A(2.0, 1.5, 4) == pytest.approx(
        2.0 * ex.att_lattice_sum(1.5) / 2 * 6 / (math.pi * 64) * 3, rel=1e-14)
