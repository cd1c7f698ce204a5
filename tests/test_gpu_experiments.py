"""The paper's numerical validation (section "Numerical validation", Figs.
1-4) rerun on the engine (sigma 8, tau 1, FP64).

The paper prints no data points, only curves and the observations it draws
from them, so these are reproductions, not parity: each test checks the
engine against the oracle or the linear symbol where those apply, and then
the paper's observations on the engine's own results:

  Fig. 1  the collisional viscosity equals the Longuet-Higgins-Pople form
          (with the sqrt(pi) the current coupling of eq. (12) implies) and
          lies below Enskog's;
  Fig. 2  the fluid is more inhomogeneous at higher density, with
          oscillations at the walls that fade toward the centre;
  Fig. 3  the mean streaming velocity falls as the density rises, and the
          profiles turn non-monotonic next to the walls at high density;
  Fig. 4  the centre of the slit follows a parabola with the bulk
          Navier-Stokes curvature, and the near-wall structure is stronger
          in narrower slits."""
import math

import numpy as np
import pytest

import oracle
from oracle import symbol as sy
from paper_0712_2247_amd import experiments as ex
from paper_0712_2247_amd import workloads

pytestmark = pytest.mark.gpu


def test_slit_profiles_against_oracle_column():
    """Fig. 3's densest slit (L = 10 sigma, n* = 0.512, g = 2.4e-6) on the
    16 x 16 lateral grid the experiments use, against a 1 x 1 oracle column
    (the state is laterally uniform), after 3000 steps."""
    sigma, H, ns = 8, 80, 0.512
    wl, s = ex._slit_sim(sigma, H, ns, 1.0, 2.4e-6, "f64")
    n, u = wl.fields()
    o = oracle.Oracle(**wl.with_size(nx=1, ny=1).params())
    o.init(n[:, :1, :1], u[:, :, :1, :1])
    s.step(3000)
    o.step(3000)
    gn, gu = s.profiles()
    s.close()
    on, ou = o.profiles()
    en = np.abs(gn - on).max() / np.abs(on).max()
    eu = np.abs(gu - ou).max() / np.abs(ou[0]).max()
    print(f"slit L = 10 sigma, n* 0.512, 3000 steps: profile differences n {en:.2e}, u {eu:.2e}", flush=True)
    assert en <= 1e-10 and eu <= 1e-10


def test_fig1_collisional_viscosity():
    res = ex.viscosity_sweep((0.128, 0.256, 0.512, 0.609))
    for r in res["rows"]:
        nu_sym = sy.shear_nu(res["L"], res["sigma"], r["eta"], res["tau"])
        ratio = r["eta_star"] / r["lhp_sqrt_pi"]
        print(f"n* {r['n_star']}: nu {r['nu']:.6f} (symbol {nu_sym:.6f}); eta* / LHP(sqrt pi) {ratio:.4f}, "
              f"eta* / printed LHP {r['eta_star'] / r['lhp_printed']:.4f}, eta* / Enskog "
              f"{r['eta_star'] / r['enskog']:.4f}", flush=True)
        assert r["nu"] == pytest.approx(nu_sym, rel=1e-4)
        assert 1.0 < ratio < 1.03
        assert r["eta_star"] < r["enskog"]


def test_fig2_statics():
    res = ex.statics(ex.FIG2_NSTARS)
    rows = res["rows"]
    for r in rows:
        print(f"n* {r['n_star']}: contact {r['contact']:.3f}, std {r['std']:.3f}, deviation near the "
              f"walls {r['dev_wall']:.3f}, in the centre {r['dev_centre']:.3f}", flush=True)
        assert r["last_change"] < 1e-11
        # oscillations fade toward the centre
        assert r["dev_centre"] < r["dev_wall"] / 3
        # the two walls are mirror images
        p = np.array(r["n_over_nb"])
        assert np.abs(p - p[::-1]).max() <= 1e-9 * p.max()
    # more inhomogeneous at higher density
    assert all(a["contact"] < b["contact"] and a["std"] < b["std"] for a, b in zip(rows, rows[1:]))


def test_fig3_density_sweep():
    res = ex.poiseuille_density(ex.FIG3_NSTARS)
    rows = res["rows"]
    for r in rows:
        print(f"n* {r['n_star']}: {r['steps']} steps, mean u {r['u_mean']:.4e}, near-wall drop "
              f"{r['near_wall_drop']:.3f}", flush=True)
        assert r["last_change"] < 1e-8
        # the unshifted velocity and the one with half the step's force added
        # differ where the layering makes C1_x large (a few percent of the
        # peak at the walls at n* = 0.512), far less in the centre
        d = np.abs(np.array(r["ux"]) - np.array(r["ux_midstep"])) / r["u_max"]
        print(f"   unshifted vs mid-step velocity: {d.max():.2e} (centre half {d[20:60].max():.2e})", flush=True)
        assert d.max() < 3e-2 and d[20:60].max() < 5e-3
    u_mean = [r["u_mean"] for r in rows]
    assert all(a > b for a, b in zip(u_mean, u_mean[1:]))
    drop = {r["n_star"]: r["near_wall_drop"] for r in rows}
    assert drop[0.064] == 0.0 and drop[0.128] == 0.0
    assert 0.0 < drop[0.256] < drop[0.384] < drop[0.512]
    assert drop[0.512] > 0.2


def test_fig4_width_sweep():
    res = ex.poiseuille_width(ex.FIG4_WIDTHS)
    rows = res["rows"]
    for r in rows:
        print(f"L {r['H'] // 8} sigma: near-wall drop {r['near_wall_drop']:.3f}, central fit residual "
              f"{r['central_fit_resid']:.2e}, nu fit {r['nu_fit']:.4f} vs Navier-Stokes {r['nu_ns']:.4f}, "
              f"centre velocity vs the no-slip parabola {r['ns_centre_offset']:+.2e}", flush=True)
        assert r["last_change"] < 1e-8
    drop = [r["near_wall_drop"] for r in rows]
    resid = [r["central_fit_resid"] for r in rows]
    assert all(a > b for a, b in zip(drop, drop[1:]))
    assert all(a > b for a, b in zip(resid, resid[1:]))
    assert rows[-1]["central_fit_resid"] < 5e-3
    # the central curvature is the bulk Navier-Stokes one
    for r in rows[2:]:
        assert r["nu_fit"] == pytest.approx(r["nu_ns"], rel=0.01)
    # the no-slip parabola misses the centre velocity by the near-wall
    # layer's apparent slip (the flow is faster), whose weight falls as the
    # slit widens
    off = [r["ns_centre_offset"] for r in rows]
    assert off[-1] > 0 and all(a > b for a, b in zip(off, off[1:]))


def test_higher_order_basis_and_the_static_current():
    """The paper names a larger Hermite basis as the alternative to the wall
    factor, which damps the coupling of the static current.  A static slit
    (sigma 4, packing 0.25, 40 layers, tau 0.8, 3000 steps) on both lattices,
    with and without the wall factor: the 39-velocity run against a 1 x 1
    oracle column, then what the runs show.  On 19 velocities the static
    current is exactly the half-step current -F_z/(2n) of the first-order
    source; on 39 velocities it is larger (the force carries k_B T = 2/3) and
    no longer exactly that; in both, dropping the wall factor enlarges it.  The
    larger basis alone does not remove it."""
    res = ex.basis_comparison()
    rows = {(r["lattice"], r["wall_reg"]): r for r in res["rows"]}
    # parity of one 39-velocity run with an oracle column (laterally uniform state)
    w, H, sigma = 2, res["H"], res["sigma"]
    nz = H + 2 * w
    nb = workloads.number_density(res["eta"], sigma)
    n = np.full((nz, 1, 1), nb)
    n[:w] = n[-w:] = 0.0
    o = oracle.Oracle(1, 1, nz, sigma, res["tau"], wall_lo=w, wall_hi=w, lattice=39, wall_reg=0)
    o.init(n)
    o.step(res["steps"])
    prof = o.profiles()[0][w:nz - w] / nb
    assert np.abs(np.array(rows[(39, 0)]["profile"]) - prof).max() <= 1e-10 * prof.max()
    for reg in (0, 1):
        assert rows[(19, reg)]["halfstep_residual"] <= 1e-12 * rows[(19, reg)]["max_uz"]
        assert rows[(39, reg)]["max_uz"] > 1.5 * rows[(19, reg)]["max_uz"]
        assert rows[(39, reg)]["halfstep_residual"] > 1e-3
    for lat in (19, 39):
        assert rows[(lat, 0)]["max_uz"] > rows[(lat, 1)]["max_uz"]
