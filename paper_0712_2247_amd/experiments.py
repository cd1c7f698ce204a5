"""Reruns of the paper's numerical validation (section "Numerical validation",
Figs. 1-4) on the engine.

Host orchestration only: every step runs in libhslb.so through ``hslb.Sim``;
this module sets up the runs, decides when a run has converged and reduces
the layer profiles the engine returns to the quantities the figures plot.
The closed forms the paper compares against (the Longuet-Higgins-Pople and
Enskog viscosities of the Fig. 1 caption, the Navier-Stokes parabola of
Fig. 4) are evaluated here for the report.

Units: lattice spacing, time step and particle mass 1, k_B T = v_T^2 = 1/3;
the sphere diameter sigma is an integer number of lattice spacings.  The
figures' reduced density is n* = n sigma^3; a slit of width L holds L fluid
layers between halfway bounce-back walls; the driving field is a force
per particle along x.  Every state is laterally uniform (no noise): a
16 x 16 lateral grid then carries the same layer profiles as an infinite one.

    python -m paper_0712_2247_amd.experiments --out results.json [--sigma 8]
"""
from __future__ import annotations

import argparse
import json
import math
import time
from typing import Dict, Sequence

import numpy as np

from . import hslb, workloads

VT2 = 1.0 / 3.0
LATERAL = 16


def g2_paper(eta: float) -> float:
    """Contact value of the pair correlation as the paper prints it
    (section "Methods and Results"); only the reference curves use it."""
    return (1.0 - eta / 2.0 + eta * eta / 4.0) / (1.0 - eta) ** 3


def eta_of(n_star: float) -> float:
    return math.pi * n_star / 6.0


def viscosity_closed_forms(n_star: float) -> Dict[str, float]:
    """Collisional shear viscosity in units of sqrt(m k_B T) / sigma^2:
    the Longuet-Higgins-Pople form as the Fig. 1 caption prints it, the same
    form with the sqrt(pi) that the current coupling 2/(v_T sqrt(pi)) of
    eq. (12) implies, and the collisional part of Enskog's viscosity from
    the same caption."""
    g = g2_paper(eta_of(n_star))
    lhp = 4.0 / 15.0 * g * n_star ** 2
    b = 2.0 * math.pi / 3.0 * n_star
    enskog = 5.0 / 16.0 / math.sqrt(math.pi) * (0.8 * b + 0.7737 * g * b * b)
    return {"lhp_printed": lhp, "lhp_sqrt_pi": math.sqrt(math.pi) * lhp, "enskog": enskog}


def _slit_sim(sigma: int, H: int, n_star: float, tau: float, g: float, precision: str):
    wl = workloads.slit(f"slit-H{H}-s{sigma}-n{n_star}", LATERAL, LATERAL, H, sigma, eta_of(n_star),
                        tau, g, 0, precision, 0, 0.0)
    s = hslb.Sim.from_workload(wl, precision=precision)
    n, u = wl.fields()
    s.init(n, u)
    return wl, s


def _run_to_steady(s, wl, key: str, block: int, max_steps: int, tol: float):
    """Steps in blocks until the largest change of the fluid layers' profile
    `key` ('n' or 'ux') over a block is below tol times its largest value."""
    fl = slice(wl.wall_lo, wl.nz - wl.wall_hi)
    prev = None
    done = 0
    change = math.inf
    while done < max_steps:
        s.step(block)
        done += block
        pn, pu = s.profiles()
        cur = (pn if key == "n" else pu[0])[fl].copy()
        if not np.isfinite(cur).all():
            raise RuntimeError(f"{wl.name}: non-finite profile after {done} steps")
        if prev is not None:
            change = float(np.abs(cur - prev).max() / np.abs(cur).max())
            if change < tol:
                break
        prev = cur
    return done, change


def _layer_velocity_midstep(s, wl) -> np.ndarray:
    """u_x of each fluid layer with half the step's force added to the current,
    (sum of j_x + F_x / 2) / (sum of n): the velocity of the second-order
    reading of the forcing, reported beside the unshifted one."""
    n, u = s.moments()
    F = s.force()
    fl = slice(wl.wall_lo, wl.nz - wl.wall_hi)
    jx = (n * u[0] + 0.5 * F[0])[fl].sum(axis=(1, 2))
    return jx / n[fl].sum(axis=(1, 2))


def near_wall_drop(u: np.ndarray) -> float:
    """Largest fall of u met when walking from a wall to the centre, in units
    of max u (0 for a profile rising monotonically from both walls)."""
    h = (u.size + 1) // 2
    best = 0.0
    for half in (u[:h], u[::-1][:h]):
        run = np.maximum.accumulate(half)
        best = max(best, float((run - half).max()))
    return best / float(np.abs(u).max())


def viscosity_sweep(n_stars: Sequence[float], sigma: int = 8, tau: float = 1.0, L: int = 256,
                    amp: float = 1e-4, precision: str = "f64", log=None) -> Dict:
    """Fig. 1: the collisional shear viscosity from the decay of a transverse
    wave u_x = amp sin(2 pi z / L) in a periodic box (16 x 16 x L).  The
    layer-averaged shear amplitude is read at t1 and t2 (the wave decays by
    about e between them) and nu = -ln(a2/a1) / ((t2 - t1) k^2); the BGK part
    (tau - 1/2)/3 is subtracted and the rest converted to the reduced
    viscosity eta* = n* nu_c / (sigma v_T)."""
    k = 2.0 * math.pi / L
    z = np.arange(L)
    ph = np.exp(-1j * k * z)
    rows = []
    for ns in n_stars:
        eta = eta_of(ns)
        nb = workloads.number_density(eta, sigma)
        ref = viscosity_closed_forms(ns)
        nu_guess = (tau - 0.5) / 3.0 + ref["lhp_sqrt_pi"] * sigma * math.sqrt(VT2) / ns
        t1 = max(20, int(0.1 / (nu_guess * k * k)))
        t2 = t1 + max(50, int(1.0 / (nu_guess * k * k)))
        s = hslb.Sim(LATERAL, LATERAL, L, sigma, tau, precision=precision)
        n0 = np.full((L, LATERAL, LATERAL), nb)
        u0 = np.zeros((3,) + n0.shape)
        u0[0] = (amp * np.sin(k * z))[:, None, None]
        s.init(n0, u0)
        amps = []
        done = 0
        for t in (t1, t2):
            s.step(t - done)
            done = t
            pn, pu = s.profiles()
            amps.append(abs(((pn * pu[0]) * ph).sum()) / L)
        s.close()
        nu = -math.log(amps[1] / amps[0]) / ((t2 - t1) * k * k)
        nu_c = nu - (tau - 0.5) / 3.0
        row = {"n_star": ns, "eta": eta, "t1": t1, "t2": t2, "nu": nu, "nu_c": nu_c,
               "eta_star": ns * nu_c / (sigma * math.sqrt(VT2)), **ref}
        rows.append(row)
        if log:
            log(f"fig1 n* {ns:.3f}: nu {nu:.5f}, eta* {row['eta_star']:.5f} (LHP x sqrt(pi) "
                f"{ref['lhp_sqrt_pi']:.5f}, printed LHP {ref['lhp_printed']:.5f}, Enskog {ref['enskog']:.5f})")
    return {"sigma": sigma, "tau": tau, "L": L, "amp": amp, "rows": rows}


def statics(n_stars: Sequence[float], L_over_sigma: int = 5, sigma: int = 8, tau: float = 1.0,
            precision: str = "f64", max_steps: int = 40000, log=None) -> Dict:
    """Fig. 2 (the lattice Boltzmann side): equilibrium density profiles of
    a slit of width L = 5 sigma without driving, from the uniform state at
    n* (the initial mean density).  Reports n(z)/n_b over the fluid layers,
    the contact value, and the largest deviation from the centre density
    near the walls (first quarter) and in the central half."""
    H = L_over_sigma * sigma
    rows = []
    for ns in n_stars:
        wl, s = _slit_sim(sigma, H, ns, tau, 0.0, precision)
        steps, change = _run_to_steady(s, wl, "n", 500, max_steps, 1e-11)
        pn, _ = s.profiles()
        s.close()
        fl = slice(wl.wall_lo, wl.nz - wl.wall_hi)
        r = pn[fl] / wl.n_bulk
        c = slice(H // 4, H - H // 4)
        nc = float(r[c].mean())
        q = H // 4
        dev_wall = float(max(np.abs(r[:q] - nc).max(), np.abs(r[-q:] - nc).max()))
        row = {"n_star": ns, "steps": steps, "last_change": change, "n_over_nb": r.tolist(),
               "contact": float(0.5 * (r[0] + r[-1])), "centre": nc, "dev_wall": dev_wall,
               "dev_centre": float(np.abs(r[c] - nc).max()), "std": float(r.std())}
        rows.append(row)
        if log:
            log(f"fig2 n* {ns:.3f}: {steps} steps, contact {row['contact']:.3f}, centre {nc:.3f}, "
                f"deviation near walls {dev_wall:.3f}, in the centre {row['dev_centre']:.3f}")
    return {"sigma": sigma, "tau": tau, "L_over_sigma": L_over_sigma, "rows": rows}


def _poiseuille_row(sigma, H, ns, tau, g, precision, max_steps):
    wl, s = _slit_sim(sigma, H, ns, tau, g, precision)
    steps, change = _run_to_steady(s, wl, "ux", 1000, max_steps, 1e-8)
    pn, pu = s.profiles()
    um = _layer_velocity_midstep(s, wl)
    s.close()
    fl = slice(wl.wall_lo, wl.nz - wl.wall_hi)
    n, u = pn[fl], pu[0][fl]
    zc = np.arange(H) + 0.5          # distance of each layer from the lower wall plane
    c = slice(H // 4, H - H // 4)
    p = np.polyfit(zc[c], u[c], 2)
    n_centre = float(n[H // 2 - 1:H // 2 + 1].mean())
    nsc = n_centre * sigma ** 3
    nu_ns = (tau - 0.5) / 3.0 + viscosity_closed_forms(nsc)["lhp_sqrt_pi"] * sigma * math.sqrt(VT2) / nsc
    u_ns = g / (2.0 * nu_ns) * zc * (H - zc)
    return {"n_star": ns, "H": H, "steps": steps, "last_change": change,
            "n_over_nb": (n / wl.n_bulk).tolist(), "ux": u.tolist(), "ux_midstep": um.tolist(),
            "u_mean": float((n * u).sum() / n.sum()), "u_max": float(u.max()),
            "near_wall_drop": near_wall_drop(u),
            "central_fit_resid": float(np.abs(u[c] - np.polyval(p, zc[c])).max() / u.max()),
            "nu_fit": float(-g / (2.0 * p[0])), "n_star_centre": nsc, "nu_ns": nu_ns,
            "u_ns": u_ns.tolist(),
            "ns_centre_offset": float((u[H // 2] - u_ns[H // 2]) / u_ns[H // 2])}


def poiseuille_density(n_stars: Sequence[float], L_over_sigma: int = 10, sigma: int = 8,
                       tau: float = 1.0, g: float = 2.4e-6, precision: str = "f64",
                       max_steps: int = 60000, log=None) -> Dict:
    """Fig. 3: steady streaming profiles u_x(z) of a slit of width L = 10
    sigma driven by a force g per particle along x, at several densities."""
    rows = []
    for ns in n_stars:
        row = _poiseuille_row(sigma, L_over_sigma * sigma, ns, tau, g, precision, max_steps)
        rows.append(row)
        if log:
            log(f"fig3 n* {ns:.3f}: {row['steps']} steps, mean u {row['u_mean']:.4e}, max u "
                f"{row['u_max']:.4e}, near-wall drop {row['near_wall_drop']:.3f}")
    return {"sigma": sigma, "tau": tau, "g": g, "L_over_sigma": L_over_sigma, "rows": rows}


def poiseuille_width(widths: Sequence[int], n_star: float = 0.512, sigma: int = 8, tau: float = 1.0,
                     g: float = 2.4e-6, precision: str = "f64", max_steps: int = 60000, log=None) -> Dict:
    """Fig. 4: steady streaming profiles at n* = 0.512 for slit widths
    L = widths x sigma, with the Navier-Stokes parabola g z (L - z) / (2 nu)
    (nu: the BGK part plus the collisional viscosity of eq. (12) at the
    centre density) and a quadratic fitted to the central half."""
    rows = []
    for w in widths:
        row = _poiseuille_row(sigma, w * sigma, n_star, tau, g, precision, max_steps)
        rows.append(row)
        if log:
            log(f"fig4 L {w} sigma: {row['steps']} steps, max u {row['u_max']:.4e}, near-wall drop "
                f"{row['near_wall_drop']:.3f}, central fit residual {row['central_fit_resid']:.2e}, "
                f"nu fit {row['nu_fit']:.4f} vs Navier-Stokes {row['nu_ns']:.4f}")
    return {"sigma": sigma, "tau": tau, "g": g, "n_star": n_star, "rows": rows}


# ------------------------------------------------- attraction: coexistence

def att_lattice_sum(att_range: float) -> float:
    """sum_o exp(-|o|^2 / range^2) over the cube |o_a| <= ceil(3 range)."""
    R = math.ceil(3.0 * att_range)
    m = np.arange(-R, R + 1, dtype=np.float64)
    return float(np.sum(np.exp(-m * m / att_range ** 2))) ** 3


def compressibility_Z(eta: float) -> float:
    """Compressibility factor of the printed closure: Z = 1 + 4 eta g2(eta) =
    (1 + eta + eta^2) / (1 - eta)^3."""
    return (1.0 + eta + eta * eta) / (1.0 - eta) ** 3


def mean_field_A(att_eps: float, att_range: float, sigma: int) -> float:
    """The attraction's pressure -(eps G0 / 2) n^2 (G0 the lattice sum) in the
    reduced form p pi sigma^3 / (6 k_B T) = eta Z(eta) - A eta^2."""
    return att_eps * att_lattice_sum(att_range) / 2.0 * 6.0 / (math.pi * sigma ** 3) / VT2


def mean_field_pressure(eta: float, A: float) -> float:
    return eta * compressibility_Z(eta) - A * eta * eta


def mean_field_betamu(eta: float, A: float) -> float:
    """beta mu up to a constant: ln eta + beta mu_ex + Z - 1 - 2 A eta, with
    beta mu_ex = int_0^eta (Z - 1)/e de = 3 / (2 (1 - eta)^2) - 3/2 - ln(1 - eta)
    for this Z."""
    return (math.log(eta) + 1.5 / (1.0 - eta) ** 2 - 1.5 - math.log(1.0 - eta)
            + compressibility_Z(eta) - 1.0 - 2.0 * A * eta)


def mean_field_critical():
    """(eta_c, A_c) where dP/d eta and d2P/d eta2 vanish."""
    from scipy.optimize import brentq
    d1 = lambda e, h=1e-6: (e + h) * compressibility_Z(e + h) - (e - h) * compressibility_Z(e - h)  # noqa: E731
    d2 = lambda e, h=1e-4: ((e + h) * compressibility_Z(e + h) - 2 * e * compressibility_Z(e)  # noqa: E731
                           + (e - h) * compressibility_Z(e - h)) / (h * h)
    eta_c = brentq(lambda e: d1(e) / (2e-6) / e - d2(e), 0.05, 0.3)
    return eta_c, d2(eta_c) / 2.0


def mean_field_binodal(A: float):
    """Coexisting packing fractions (vapour, liquid): equal pressure and
    chemical potential (the Maxwell construction of the mean-field EOS), by
    nested bisection between the spinodal points; None at or above the
    critical point."""
    from scipy.optimize import brentq
    eta_c, A_c = mean_field_critical()
    if A <= A_c * (1 + 1e-9):
        return None
    dP = lambda e, h=1e-7: (mean_field_pressure(e + h, A) - mean_field_pressure(e - h, A)) / (2 * h)  # noqa: E731
    s1 = brentq(dP, 1e-6, eta_c)        # spinodal, vapour side
    s2 = brentq(dP, eta_c, 0.6)         # spinodal, liquid side

    def vapour_at(eta_l):
        p = mean_field_pressure(eta_l, A)
        return brentq(lambda e: mean_field_pressure(e, A) - p, 1e-12, s1)

    def mismatch(eta_l):
        return mean_field_betamu(vapour_at(eta_l), A) - mean_field_betamu(eta_l, A)

    # liquid packings whose pressure lies within the vapour branch's range
    p_lo, p_hi = mean_field_pressure(1e-12, A), mean_field_pressure(s1, A)
    lo = brentq(lambda e: mean_field_pressure(e, A) - p_lo, s2, 0.7) if mean_field_pressure(s2, A) < p_lo else s2
    hi = brentq(lambda e: mean_field_pressure(e, A) - p_hi, s2, 0.7)
    span = hi - lo
    eta_l = brentq(mismatch, lo + 1e-9 * span, hi - 1e-9 * span)
    return float(vapour_at(eta_l)), float(eta_l)


def coexistence(quenches: Sequence[float], sigma: int = 4, tau: float = 1.0, att_range: float = 4.0,
                L: int = 128, precision: str = "f64", max_steps: int = 30000, log=None) -> Dict:
    """Liquid-vapour separation with the mean-field attraction: a periodic
    16 x 16 x L box at the critical packing of the mean-field EOS, attraction
    depth `quench` times its critical value, density n_c (1 + 0.02 cos(2 pi z/L)),
    run until the profile is steady.  Reports the plateau packings against
    the Maxwell construction of the same EOS."""
    eta_c, A_c = mean_field_critical()
    G0 = att_lattice_sum(att_range)
    eps_c = A_c * 2.0 * VT2 * math.pi * sigma ** 3 / 6.0 / G0
    n_c = workloads.number_density(eta_c, sigma)
    z = np.arange(L)
    rows = []
    for q in quenches:
        eps = q * eps_c
        s = hslb.Sim(LATERAL, LATERAL, L, sigma, tau, precision=precision, att_eps=eps, att_range=att_range)
        n0 = np.broadcast_to((n_c * (1.0 + 0.02 * np.cos(2.0 * math.pi * z / L)))[:, None, None],
                             (L, LATERAL, LATERAL)).copy()
        s.init(n0)
        prev, done, change = None, 0, math.inf
        while done < max_steps:
            s.step(1000)
            done += 1000
            pn, _ = s.profiles()
            if not np.isfinite(pn).all():
                raise RuntimeError(f"coexistence run at quench {q} diverged by step {done}")
            if prev is not None:
                change = float(np.abs(pn - prev).max() / pn.max())
                if change < 1e-10:
                    break
            prev = pn.copy()
        pn, pu = s.profiles()
        s.close()
        eta = pn * math.pi * sigma ** 3 / 6.0
        bi = mean_field_binodal(mean_field_A(eps, att_range, sigma))
        row = {"quench": q, "eps": eps, "steps": done, "last_change": change, "eta_profile": eta.tolist(),
               "eta_vapour": float(eta.min()), "eta_liquid": float(eta.max()),
               "binodal": bi, "max_u": float(np.abs(pu).max())}
        rows.append(row)
        if log:
            log(f"coexistence quench {q}: {done} steps, vapour {row['eta_vapour']:.4f} liquid "
                f"{row['eta_liquid']:.4f} (mean-field binodal {bi[0]:.4f} / {bi[1]:.4f})" if bi else
                f"coexistence quench {q}: {done} steps, packing {row['eta_vapour']:.4f}..{row['eta_liquid']:.4f}")
    return {"sigma": sigma, "tau": tau, "att_range": att_range, "L": L, "eta_c": eta_c, "eps_c": eps_c,
            "rows": rows}


FIG1_NSTARS = (0.064, 0.128, 0.192, 0.256, 0.32, 0.384, 0.448, 0.512, 0.576, 0.609)
FIG2_NSTARS = (0.256, 0.512, 0.609)
FIG3_NSTARS = (0.064, 0.128, 0.256, 0.384, 0.512)
FIG4_WIDTHS = (5, 10, 15, 20)


def basis_comparison(sigma: int = 4, eta: float = 0.25, H: int = 40, tau: float = 0.8, steps: int = 3000,
                     lateral: int = 8, log=print) -> Dict:
    """The question the paper attaches to the higher-order basis: does it make
    the wall factor unnecessary?  A static slit (no driving field, uniform
    start) on the 19- and 39-velocity lattices, with and without the wall
    factor, run to rest (`steps` steps, FP64).  Reported per run: the static
    current max |u_z| (the current the wall factor damps in the coupling term),
    its departure from the half-step current -F_z/(2n) of the first-order
    source, and the contact, maximum and minimum density of the profile
    relative to the bulk."""
    w = 2
    nz = H + 2 * w
    nb = workloads.number_density(eta, sigma)
    n = np.full((nz, lateral, lateral), nb)
    n[:w] = n[-w:] = 0.0
    rows = []
    for lat in (hslb.HSLB_D3Q19, hslb.HSLB_D3Q39):
        for reg in (1, 0):
            s = hslb.Sim(lateral, lateral, nz, sigma, tau, wall_lo=w, wall_hi=w, precision="f64", lattice=lat,
                         wall_reg=reg)
            s.init(n)
            s.step(steps)
            nn, uu = s.moments()
            F = s.force()
            s.close()
            fl = slice(w, nz - w)
            uz = uu[2, fl, 0, 0]
            half = -F[2, fl, 0, 0] / (2.0 * nn[fl, 0, 0])
            prof = nn[fl, 0, 0] / nb
            row = {"lattice": 39 if lat == hslb.HSLB_D3Q39 else 19, "wall_reg": reg,
                   "max_uz": float(np.abs(uz).max()), "halfstep_residual": float(np.abs(uz - half).max()),
                   "contact": float(prof[0]), "max": float(prof.max()), "min": float(prof.min()),
                   "profile": prof.tolist()}
            log(f"basis: {row['lattice']} velocities, wall factor {reg}: max|u_z| {row['max_uz']:.4g}, "
                f"|u_z + F_z/2n| {row['halfstep_residual']:.2e}, contact {row['contact']:.4f}, "
                f"min {row['min']:.4f}")
            rows.append(row)
    return {"sigma": sigma, "eta": eta, "H": H, "tau": tau, "steps": steps, "rows": rows}


def run_all(sigma: int = 8, log=print) -> Dict:
    t0 = time.perf_counter()
    out = {"fig1": viscosity_sweep(FIG1_NSTARS, sigma=sigma, log=log),
           "fig2": statics(FIG2_NSTARS, sigma=sigma, log=log),
           "fig3": poiseuille_density(FIG3_NSTARS, sigma=sigma, log=log),
           "fig4": poiseuille_width(FIG4_WIDTHS, sigma=sigma, log=log),
           "coexistence": coexistence((0.9, 1.05, 1.1), log=log),
           "basis": basis_comparison(log=log)}
    out["seconds"] = time.perf_counter() - t0
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--sigma", type=int, default=8)
    a = ap.parse_args(argv)
    res = run_all(a.sigma, log=lambda m: print(m, flush=True))
    with open(a.out, "w") as fh:
        json.dump(res, fh)
    print(f"wrote {a.out} ({res['seconds']:.1f} s)", flush=True)


if __name__ == "__main__":
    main()
