"""The 256^3 periodic bulk (sigma 6, packing 0.25, tau 1, shear wave
u_x = 1e-3 sin(2 pi z / 256), Gaussian density noise 1e-3) on the GPU: its
layer-averaged modes against the oracle and the linear symbol.

The initial velocity depends on z only, so the layer means of the initial
equilibrium populations are the equilibrium of the layer-mean density: the
modes along z of the 3-D run evolve (to linear order, the lateral noise does
not feed them) as a 1 x 1 x 256 column of the oracle started from the layer
means.  The shear mode gives the viscosity the method predicts (symbol:
nu = (tau - 1/2)/3 + the discrete collisional part)."""
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


def test_bulk_256_modes_against_oracle_column_and_symbol():
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
    shear = {}
    for t in (200, 600):
        g.step(t - done)
        o.step(t - done)
        done = t
        gm = modes(*g.profiles(), ms)
        on, ou = o.profiles()
        om = modes(on, ou, ms)
        e_shear = abs(gm[1][1] - om[1][1]) / abs(om[1][1])
        e_dens = max(abs(gm[m][0] - om[m][0]) / abs(om[m][0]) for m in ms)
        print(f"t {t}: shear mode {e_shear:.2e}, density modes {e_dens:.2e} "
              f"(|n_1| / n_b = {abs(om[1][0]) / wl.n_bulk:.1e})", flush=True)
        assert e_shear <= 1e-5
        assert e_dens <= 1e-3
        shear[t] = gm[1][1]
    nu = -math.log(abs(shear[600] / shear[200])) / (400 * k * k)
    nu_sym = sy.shear_nu(wl.nz, wl.sigma, wl.eta, wl.tau)
    c, gam = sy.sound(wl.nz, wl.sigma, wl.eta, wl.tau)
    print(f"bulk 256^3: nu measured {nu:.6f}, symbol {nu_sym:.6f}; sound speed {c:.5f}, "
          f"damping {gam:.3e} per step at k = 2 pi / 256", flush=True)
    assert nu == pytest.approx(nu_sym, rel=1e-4)
