"""TEST INFRASTRUCTURE ONLY: linear symbol of the hard-sphere lattice Boltzmann
step about a uniform fluid at rest (density n0, packing eta0, no walls).

Only the test suite uses this module; it shares no code with the GPU library
or with the real-space oracle (the shell table, ball and closure are rebuilt
here from their definitions).

A perturbation f_i = w_i n0 + a_i exp(i k.r) evolves linearly as
a(t+1) = A(k) a(t).  With dn = sum a_i, dj = sum c_i a_i (u0 = 0):

  - equilibrium (eq. 11) to first order: df_eq,i = w_i (dn + 3 c_i . dj);
  - interaction force (eq. 12; the uniform state has zero force, so only the
    bracket varies): dC1 = -v_T^2 sigma^2 4 pi n0 dS with
        dS = dn  sum_q W_q s_q sum_c alpha_c [n0 g2'(eta0) (pi sigma^3/6) B(k) M_d(k) + G0 e^{ik.d}]
           - kappa G0 sum_q W_q s_q (s_q . dj) sum_c alpha_c (e^{ik.d} - 1),
    where B(k) is the mean of e^{ik.o} over the smearing ball, M_d(k) the mean
    of e^{ik.m} over the lattice nodes nearest the midpoint d/2, and G0, g2'
    the closure and its derivative at eta0 (the current term's velocity at the
    receiving node enters as n0 du = dj);
  - optional mean-field attraction (its real-space form is in the header of
    hsref.c): Phi = -eps (g * n) with the separable Gaussian weights g, so
    dPhi = -eps g_hat(k) dn and the central difference of Phi gives
    dC1_att = -n0 i sin(k) dPhi = i eps n0 g_hat(k) sin(k) dn, where
    g_hat(k) = prod_a sum_{|m| <= R} exp(-m^2/lambda^2) cos(k_a m);
  - collision with the first-order source (eq. 10):
    a*_i = a_i - (a_i - df_eq,i)/tau + 3 w_i c_i . dC1;
  - push propagation: a_i(t+1) = exp(-i k.c_i) a*_i.

The eigenvalues of A(k) give linear stability (all |lambda| <= 1) and the
transport coefficients the discrete scheme predicts: the shear mode decays as
lambda = exp(-nu k^2 + O(k^4)), sound modes as exp(+-i c k - Gamma k^2).
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

C = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
              (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
              (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)], dtype=np.int64)
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
VT2 = 1.0 / 3.0
KAPPA = 2.0 / (math.sqrt(VT2) * math.sqrt(math.pi))
G2_PAPER, G2_CS = 0, 1


def g2(model: int, eta: float) -> float:
    if model == G2_PAPER:
        return (1 - eta / 2 + eta * eta / 4) / (1 - eta) ** 3
    return (1 - eta / 2) / (1 - eta) ** 3


def dg2(model: int, eta: float) -> float:
    """d g2 / d eta of the closure (quotient rule)."""
    if model == G2_PAPER:
        num, dnum = 1 - eta / 2 + eta * eta / 4, -0.5 + eta / 2
    else:
        num, dnum = 1 - eta / 2, -0.5
    return dnum / (1 - eta) ** 3 + 3 * num / (1 - eta) ** 4


def shell(sigma: int) -> List[Tuple[float, np.ndarray, List[Tuple[np.ndarray, float]]]]:
    """The 18 quadrature directions: (W, unit vector, [(lattice offset, weight)])."""
    out = []
    for a in range(3):
        for sgn in (1, -1):
            s = np.zeros(3)
            s[a] = sgn
            out.append((1 / 30, s, [(np.rint(sigma * s).astype(np.int64), 1.0)]))
    A = sigma / math.sqrt(2.0)
    l = int(math.floor(A))
    th = A - l
    om = {l: 1 - th, l + 1: th}
    for a, b in ((0, 1), (0, 2), (1, 2)):
        for sa in (1, -1):
            for sb in (1, -1):
                s = np.zeros(3)
                s[a], s[b] = sa / math.sqrt(2), sb / math.sqrt(2)
                corners = []
                for i in (l, l + 1):
                    for j in (l, l + 1):
                        d = np.zeros(3, dtype=np.int64)
                        d[a], d[b] = sa * i, sb * j
                        corners.append((d, om[i] * om[j]))
                out.append((1 / 15, s, corners))
    return out


def ball(sigma: int) -> np.ndarray:
    r = sigma // 2 + 1
    g = np.arange(-r, r + 1)
    o = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).T
    return o[4 * (o * o).sum(axis=1) <= sigma * sigma]


def midpoint_nodes(d: np.ndarray) -> np.ndarray:
    """Lattice nodes nearest d/2: each odd coordinate contributes both of its
    neighbouring integers."""
    choices = [[v // 2] if v % 2 == 0 else [(v - 1) // 2, (v + 1) // 2] for v in d]
    return np.array(np.meshgrid(*choices, indexing="ij")).reshape(3, -1).T


def att_cutoff(att_range: float) -> int:
    return int(math.ceil(3.0 * att_range))


def att_ghat(k, att_range: float) -> float:
    """Lattice Fourier transform of the truncated Gaussian weights at k."""
    R = att_cutoff(att_range)
    m = np.arange(-R, R + 1, dtype=np.float64)
    g1 = np.exp(-m * m / att_range ** 2)
    return float(np.prod([np.sum(g1 * np.cos(ka * m)) for ka in np.asarray(k, dtype=np.float64)]))


def amplification(k, sigma: int, eta: float, tau: float, model: int = G2_PAPER,
                  hs_on: bool = True, att_eps: float = 0.0, att_range: float = 0.0) -> np.ndarray:
    """A(k), 19 x 19 complex."""
    k = np.asarray(k, dtype=np.float64)
    n0 = 6 * eta / (math.pi * sigma ** 3)
    om = 1.0 / tau
    c = C.astype(np.float64)
    # collision of the moments' equilibrium: df_eq = Weq a
    Weq = W[:, None] * (1.0 + 3.0 * c @ c.T)
    M = (1 - om) * np.eye(19) + om * Weq
    if hs_on:
        G0, dG = g2(model, eta), dg2(model, eta)
        Bk = np.exp(1j * ball(sigma) @ k).mean()
        pref_eta = math.pi * sigma ** 3 / 6
        sn = np.zeros(3, dtype=complex)
        T = np.zeros((3, 3), dtype=complex)
        for Wq, s, corners in shell(sigma):
            an = 0.0 + 0.0j
            aj = 0.0 + 0.0j
            for d, al in corners:
                Md = np.exp(1j * midpoint_nodes(d) @ k).mean()
                ph = np.exp(1j * d @ k)
                an += al * (n0 * dG * pref_eta * Bk * Md + G0 * ph)
                aj += al * (ph - 1.0)
            sn += Wq * s * an
            T += Wq * np.outer(s, s) * aj
        pref = -VT2 * sigma * sigma * 4 * math.pi * n0
        # dC1 = pref (sn dn - kappa G0 T dj); dn = 1.a, dj = c^T a
        MF = pref * (np.outer(sn, np.ones(19)) - KAPPA * G0 * T @ c.T)   # 3 x 19
        M = M + 3.0 * (W[:, None] * c) @ MF
    if att_eps != 0.0:
        att = 1j * att_eps * n0 * att_ghat(k, att_range) * np.sin(k)
        M = M + 3.0 * (W[:, None] * c) @ np.outer(att, np.ones(19))
    E = np.exp(-1j * (c @ k))
    return E[:, None] * M


def eigen(k, sigma, eta, tau, model=G2_PAPER, hs_on=True, att_eps=0.0, att_range=0.0):
    lam, vec = np.linalg.eig(amplification(k, sigma, eta, tau, model, hs_on, att_eps, att_range))
    return lam, vec


def shear_nu(L: int, sigma: int, eta: float, tau: float, model=G2_PAPER, hs_on=True) -> float:
    """nu from the shear eigenvalue at k = 2 pi / L along z (eigenvector with the
    largest x-momentum share): lambda = exp(-nu k^2)."""
    k = np.array([0.0, 0.0, 2 * math.pi / L])
    lam, vec = eigen(k, sigma, eta, tau, model, hs_on)
    jx = np.abs(C[:, 0].astype(float) @ vec) / np.linalg.norm(vec, axis=0)
    m = int(np.argmax(jx))
    return float(-math.log(abs(lam[m])) / (k[2] ** 2))


def shear_lambda(L: int, sigma: int, eta: float, tau: float, model=G2_PAPER, hs_on=True) -> complex:
    k = np.array([0.0, 0.0, 2 * math.pi / L])
    lam, vec = eigen(k, sigma, eta, tau, model, hs_on)
    jx = np.abs(C[:, 0].astype(float) @ vec) / np.linalg.norm(vec, axis=0)
    return complex(lam[int(np.argmax(jx))])


def sound(L: int, sigma: int, eta: float, tau: float, model=G2_PAPER, hs_on=True, att_eps=0.0,
          att_range=0.0):
    """(speed, amplitude damping rate per step) of the sound pair at k = 2 pi / L
    along z: the two eigenvalues with the largest density share."""
    k = np.array([0.0, 0.0, 2 * math.pi / L])
    lam, vec = eigen(k, sigma, eta, tau, model, hs_on, att_eps, att_range)
    nshare = np.abs(vec.sum(axis=0)) / np.linalg.norm(vec, axis=0)
    m = int(np.argmax(nshare))
    return abs(np.angle(lam[m])) / k[2], -math.log(abs(lam[m]))


def max_growth(L: int, sigma: int, eta: float, tau: float, model=G2_PAPER, axes: str = "xyz",
               att_eps: float = 0.0, att_range: float = 0.0) -> float:
    """Largest |lambda| over the wavevectors 2 pi m / L of an L^3 periodic box,
    m1 >= m2 >= m3 >= 0 (cubic symmetry; axes='z' for k along z only)."""
    best = 0.0
    h = L // 2
    if axes == "z":
        ms = [(0, 0, m) for m in range(0, h + 1)]
    else:
        ms = [(a, b, c) for a in range(h + 1) for b in range(a + 1) for c in range(b + 1)]
    for m in ms:
        k = 2 * math.pi * np.array(m, dtype=np.float64) / L
        lam = np.linalg.eigvals(amplification(k, sigma, eta, tau, model, True, att_eps, att_range))
        best = max(best, float(np.abs(lam).max()))
    return best
