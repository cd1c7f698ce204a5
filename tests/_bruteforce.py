"""Brute-force evaluation of the hard-sphere force of equation (12), written
from the geometry of the paper's prescription rather than from tables: the
coarse-grained density by a distance test over every offset, each of the 18
quadrature points placed at r + sigma s_hat in real coordinates, and every
off-lattice point spread over the four lattice corners of its in-plane cell by
ordinary bilinear interpolation.  Pure Python loops: tiny grids only.

Used by the tests to pin the oracle; it is not the oracle and shares nothing
with it or with the GPU library.
"""
from __future__ import annotations

import math

import numpy as np

VT2 = 1.0 / 3.0
KAPPA = 2.0 / (math.sqrt(VT2) * math.sqrt(math.pi))


def g2(eta, model=0):
    if model == 1:
        return (1.0 - eta / 2.0) / (1.0 - eta) ** 3
    return (1.0 - eta / 2.0 + eta * eta / 4.0) / (1.0 - eta) ** 3


def quadrature_points():
    """The 18 points: 6 axis (weight 1/30) and 12 face diagonals (1/15)."""
    pts = []
    for a in range(3):
        for s in (1.0, -1.0):
            v = [0.0, 0.0, 0.0]
            v[a] = s
            pts.append((1.0 / 30.0, tuple(v)))
    r = 1.0 / math.sqrt(2.0)
    for a, b in ((0, 1), (0, 2), (1, 2)):
        for sa in (1.0, -1.0):
            for sb in (1.0, -1.0):
                v = [0.0, 0.0, 0.0]
                v[a] = sa * r
                v[b] = sb * r
                pts.append((1.0 / 15.0, tuple(v)))
    return pts


def corners(sigma, s):
    """Lattice corners and bilinear weights of the point sigma*s (relative to
    the node): a single corner for an axis point, the four corners of the
    in-plane unit cell otherwise."""
    p = [sigma * c for c in s]
    nz_axes = [a for a in range(3) if s[a] != 0.0]
    if len(nz_axes) == 1:
        return [(tuple(int(round(c)) for c in p), 1.0)]
    a, b = nz_axes
    fa, fb = math.floor(p[a]), math.floor(p[b])
    ta, tb = p[a] - fa, p[b] - fb
    out = []
    for ia, wa in ((0, 1.0 - ta), (1, ta)):
        for ib, wb in ((0, 1.0 - tb), (1, tb)):
            d = [0, 0, 0]
            d[a] = fa + ia
            d[b] = fb + ib
            out.append((tuple(d), wa * wb))
    return out


class Grid:
    def __init__(self, n, j, sigma, wall_lo=0, wall_hi=0, g2_model=0, wall_reg=1):
        self.n = np.asarray(n, dtype=np.float64)
        self.j = np.asarray(j, dtype=np.float64)
        self.nz, self.ny, self.nx = self.n.shape
        self.sigma = sigma
        self.wl, self.wh = wall_lo, wall_hi
        self.zper = wall_lo == 0 and wall_hi == 0
        self.g2_model = g2_model
        self.wall_reg = wall_reg

    def solid(self, z):
        return z < self.wl or z >= self.nz - self.wh

    def inside(self, z):
        return self.zper or 0 <= z < self.nz

    def wrap(self, x, y, z):
        return x % self.nx, y % self.ny, (z % self.nz) if self.zper else z

    def dens(self, x, y, z):
        x, y, z = self.wrap(x, y, z)
        if not self.inside(z) or self.solid(z):
            return 0.0, (0.0, 0.0, 0.0)
        return self.n[z, y, x], tuple(self.j[a, z, y, x] for a in range(3))

    def eta_bar(self, x, y, z):
        R = self.sigma / 2.0
        k = int(math.ceil(R))
        tot = 0.0
        cnt = 0
        for oz in range(-k, k + 1):
            for oy in range(-k, k + 1):
                for ox in range(-k, k + 1):
                    if math.sqrt(ox * ox + oy * oy + oz * oz) <= R + 1e-12:
                        cnt += 1
                        tot += self.dens(x + ox, y + oy, z + oz)[0]
        return math.pi * self.sigma ** 3 / 6.0 * tot / cnt

    def chi(self, z):
        if self.zper or not self.wall_reg:
            return 1.0
        za, zb = self.wl - 0.5, self.nz - self.wh - 0.5
        return 1.0 - math.exp(-min(z - za, zb - z) / self.sigma)

    def force_at(self, nodes):
        """C^(1) at the given nodes [(x, y, z), ...] (fluid nodes), and for
        each the sum of the magnitudes of the terms it is made of,
        |v_T^2 sigma^2 4 pi n| sum_q W_q |s_q| sum_k alpha_k G (|n'| + chi
        kappa |s.j'| + chi kappa |n' s.u|), the scale of its rounding error."""
        eb = {}

        def ebar(x, y, z):
            key = self.wrap(x, y, z)
            if key not in eb:
                eb[key] = self.eta_bar(*key)
            return eb[key]

        pts = quadrature_points()
        F = np.zeros((3, len(nodes)))
        A = np.zeros((3, len(nodes)))
        pref = VT2 * self.sigma ** 2 * 4.0 * math.pi
        for i, (x, y, z) in enumerate(nodes):
            nr, jr = self.dens(x, y, z)
            ur = [jr[a] / nr if nr != 0 else 0.0 for a in range(3)]
            S = [0.0, 0.0, 0.0]
            Sa = [0.0, 0.0, 0.0]
            for W, s in pts:
                acc = 0.0
                acca = 0.0
                for d, al in corners(self.sigma, s):
                    cx, cy, cz = x + d[0], y + d[1], z + d[2]
                    nc, jc = self.dens(cx, cy, cz)
                    mids = []
                    for r0, c0 in ((x, cx), (y, cy), (z, cz)):
                        h = (r0 + c0) / 2.0
                        mids.append(sorted({math.floor(h), math.ceil(h)}))
                    vals = [ebar(mx, my, mz) for mz in mids[2] for my in mids[1] for mx in mids[0]]
                    G = g2(sum(vals) / len(vals), self.g2_model)
                    sj = sum(s[a] * jc[a] for a in range(3))
                    su = sum(s[a] * ur[a] for a in range(3))
                    ck = self.chi(z) * KAPPA
                    acc += al * G * (nc - ck * (sj - nc * su))
                    acca += al * G * (abs(nc) + ck * (abs(sj) + abs(nc * su)))
                for a in range(3):
                    S[a] += W * s[a] * acc
                    Sa[a] += W * abs(s[a]) * acca
            for a in range(3):
                F[a, i] = -pref * nr * S[a]
                A[a, i] = pref * abs(nr) * Sa[a]
        return F, A

    def force(self, accel=(0.0, 0.0, 0.0)):
        F = np.zeros((3, self.nz, self.ny, self.nx))
        eb = {}

        def ebar(x, y, z):
            key = self.wrap(x, y, z)
            if key not in eb:
                eb[key] = self.eta_bar(*key)
            return eb[key]

        pts = quadrature_points()
        for z in range(self.nz):
            if self.solid(z):
                continue
            for y in range(self.ny):
                for x in range(self.nx):
                    nr, jr = self.dens(x, y, z)
                    ur = [jr[a] / nr if nr != 0 else 0.0 for a in range(3)]
                    S = [0.0, 0.0, 0.0]
                    for W, s in pts:
                        acc = 0.0
                        for d, al in corners(self.sigma, s):
                            cx, cy, cz = x + d[0], y + d[1], z + d[2]
                            nc, jc = self.dens(cx, cy, cz)
                            if nc == 0.0 and jc == (0.0, 0.0, 0.0):
                                continue
                            mids = []
                            for r0, c0 in ((x, cx), (y, cy), (z, cz)):
                                h = (r0 + c0) / 2.0
                                mids.append(sorted({math.floor(h), math.ceil(h)}))
                            vals = [ebar(mx, my, mz) for mz in mids[2] for my in mids[1]
                                    for mx in mids[0]]
                            G = g2(sum(vals) / len(vals), self.g2_model)
                            cur = sum(s[a] * (jc[a] - nc * ur[a]) for a in range(3))
                            acc += al * G * (nc - self.chi(z) * KAPPA * cur)
                        for a in range(3):
                            S[a] += W * s[a] * acc
                    for a in range(3):
                        F[a, z, y, x] = -VT2 * self.sigma ** 2 * 4.0 * math.pi * nr * S[a] \
                            + nr * accel[a]
        return F


def thermal_force(grid: Grid, T, accel=(0.0, 0.0, 0.0)):
    """The non-isothermal C^(1) and the energy source C^(2) (readings in the
    oracle's header: v_T^2 = T(r) at the receiving node, the partner's T at
    r + sigma s_hat), by the same geometry as Grid.force: returns (F, Q)."""
    T = np.asarray(T, dtype=np.float64)
    F = np.zeros((3, grid.nz, grid.ny, grid.nx))
    Q = np.zeros((grid.nz, grid.ny, grid.nx))
    eb = {}

    def ebar(x, y, z):
        key = grid.wrap(x, y, z)
        if key not in eb:
            eb[key] = grid.eta_bar(*key)
        return eb[key]

    def temp(x, y, z):
        x, y, z = grid.wrap(x, y, z)
        return T[z, y, x]

    for z in range(grid.nz):
        if grid.solid(z):
            continue
        for y in range(grid.ny):
            for x in range(grid.nx):
                nr, jr = grid.dens(x, y, z)
                ur = [jr[a] / nr if nr != 0 else 0.0 for a in range(3)]
                Tr = T[z, y, x]
                vt = math.sqrt(Tr)
                kap = 2.0 / (vt * math.sqrt(math.pi))
                S = [0.0, 0.0, 0.0]
                Qs = 0.0
                for W, s in quadrature_points():
                    acc = accq = 0.0
                    for d, al in corners(grid.sigma, s):
                        cx, cy, cz = x + d[0], y + d[1], z + d[2]
                        nc, jc = grid.dens(cx, cy, cz)
                        if nc == 0.0 and jc == (0.0, 0.0, 0.0):
                            continue
                        mids = []
                        for r0, c0 in ((x, cx), (y, cy), (z, cz)):
                            h = (r0 + c0) / 2.0
                            mids.append(sorted({math.floor(h), math.ceil(h)}))
                        vals = [ebar(mx, my, mz) for mz in mids[2] for my in mids[1] for mx in mids[0]]
                        G = g2(sum(vals) / len(vals), grid.g2_model)
                        cur = sum(s[a] * (jc[a] - nc * ur[a]) for a in range(3))
                        dT = temp(cx, cy, cz) - Tr
                        acc += al * G * (nc - grid.chi(z) * kap * cur + nc * dT / (2.0 * Tr))
                        accq += al * G * (-0.5 * cur + nc * dT / (math.sqrt(math.pi) * vt))
                    for a in range(3):
                        S[a] += W * s[a] * acc
                    Qs += W * accq
                pre = Tr * grid.sigma ** 2 * 4.0 * math.pi * nr
                for a in range(3):
                    F[a, z, y, x] = -pre * S[a] + nr * accel[a]
                Q[z, y, x] = pre * Qs
    return F, Q
