"""TEST INFRASTRUCTURE ONLY: the plain FP64 CPU oracle of the hard-sphere
lattice Boltzmann step, and a plain FP64 reference of the learned force
surrogate's network.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The GPU library neither links nor calls it and
shares no source with it.

``hsref.c`` holds the lattice Boltzmann oracle (see its header for the equations
and readings it follows); this module loads it through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hsref.c")
_LIB = os.path.join(_HERE, "libhsref.so")

FORCE_EXACT = 0
FORCE_OFF = 2
G2_PAPER = 0
G2_CS = 1


# Plain IEEE FP64: no contraction into fused multiply-adds, no reassociation
# (-O3 vectorises nothing that would reorder a sum).  The library is built on
# one host and run on another, so the target is the x86-64-v3 level (AVX2)
# rather than -march=native.
CFLAGS = ["-O3", "-march=x86-64-v3", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-ffp-contract=off"]


def build(verbose: bool = False) -> str:
    """Compile ``hsref.c`` into ``libhsref.so`` (plain IEEE FP64, OpenMP)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("wall_lo", ctypes.c_int32), ("wall_hi", ctypes.c_int32),
        ("sigma", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("accel", ctypes.c_double * 3),
        ("g2_model", ctypes.c_int32), ("wall_reg", ctypes.c_int32),
        ("force_mode", ctypes.c_int32),
        ("att_eps", ctypes.c_double), ("att_range", ctypes.c_double),
        ("lattice", ctypes.c_int32), ("thermal", ctypes.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER
    d = P(ctypes.c_double)
    lib.hsref_create.restype = ctypes.c_void_p
    lib.hsref_create.argtypes = [P(_Params)]
    lib.hsref_destroy.argtypes = [ctypes.c_void_p]
    for name in ("hsref_init", "hsref_moments", "hsref_profiles"):
        getattr(lib, name).argtypes = [ctypes.c_void_p, d, d]
        getattr(lib, name).restype = ctypes.c_int
    for name in ("hsref_force", "hsref_eta_bar", "hsref_get_populations", "hsref_set_populations",
                 "hsref_step_with_force", "hsref_attraction_potential"):
        getattr(lib, name).argtypes = [ctypes.c_void_p, d]
        getattr(lib, name).restype = ctypes.c_int
    lib.hsref_init_thermal.argtypes = [ctypes.c_void_p, d, d, d]
    lib.hsref_init_thermal.restype = ctypes.c_int
    lib.hsref_thermal_fields.argtypes = [ctypes.c_void_p, d, d]
    lib.hsref_thermal_fields.restype = ctypes.c_int
    lib.hsref_set_solid.argtypes = [ctypes.c_void_p, P(ctypes.c_uint8)]
    lib.hsref_set_solid.restype = ctypes.c_int
    lib.hsref_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    lib.hsref_step.restype = ctypes.c_int
    lib.hsref_g2.argtypes = [ctypes.c_int, ctypes.c_double]
    lib.hsref_g2.restype = ctypes.c_double
    lib.hsref_shell_table.argtypes = [ctypes.c_int, d, d, P(ctypes.c_int), P(ctypes.c_int), d]
    lib.hsref_ball_count.argtypes = [ctypes.c_int]
    lib.hsref_lattice.argtypes = [P(ctypes.c_int), d]
    lib.hsref_lattice_q.argtypes = [ctypes.c_int, P(ctypes.c_int), d]
    lib.hsref_lattice_q.restype = ctypes.c_int
    lib.hsref_q.argtypes = [ctypes.c_void_p]
    lib.hsref_q.restype = ctypes.c_int
    lib.hsref_set_threads.argtypes = [ctypes.c_int]
    lib.hsref_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(n: int) -> None:
    _load().hsref_set_threads(int(n))


def max_threads() -> int:
    return int(_load().hsref_max_threads())


def g2(eta: float, model: int = G2_PAPER) -> float:
    return float(_load().hsref_g2(int(model), float(eta)))


def shell_table(sigma: int):
    """Return (W[18], s[18,3], ncorner[18], d[18,4,3], alpha[18,4])."""
    lib = _load()
    W = np.zeros(18)
    s = np.zeros((18, 3))
    nc = np.zeros(18, dtype=np.int32)
    d = np.zeros((18, 4, 3), dtype=np.int32)
    al = np.zeros((18, 4))
    rc = lib.hsref_shell_table(int(sigma), _dptr(W), _dptr(s),
                               nc.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                               d.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dptr(al))
    assert rc == 0
    return W, s, nc, d, al


def ball_count(sigma: int) -> int:
    return int(_load().hsref_ball_count(int(sigma)))


def lattice():
    """Return (c[19,3], w[19]) of the D3Q19 lattice."""
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    _load().hsref_lattice(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dptr(w))
    return c, w


def lattice_q(q: int):
    """Return (c[q,3], w[q]) of the lattice with q = 19 or 39 velocities."""
    c = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    rc = _load().hsref_lattice_q(int(q), c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dptr(w))
    if rc != q:
        raise ValueError(f"no lattice with {q} velocities")
    return c, w


def attraction_potential_at(n, nodes, att_eps: float, att_range: float, zperiodic: bool):
    """Mean-field attraction potential (its definition is in the header of
    hsref.c) at the listed nodes (z, y, x) of the density field n [nz, ny, nx],
    each as its own direct sum over the cube of offsets: for spot checks of
    grids too large for the full oracle."""
    nz, ny, nx = n.shape
    R = int(np.ceil(3.0 * att_range))
    o = np.arange(-R, R + 1)
    OZ, OY, OX = np.meshgrid(o, o, o, indexing="ij")
    g = np.exp(-(OX * OX + OY * OY + OZ * OZ).astype(np.float64) / att_range ** 2)
    out = []
    for z, y, x in nodes:
        zz = z + OZ
        inside = np.ones(zz.shape, dtype=bool)
        if zperiodic:
            zz = zz % nz
        else:
            inside = (zz >= 0) & (zz < nz)
            zz = np.clip(zz, 0, nz - 1)
        vals = n[zz, (y + OY) % ny, (x + OX) % nx]
        out.append(-att_eps * float(np.sum(np.where(inside, g * vals, 0.0))))
    return np.array(out)


class Oracle:
    """One lattice on the CPU.  Fields use the node order x fastest, then y, then
    z: arrays are shaped (nz, ny, nx) and vectors (3, nz, ny, nx)."""

    def __init__(self, nx, ny, nz, sigma, tau, accel=(0.0, 0.0, 0.0), wall_lo=0, wall_hi=0,
                 g2_model=G2_PAPER, wall_reg=1, force_mode=FORCE_EXACT, att_eps=0.0, att_range=0.0,
                 lattice=19, thermal=0):
        self._lib = _load()
        p = _Params()
        p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
        p.wall_lo, p.wall_hi = int(wall_lo), int(wall_hi)
        p.sigma = int(sigma)
        p.tau = float(tau)
        p.accel = (ctypes.c_double * 3)(*[float(a) for a in accel])
        p.g2_model, p.wall_reg, p.force_mode = int(g2_model), int(wall_reg), int(force_mode)
        p.att_eps, p.att_range = float(att_eps), float(att_range)
        p.lattice = int(lattice)
        p.thermal = int(thermal)
        self.params = p
        self.shape = (int(nz), int(ny), int(nx))
        self.N = int(nx) * int(ny) * int(nz)
        self._ctx = self._lib.hsref_create(ctypes.byref(p))
        if not self._ctx:
            raise ValueError("oracle rejected the parameters")
        self.q = int(self._lib.hsref_q(self._ctx))

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx:
            self._lib.hsref_destroy(ctx)
            self._ctx = None

    def _chk(self, rc, what):
        if rc != 0:
            raise ValueError(f"oracle {what} failed ({rc})")

    def set_solid(self, solid):
        """Solid mask [nz, ny, nx] (nonzero: solid), before init."""
        m = np.ascontiguousarray(np.asarray(solid) != 0, dtype=np.uint8).reshape(self.N)
        self._chk(self._lib.hsref_set_solid(self._ctx, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))),
                  "set_solid")

    def init(self, n, u=None, T=None):
        """Equilibrium populations of (n, u), and of T in a thermal context
        (T None: the lattice temperature 2/3 everywhere)."""
        n = np.ascontiguousarray(n, dtype=np.float64).reshape(self.N)
        if u is None:
            u = np.zeros(3 * self.N)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(3 * self.N)
        if self.params.thermal:
            Tp = None if T is None else _dptr(np.ascontiguousarray(T, dtype=np.float64).reshape(self.N))
            self._chk(self._lib.hsref_init_thermal(self._ctx, _dptr(n), _dptr(u), Tp), "init_thermal")
        else:
            if T is not None:
                raise ValueError("a temperature field needs thermal=1")
            self._chk(self._lib.hsref_init(self._ctx, _dptr(n), _dptr(u)), "init")

    def thermal_fields(self):
        """Temperature T and energy source C^(2) [nz, ny, nx] of the current state."""
        T = np.zeros(self.N)
        Q = np.zeros(self.N)
        self._chk(self._lib.hsref_thermal_fields(self._ctx, _dptr(T), _dptr(Q)), "thermal_fields")
        return T.reshape(self.shape), Q.reshape(self.shape)

    def step(self, nsteps=1):
        self._chk(self._lib.hsref_step(self._ctx, int(nsteps)), "step")

    def moments(self):
        n = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        self._chk(self._lib.hsref_moments(self._ctx, _dptr(n), _dptr(u)), "moments")
        return n.reshape(self.shape), u.reshape((3,) + self.shape)

    def profiles(self):
        nz = self.shape[0]
        pn = np.zeros(nz)
        pu = np.zeros(3 * nz)
        self._chk(self._lib.hsref_profiles(self._ctx, _dptr(pn), _dptr(pu)), "profiles")
        return pn, pu.reshape(3, nz)

    def force(self):
        F = np.zeros(3 * self.N)
        self._chk(self._lib.hsref_force(self._ctx, _dptr(F)), "force")
        return F.reshape((3,) + self.shape)

    def step_with_force(self, C1):
        """One step with the interaction force C1 [3, nz, ny, nx] given (plus
        the external field n g) instead of the shell sum."""
        C1 = np.ascontiguousarray(C1, dtype=np.float64).reshape(3 * self.N)
        self._chk(self._lib.hsref_step_with_force(self._ctx, _dptr(C1)), "step_with_force")

    def attraction_potential(self):
        """Mean-field attraction potential Phi [nz, ny, nx] of the current state."""
        phi = np.zeros(self.N)
        self._chk(self._lib.hsref_attraction_potential(self._ctx, _dptr(phi)), "attraction_potential")
        return phi.reshape(self.shape)

    def eta_bar(self):
        e = np.zeros(self.N)
        self._chk(self._lib.hsref_eta_bar(self._ctx, _dptr(e)), "eta_bar")
        return e.reshape(self.shape)

    def get_populations(self):
        f = np.zeros(self.q * self.N)
        self._chk(self._lib.hsref_get_populations(self._ctx, _dptr(f)), "get_populations")
        return f.reshape((self.q,) + self.shape)

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.q * self.N)
        self._chk(self._lib.hsref_set_populations(self._ctx, _dptr(f)), "set_populations")
