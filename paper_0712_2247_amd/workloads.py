"""Seeded synthetic workloads shaped like the hard-sphere slit and bulk flows of
the paper's subsection "Numerical validation" (slits a few to twenty sphere
diameters wide, bulk reduced densities up to n* ~ 0.6, a weak driving field
parallel to the walls).

This module only draws inputs: grid sizes, wall layers, parameters and the
initial density and velocity fields.  It holds none of the method's arithmetic,
and both the GPU path and the CPU oracle take their inputs from here.

Random numbers come from NumPy's PCG64 generator seeded per workload.  Fields are
float64 arrays shaped (nz, ny, nx) (x fastest in memory) and velocities
(3, nz, ny, nx).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np


def number_density(eta: float, sigma: int) -> float:
    """Number density of hard spheres of diameter sigma at packing fraction eta
    (eta = pi sigma^3 n / 6, section "Methods and Results")."""
    return 6.0 * eta / (math.pi * sigma ** 3)


def wall_layers(sigma: int) -> int:
    """Solid layers per wall: ceil(sigma/2), enough to hold every ball read of a
    fluid node inside the array."""
    return (int(sigma) + 1) // 2


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    wall_lo: int
    wall_hi: int
    sigma: int
    eta: float
    tau: float
    accel: Tuple[float, float, float]
    steps: int
    precision: str          # "f64" or "f32"
    seed: int
    noise: float = 0.0      # relative amplitude of the uniform density noise
    gauss_noise: float = 0.0  # relative amplitude of Gaussian density noise
    shear_amp: float = 0.0  # amplitude of u_x = A sin(2 pi z / nz)

    @property
    def n_bulk(self) -> float:
        return number_density(self.eta, self.sigma)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def fluid_nodes(self) -> int:
        return self.nx * self.ny * (self.nz - self.wall_lo - self.wall_hi)

    def fields(self) -> Tuple[np.ndarray, np.ndarray]:
        """Initial (n, u).  Draws one random number per node in node order, then
        zeroes the solid layers."""
        rng = np.random.default_rng(self.seed)
        shape = (self.nz, self.ny, self.nx)
        n = np.full(shape, self.n_bulk)
        if self.noise:
            n = n * (1.0 + self.noise * rng.uniform(-1.0, 1.0, size=shape))
        if self.gauss_noise:
            n = n * (1.0 + self.gauss_noise * rng.standard_normal(size=shape))
        u = np.zeros((3,) + shape)
        if self.shear_amp:
            z = np.arange(self.nz, dtype=np.float64)
            u[0] = (self.shear_amp * np.sin(2.0 * math.pi * z / self.nz))[:, None, None]
        if self.wall_lo:
            n[: self.wall_lo] = 0.0
            u[:, : self.wall_lo] = 0.0
        if self.wall_hi:
            n[self.nz - self.wall_hi:] = 0.0
            u[:, self.nz - self.wall_hi:] = 0.0
        return n, u

    def params(self) -> dict:
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, wall_lo=self.wall_lo,
                    wall_hi=self.wall_hi, sigma=self.sigma, tau=self.tau,
                    accel=tuple(self.accel))

    def with_size(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def slit(name, nx, ny, fluid_h, sigma, eta, tau, gx, steps, precision, seed, noise):
    w = wall_layers(sigma)
    return Workload(name=name, nx=nx, ny=ny, nz=fluid_h + 2 * w, wall_lo=w, wall_hi=w,
                    sigma=sigma, eta=eta, tau=tau, accel=(gx, 0.0, 0.0), steps=steps,
                    precision=precision, seed=seed, noise=noise)


def slit_small_f64() -> Workload:
    """8x8x24 slit (20 fluid layers), sigma 4, eta 0.30, tau 1, g 1e-5 x,
    +-1% uniform noise, 2000 steps, FP64."""
    return slit("slit-8x8x24-s4-eta0.30-f64", 8, 8, 20, 4, 0.30, 1.0, 1e-5, 2000, "f64",
                1001, 0.01)


def slit_64_f32() -> Workload:
    """64x64x136 slit (128 fluid layers), sigma 8, eta 0.35, tau 0.8, g 2e-6 x,
    +-0.5% uniform noise, 20000 steps, FP32 populations."""
    return slit("slit-64x64x136-s8-eta0.35-f32", 64, 64, 128, 8, 0.35, 0.8, 2e-6, 20000,
                "f32", 1002, 0.005)


def slit_64_f32_stable() -> Workload:
    """The 64x64x136 slit at packing fraction 0.25 instead of 0.35 (everything
    else, and the cost of a step, unchanged).  On this grid the scheme diverges
    from the noisy uniform start at 0.30 and above (0.35: within ~15 steps);
    0.27 and below reach a steady flow."""
    return slit("slit-64x64x136-s8-eta0.25-f32", 64, 64, 128, 8, 0.25, 0.8, 2e-6, 20000,
                "f32", 1002, 0.005)


def bulk_256_f32() -> Workload:
    """256^3 periodic bulk, sigma 6, eta 0.25, tau 1, shear wave
    u_x = 1e-3 sin(2 pi z/256), Gaussian density noise of relative amplitude
    1e-3, 5000 steps, FP32."""
    return Workload(name="bulk-256^3-s6-eta0.25-f32", nx=256, ny=256, nz=256, wall_lo=0,
                    wall_hi=0, sigma=6, eta=0.25, tau=1.0, accel=(0.0, 0.0, 0.0), steps=5000,
                    precision="f32", seed=1003, gauss_noise=1e-3, shear_amp=1e-3)


def slit_128_f32() -> Workload:
    """128x128x264 slit (256 fluid layers), sigma 8, eta 0.38, tau 1, g 1e-6 x,
    50000 steps: the held-out evaluation slit of the learned force."""
    return slit("slit-128x128x264-s8-eta0.38-f32", 128, 128, 256, 8, 0.38, 1.0, 1e-6, 50000,
                "f32", 1005, 0.005)


def slit_128_f32_stable() -> Workload:
    """The held-out evaluation slit at packing fraction 0.28 instead of 0.38
    (everything else unchanged): 0.38 is linearly unstable under the scheme
    (sigma 8, tau 1: the uniform state's symbol grows for packing above 0.32),
    and on this slit 0.30 already diverges within 500 steps while 0.28 stays
    finite over 6000; 0.28 is the largest of 0.26, 0.28, 0.30, 0.32 that runs."""
    return slit("slit-128x128x264-s8-eta0.28-f32", 128, 128, 256, 8, 0.28, 1.0, 1e-6, 50000,
                "f32", 1005, 0.005)


def ensemble(nslits: int = 512, seed: int = 1004, steps: int = 10000) -> List[Workload]:
    """Ragged ensemble of slits with a 16x16 periodic cross section.  Per slit, in
    slit order: fluid width H ~ U{10..60}, sigma ~ U{3,4,5,6,8},
    eta ~ U[0.10, 0.40], g ~ U[1e-6, 1e-5] along x; tau = 1; uniform initial
    density, zero velocity."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(nslits):
        H = int(rng.integers(10, 61))
        sigma = int(rng.choice([3, 4, 5, 6, 8]))
        eta = float(rng.uniform(0.10, 0.40))
        g = float(rng.uniform(1e-6, 1e-5))
        out.append(slit(f"ensemble[{s}]", 16, 16, H, sigma, eta, 1.0, g, steps, "f32",
                        seed * 1000 + s, 0.0))
    return out


def surrogate_training_runs(nruns: int = 40, seed: int = 1006) -> List[Workload]:
    """Training slits of the learned force: 64x64xnz with nz ~ U{40..136}
    (walls included), sigma ~ U{4..8}, eta ~ U[0.1, 0.4], tau 1, g 1e-6 x,
    +-1% noise."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(nruns):
        nz = int(rng.integers(40, 137))
        sigma = int(rng.integers(4, 9))
        eta = float(rng.uniform(0.10, 0.40))
        w = wall_layers(sigma)
        out.append(Workload(name=f"train[{r}]", nx=64, ny=64, nz=nz, wall_lo=w, wall_hi=w,
                            sigma=sigma, eta=eta, tau=1.0, accel=(1e-6, 0.0, 0.0), steps=2000,
                            precision="f32", seed=seed * 1000 + r, noise=0.01))
    return out


# Learned force: canonical weight vector W1[32][1][125], b1[32], W2[32][32][125],
# b2[32], W3[3][32][125], b3[3] (tap t = (dz+2)*25 + (dy+2)*5 + (dx+2)).
CNN_SHAPES = [(32, 1, 125), (32,), (32, 32, 125), (32,), (3, 32, 125), (3,)]
CNN_NWEIGHTS = sum(int(np.prod(s)) for s in CNN_SHAPES)


def cnn_init_weights(seed: int = 1007) -> np.ndarray:
    """Initial weights of the learned force, FP32 values: W ~ N(0, 2/fan_in)
    for the two GELU layers, N(0, 1/fan_in) for the output layer, zero
    biases (fan_in = 125 x input channels)."""
    rng = np.random.default_rng(seed)
    parts = []
    for shp, gain in zip(CNN_SHAPES, (2.0, None, 2.0, None, 1.0, None)):
        if gain is None:
            parts.append(np.zeros(shp))
        else:
            parts.append(rng.standard_normal(shp) * math.sqrt(gain / (shp[1] * shp[2])))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def bf16_grid_values(shape, scale: float, seed: int) -> np.ndarray:
    """Seeded random values that are exactly representable in bfloat16
    (FP32 draws with the low 16 bits cleared), as float32."""
    rng = np.random.default_rng(seed)
    a = (scale * rng.standard_normal(size=shape)).astype(np.float32)
    return (a.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)


WORKLOADS = {
    "slit_small_f64": slit_small_f64,
    "slit_64_f32": slit_64_f32,
    "slit_64_f32_stable": slit_64_f32_stable,
    "slit_128_f32_stable": slit_128_f32_stable,
    "bulk_256_f32": bulk_256_f32,
    "slit_128_f32": slit_128_f32,
}


def get(name: str) -> Workload:
    return WORKLOADS[name]()


def random_state(shape, n_bulk: float, rel: float, jscale: float, seed: int,
                 solid_lo: int = 0, solid_hi: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Random (n, u) for kernel-level checks: n = n_bulk (1 + rel U(-1,1)),
    u = jscale U(-1,1) per component, zero on solid layers."""
    rng = np.random.default_rng(seed)
    n = n_bulk * (1.0 + rel * rng.uniform(-1.0, 1.0, size=shape))
    u = jscale * rng.uniform(-1.0, 1.0, size=(3,) + tuple(shape))
    nz = shape[0]
    if solid_lo:
        n[:solid_lo] = 0.0
        u[:, :solid_lo] = 0.0
    if solid_hi:
        n[nz - solid_hi:] = 0.0
        u[:, nz - solid_hi:] = 0.0
    return n, u
