"""TEST INFRASTRUCTURE ONLY: plain FP64 reference of the learned hard-sphere force.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg use this module.  It shares no code with the GPU library.

The paper computes the interaction force C^(1) exactly: the surface integral of
eq. (12), with the coarse-grained density and midpoint closure of section
"Methods and Results".  The learned force is not in the paper.  It is a
three-layer 3-D convolutional network that maps the packing-fraction field
eta = pi sigma^3 n / 6 to a dimensionless force field F_hat.  The force in
lattice units is

    C^(1) ~= F_hat * v_T^2 (6/pi)^2 4 pi / sigma^4

(see ``force_scale``): C^(1) = -v_T^2 sigma^2 4 pi n S is quadratic in n, and
n = (6/pi) eta / sigma^3.

Network, all convolutions 5x5x5 with bias:

    z1 = conv(x, W1) + b1      (1 -> 32 channels)   a1 = GELU(z1)
    z2 = conv(a1, W2) + b2     (32 -> 32)           a2 = GELU(z2)
    F  = conv(a2, W3) + b3     (32 -> 3)

GELU(z) = z Phi(z) with Phi the standard normal distribution function (the exact form).

conv(x, W)[co, z, y, x] = sum_ci sum_t W[co, ci, t] x[ci, z + dz_t, y + dy_t, x + dx_t],
with taps t = (dz+2)*25 + (dy+2)*5 + (dx+2) and dz, dy, dx in -2..2.  x and y
wrap periodically.  z wraps too when the lattice has no walls; otherwise reads
beyond the array are 0, the same rule as reads into the walls (the walls hold
n = 0).

Precision of the GPU path: x, weights and the activations a1 and a2 are
rounded to bfloat16 (round to nearest, ties to even) before each convolution.
The convolutions accumulate in FP32, and biases, GELU and outputs are FP32.
``forward(..., bf16_round=True)`` applies the same roundings and does everything
else in FP64.  ``bf16_round=False`` gives the plain FP64 network that the
finite-difference checks use.

The loss is the mean over fluid nodes and the 3 components of
(F - target)^2.  Training uses Adam (Kingma and Ba, 2015): beta1 0.9,
beta2 0.999, eps 1e-8, with bias correction.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, erfc

NT = 125
C1 = 32
C2 = 32
CO = 3
TAPS = [(t // 25 - 2, (t // 5) % 5 - 2, t % 5 - 2) for t in range(NT)]   # (dz, dy, dx)

# canonical flat weight vector: W1, b1, W2, b2, W3, b3
SHAPES = [("W1", (C1, 1, NT)), ("b1", (C1,)), ("W2", (C2, C1, NT)), ("b2", (C2,)),
          ("W3", (CO, C2, NT)), ("b3", (CO,))]
NWEIGHTS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.size == NWEIGHTS
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = w[o:o + k].reshape(shp)
        o += k
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def force_scale(sigma: int) -> float:
    """Multiplier from the dimensionless network output to C^(1) in lattice
    units (v_T^2 = 1/3)."""
    return (1.0 / 3.0) * (6.0 / math.pi) ** 2 * 4.0 * math.pi / float(sigma) ** 4


def eta_field(n, sigma: int):
    """Network input: the packing fraction pi sigma^3 n / 6 at every node."""
    return math.pi * float(sigma) ** 3 * np.asarray(n, dtype=np.float64) / 6.0


def bf16(a):
    """Round to the nearest bfloat16 (8 significant bits), ties to even, as
    float64 values.  Written from the definition: a = m 2^e with m in
    [0.5, 1); keep m to 8 bits.  Inputs here are finite and far from the
    subnormal range."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def norm_cdf(z):
    """Phi(z) = erfc(-z / sqrt 2) / 2, the same as (1 + erf(z / sqrt 2)) / 2 but
    without its cancellation for z << 0."""
    return 0.5 * erfc(-np.asarray(z, dtype=np.float64) / math.sqrt(2.0))


def gelu(z):
    return z * norm_cdf(z)


def gelu_grad(z):
    """d GELU / dz = Phi(z) + z phi(z)."""
    return norm_cdf(z) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def shift(x, dz, dy, dx, zper: bool):
    """s[..., z, y, x] = x[..., z + dz, y + dy, x + dx] over the last three
    axes: periodic in y and x, periodic or zero beyond the array in z."""
    s = np.roll(x, (-dy, -dx), axis=(-2, -1))
    if zper:
        return np.roll(s, -dz, axis=-3)
    out = np.zeros_like(s)
    nz = x.shape[-3]
    if dz >= 0:
        out[..., : nz - dz, :, :] = s[..., dz:, :, :]
    else:
        out[..., -dz:, :, :] = s[..., : nz + dz, :, :]
    return out


def conv(x, W, b=None, zper=False):
    """x [ci, nz, ny, nx], W [co, ci, 125] -> [co, nz, ny, nx] (plus bias)."""
    co = W.shape[0]
    out = np.zeros((co,) + x.shape[1:])
    for t, (dz, dy, dx) in enumerate(TAPS):
        out += np.tensordot(W[:, :, t], shift(x, dz, dy, dx, zper), axes=(1, 0))
    if b is not None:
        out += b[:, None, None, None]
    return out


def conv_transpose(g, W, zper=False):
    """Adjoint of conv in its input: g [co, ...] -> [ci, ...] with
    sum(conv(x, W) * g) = sum(x * conv_transpose(g, W)) for every x."""
    ci = W.shape[1]
    out = np.zeros((ci,) + g.shape[1:])
    for t, (dz, dy, dx) in enumerate(TAPS):
        out += np.tensordot(W[:, :, t].T, shift(g, -dz, -dy, -dx, zper), axes=(1, 0))
    return out


def conv_weight_grad(x, g, zper=False):
    """dL/dW[co, ci, t] = sum over nodes of g[co] * shift(x, t)[ci]."""
    co, ci = g.shape[0], x.shape[0]
    out = np.zeros((co, ci, NT))
    gf = g.reshape(co, -1)
    for t, (dz, dy, dx) in enumerate(TAPS):
        out[:, :, t] = gf @ shift(x, dz, dy, dx, zper).reshape(ci, -1).T
    return out


def forward(w, eta, zper=False, bf16_round=True):
    """eta [nz, ny, nx] -> cache with z1, a1, z2, a2, out [3, nz, ny, nx]."""
    p = unflatten(w)
    rnd = bf16 if bf16_round else (lambda a: np.asarray(a, dtype=np.float64))
    W1, W2, W3 = rnd(p["W1"]), rnd(p["W2"]), rnd(p["W3"])
    x = rnd(eta)[None]
    z1 = conv(x, W1, p["b1"], zper)
    a1 = rnd(gelu(z1))
    z2 = conv(a1, W2, p["b2"], zper)
    a2 = rnd(gelu(z2))
    out = conv(a2, W3, p["b3"], zper)
    return {"x": x, "W1": W1, "W2": W2, "W3": W3, "z1": z1, "a1": a1, "z2": z2, "a2": a2,
            "out": out, "zper": zper}


def fluid_mask(nz, ny, nx, wall_lo, wall_hi):
    m = np.zeros((nz, ny, nx), dtype=bool)
    m[wall_lo: nz - wall_hi] = True
    return m


def loss_and_grad_out(out, target, mask):
    """Mean over fluid nodes and components of (out - target)^2 and its
    gradient in out."""
    d = (out - target) * mask[None]
    m = 3.0 * mask.sum()
    return float((d * d).sum() / m), 2.0 * d / m


def backward(w, cache, gout):
    """Gradient of a scalar in the weights, given its gradient gout in the
    output.  The bf16 roundings pass gradients straight through."""
    zper = cache["zper"]
    g = {}
    g["W3"] = conv_weight_grad(cache["a2"], gout, zper)
    g["b3"] = gout.reshape(CO, -1).sum(axis=1)
    da2 = conv_transpose(gout, cache["W3"], zper)
    dz2 = da2 * gelu_grad(cache["z2"])
    g["W2"] = conv_weight_grad(cache["a1"], dz2, zper)
    g["b2"] = dz2.reshape(C2, -1).sum(axis=1)
    da1 = conv_transpose(dz2, cache["W2"], zper)
    dz1 = da1 * gelu_grad(cache["z1"])
    g["W1"] = conv_weight_grad(cache["x"], dz1, zper)
    g["b1"] = dz1.reshape(C1, -1).sum(axis=1)
    return flatten(g), {"da2": da2, "dz2": dz2, "da1": da1, "dz1": dz1}


def loss_grad(w, eta, target, mask, zper=False, bf16_round=True):
    cache = forward(w, eta, zper, bf16_round)
    L, gout = loss_and_grad_out(cache["out"], target, mask)
    grad, _ = backward(w, cache, gout)
    return L, grad


def adam(w, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Step t (1-based) of Adam: returns the new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
