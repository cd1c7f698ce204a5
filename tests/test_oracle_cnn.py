"""Pins of the FP64 learned-force oracle (oracle/cnn.py) against things that
do not come from it: library routines (scipy.ndimage.correlate), published
values (the normal distribution function), the bfloat16 rounding of FP32 bit
patterns, exact identities (adjointness, linearity) and central finite
differences of the plain FP64 network."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import cnn
from paper_0712_2247_amd import workloads


def test_bf16_rounding_values():
    ulp = 2.0 ** -7  # spacing of bfloat16 in [1, 2)
    cases = [(1.0, 1.0), (1.0 + ulp / 2, 1.0),            # tie -> even
             (1.0 + 3 * ulp / 2, 1.0 + 2 * ulp),          # tie -> even (up)
             (1.0 + 0.75 * ulp, 1.0 + ulp), (1.0 + 0.25 * ulp, 1.0),
             (-3.0 - 0.3 * 2 * ulp, -3.0), (0.15625, 0.15625),
             (1e-3, 131.0 / 128.0 * 2.0 ** -10)]   # 1e-3 = 1.024 * 2^-10; 1.024 * 128 = 131.07
    for a, want in cases:
        assert cnn.bf16(a) == want, (a, cnn.bf16(a), want)


def test_bf16_rounding_matches_fp32_bit_rounding():
    """Round-to-nearest-even of FP32 bit patterns to their top 16 bits (add
    0x7FFF plus the lowest kept bit, truncate) on random FP32 values."""
    rng = np.random.default_rng(5)
    a = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-6, 3, 20000)).astype(np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    r = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16) << 16
    want = r.astype(np.uint32).view(np.float32).astype(np.float64)
    assert np.array_equal(cnn.bf16(a.astype(np.float64)), want)


def test_gelu_values_and_derivative():
    Phi1 = 0.8413447460685429  # standard normal distribution function at 1
    assert cnn.gelu(np.array(0.0)) == 0.0
    assert abs(cnn.gelu(np.array(1.0)) - Phi1) < 1e-15
    assert abs(cnn.gelu(np.array(-1.0)) + (1.0 - Phi1)) < 1e-15
    z = np.linspace(-6, 6, 241)
    assert np.allclose(cnn.gelu(z) - cnn.gelu(-z), z, rtol=0, atol=1e-14)
    h = 1e-5
    fd = (cnn.gelu(z + h) - cnn.gelu(z - h)) / (2 * h)
    assert np.abs(fd - cnn.gelu_grad(z)).max() < 1e-9
    # far left tail: Phi(-10) = 7.619853024160527e-24 (normal tables)
    assert abs(cnn.gelu(np.array(-10.0)) / (-10.0 * 7.619853024160527e-24) - 1.0) < 1e-12


@pytest.mark.parametrize("zper", [True, False])
def test_conv_matches_scipy_correlate(zper):
    rng = np.random.default_rng(6)
    x = rng.standard_normal((2, 7, 6, 9))
    W = rng.standard_normal((3, 2, cnn.NT))
    b = rng.standard_normal(3)
    out = cnn.conv(x, W, b, zper)
    for co in range(3):
        ref = np.full(x.shape[1:], b[co])
        for ci in range(2):
            k = W[co, ci].reshape(5, 5, 5)  # [dz+2, dy+2, dx+2]
            if zper:
                ref += ndi.correlate(x[ci], k, mode="wrap")
            else:  # zero layers beyond z, then wrap: the wrap only ever reads zeros in z
                xp = np.pad(x[ci], ((2, 2), (0, 0), (0, 0)))
                ref += ndi.correlate(xp, k, mode="wrap")[2:-2]
        assert np.allclose(out[co], ref, rtol=1e-13, atol=1e-12)


def test_conv_impulse_response():
    """A unit impulse at r0 gives W[co, 0, t] at r0 - offset(t)."""
    x = np.zeros((1, 9, 8, 10))
    r0 = (4, 3, 5)
    x[(0,) + r0] = 1.0
    W = np.arange(2 * cnn.NT, dtype=np.float64).reshape(2, 1, cnn.NT) + 1.0
    out = cnn.conv(x, W, None, zper=False)
    for t, (dz, dy, dx) in enumerate(cnn.TAPS):
        r = (r0[0] - dz, (r0[1] - dy) % 8, (r0[2] - dx) % 10)
        assert out[(0,) + r] == W[0, 0, t] and out[(1,) + r] == W[1, 0, t]
    assert np.count_nonzero(out[0]) == cnn.NT


@pytest.mark.parametrize("zper", [True, False])
def test_conv_transpose_is_adjoint_and_weight_grad_is_exact(zper):
    rng = np.random.default_rng(7)
    x = rng.standard_normal((3, 6, 5, 7))
    g = rng.standard_normal((2, 6, 5, 7))
    W = rng.standard_normal((2, 3, cnn.NT))
    lhs = (cnn.conv(x, W, None, zper) * g).sum()
    assert abs(lhs - (x * cnn.conv_transpose(g, W, zper)).sum()) <= 1e-12 * abs(lhs)
    # <conv(x, W), g> is linear in W: its gradient is conv_weight_grad exactly
    D = rng.standard_normal(W.shape)
    dW = cnn.conv_weight_grad(x, g, zper)
    lin = (cnn.conv(x, D, None, zper) * g).sum()
    assert abs(lin - (D * dW).sum()) <= 1e-12 * abs(lin)


@pytest.mark.parametrize("zper,walls", [(True, 0), (False, 2)])
def test_backward_matches_central_differences(zper, walls):
    """Gradient of the plain FP64 network loss (no bf16 rounding) in random
    directions, against central differences."""
    nz, ny, nx = 8, 6, 7
    rng = np.random.default_rng(8)
    w = workloads.cnn_init_weights(11).astype(np.float64)
    w[cnn.NWEIGHTS - 3:] = rng.standard_normal(3) * 0.1            # nonzero output bias
    eta = 0.3 * (1.0 + 0.2 * rng.uniform(-1, 1, (nz, ny, nx)))
    if walls:
        eta[:walls] = 0.0
        eta[nz - walls:] = 0.0
    mask = cnn.fluid_mask(nz, ny, nx, walls, walls)
    target = rng.standard_normal((3, nz, ny, nx)) * 0.05
    L, g = cnn.loss_grad(w, eta, target, mask, zper, bf16_round=False)
    for k in range(4):
        d = rng.standard_normal(w.size)
        d /= np.linalg.norm(d)
        h = 1e-4
        Lp, _ = cnn.loss_grad(w + h * d, eta, target, mask, zper, bf16_round=False)
        Lm, _ = cnn.loss_grad(w - h * d, eta, target, mask, zper, bf16_round=False)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * abs(g @ d), (k, fd, g @ d)
    # single coordinates of each tensor (first-layer weight, bias, output weight)
    for idx in (5, 32 * 125 + 3, cnn.NWEIGHTS - 2, cnn.NWEIGHTS - 100):
        e = np.zeros(w.size)
        e[idx] = 1.0
        h = 1e-4
        Lp, _ = cnn.loss_grad(w + h * e, eta, target, mask, zper, bf16_round=False)
        Lm, _ = cnn.loss_grad(w - h * e, eta, target, mask, zper, bf16_round=False)
        assert abs((Lp - Lm) / (2 * h) - g[idx]) <= 1e-6 * max(abs(g[idx]), 1e-12) + 1e-13


def test_adam_first_step_and_convergence():
    """First step: m_hat = g, v_hat = g^2, so w moves by lr g / (|g| + eps);
    on a quadratic bowl the iteration reaches the minimum."""
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    w1, m, v = cnn.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, 0.01)
    assert np.allclose(w1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)
    c = np.array([1.0, -2.0, 0.5])
    w, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        w, m, v = cnn.adam(w, m, v, 2.0 * (w - c), t, 0.01)
    assert np.abs(w - c).max() < 1e-3


def test_forward_bf16_rounds_inputs_weights_and_activations():
    """The rounded forward equals the plain FP64 network applied to bf16
    values of x and the weights, with bf16 activations in between."""
    rng = np.random.default_rng(9)
    w = workloads.cnn_init_weights(12).astype(np.float64)
    eta = 0.25 * (1.0 + 0.1 * rng.uniform(-1, 1, (6, 5, 5)))
    c = cnn.forward(w, eta, zper=True)
    assert np.array_equal(c["a1"], cnn.bf16(c["a1"])) and np.array_equal(c["x"], cnn.bf16(c["x"]))
    p = cnn.unflatten(w)
    z1 = cnn.conv(cnn.bf16(eta)[None], cnn.bf16(p["W1"]), p["b1"], True)
    assert np.array_equal(z1, c["z1"])
    plain = cnn.forward(w, eta, zper=True, bf16_round=False)
    e = np.linalg.norm(c["out"] - plain["out"]) / np.linalg.norm(plain["out"])
    assert 1e-5 < e < 3e-2   # bf16 changes the result, by about its precision
