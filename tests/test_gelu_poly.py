"""Host checks of the learned force's fast GELU (phi_cdf_fast in
hslb_cnn.hip): its coefficients are the ones csrc/gen_phi_poly.py fits, and
the formula evaluated in FP32 arithmetic (each operation rounded, FMAs
rounded once; the base-2 exponential and the reciprocal correctly rounded
here, about 1 ulp on the GPU) stays within 16 FP32 ulps of z * erfc(-z / sqrt 2) / 2, half the
32-ulp window around a bf16 rounding tie inside which the kernel evaluates
the erfcf form instead."""
import importlib.util
import os
import re

import numpy as np
from scipy.special import erfc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0712_2247_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_phi_poly", os.path.join(CSRC, "gen_phi_poly.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _kernel_coefficients():
    src = open(os.path.join(CSRC, "hslb_cnn.hip")).read()
    body = src[src.index("float phi_cdf_fast("):src.index("phi_cdf_ref(")]
    first = re.search(r"float p = (-?[0-9.e-]+)f;", body).group(1)
    rest = re.findall(r"p = fmaf\(p, u, (-?[0-9.e-]+)f\);", body)
    return [float(v) for v in reversed([first] + rest)]   # lowest degree first


def test_kernel_coefficients_are_the_fit():
    g = _gen()
    c, err = g.fit()
    assert err < 1e-8
    kc = _kernel_coefficients()
    assert len(kc) == g.DEG + 1
    assert np.array_equal(np.float32(kc), np.float32(c))
    assert abs(sum(kc) - 1.0) < 1e-6     # E(0) = 1


def _gelu_fast_f32(z, coef):
    f = np.float32
    z = z.astype(np.float32)
    t = np.abs(z)
    q = z * z
    ql = (z.astype(np.float64) ** 2 - q).astype(np.float32)               # fmaf(z, z, -q)
    CH, CL = f(-0.7213475108146667), f(-9.629815167500055e-09)
    p = (q * CH).astype(np.float32)
    pl1 = (q.astype(np.float64) * CH - p).astype(np.float32)                # fmaf(q, CH, -p)
    pl2 = (q.astype(np.float64) * CL + np.float64((ql * CH).astype(np.float32))).astype(np.float32)
    pl = (pl1 + pl2).astype(np.float32)
    corr = (pl.astype(np.float64) * np.float64(f(0.69314718055994531)) + 1.0).astype(np.float32)
    e = np.exp2(p.astype(np.float64)).astype(np.float32) * corr             # v_exp_f32(p) (1 + ln2 pl)
    u = (1.0 / (0.3 * t.astype(np.float64) + 1.0)).astype(np.float32)     # rcp(fmaf(0.3, t, 1))
    p = np.full_like(u, f(coef[-1]))
    for k in range(len(coef) - 2, -1, -1):
        p = (p.astype(np.float64) * u + np.float64(f(coef[k]))).astype(np.float32)
    tail = f(0.5) * e * (u * p)
    phi = np.where(z < 0, tail, f(1) - tail)
    return z * phi


def test_fast_gelu_is_within_the_tie_window():
    coef = _kernel_coefficients()
    z = np.concatenate([np.linspace(-13.0, 13.0, 400001),   # below -13 the kernel takes erfcf
                        np.random.default_rng(5).standard_normal(200000) * 2.0]).astype(np.float32)
    zd = z.astype(np.float64)
    ref = zd * 0.5 * erfc(-zd / np.sqrt(2.0))
    got = _gelu_fast_f32(z, coef).astype(np.float64)
    nz = ref != 0.0
    ulp = np.spacing(np.abs(ref[nz]).astype(np.float32)).astype(np.float64)
    err_ulps = np.abs(got[nz] - ref[nz]) / ulp
    rel = np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])
    print(f"largest error {err_ulps.max():.1f} ulp, {rel.max():.2e} relative")
    assert err_ulps.max() <= 16.0
    assert rel.max() <= 1e-6
