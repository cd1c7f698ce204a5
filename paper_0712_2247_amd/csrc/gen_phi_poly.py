"""Coefficients of the FP32 normal-distribution function of the learned
force's GELU (phi_cdf in hslb_cnn.hip).

For t >= 0, Phi(-t) = exp(-t^2/2) E(t) / 2 with E(t) = exp(t^2/2) erfc(t/sqrt 2),
a smooth function that falls from 1 to sqrt(2/pi)/t.  With u = 1/(1 + A t),
E(t) = u P(u) where P is a polynomial of degree DEG fitted here by weighted
least squares to the relative error of E on t in [0, 16], the weights raised
where the error peaks (Lawson's iteration toward the minimax fit).  Prints the
coefficients as FP32 literals, lowest degree first, and the fit's largest
relative error in double precision.  Needs numpy and scipy.
"""
import numpy as np
from scipy.special import erfcx

A, DEG, T = 0.3, 9, 16.0


def fit(iters: int = 40):
    t = np.concatenate([np.linspace(0.0, 2.0, 6000), np.linspace(2.0, T, 12000)])
    u = 1.0 / (1.0 + A * t)
    E = erfcx(t / np.sqrt(2.0))
    V = np.vander(u, DEG + 1, increasing=True)
    w = np.ones_like(t)
    for _ in range(iters):
        W = w * u / E
        c, *_ = np.linalg.lstsq(V * W[:, None], (E / u) * W, rcond=None)
        r = (u * (V @ c) - E) / E
        w = w * (1.0 + 50.0 * np.abs(r) / np.abs(r).max())
    return c, float(np.abs(r).max())


if __name__ == "__main__":
    c, err = fit()
    print(f"// A = {A}, degree {DEG}, largest relative error of E on [0, {T:g}]: {err:.2e}")
    for k, v in enumerate(c):
        print(f"    {repr(float(np.float32(v)))}f,  // u^{k}")
