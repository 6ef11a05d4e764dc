"""Coefficients of the GELU evaluation used by the MLP kernels (csrc/mlp.hpp).

GELU in the exact erf form, gelu(z) = z Phi(z) with Phi the standard normal
distribution function, equals max(z, 0) - |z| Phi(-|z|) for every z (for z >= 0
because Phi(z) = 1 - Phi(-z), for z < 0 directly).  The kernels evaluate

    Phi(-x) ~= 2^H(x),   x = min(|z|, X),   H a polynomial of degree DEG,

so that one exponential and DEG fused multiply-adds give the activation.  H is
fitted to log2 Phi(-x) on [0, X] by Lawson's iteratively reweighted least squares
(a Chebyshev basis for conditioning), minimising the largest absolute error of
the correction term x Phi(-x), then converted to monomials in x.  Beyond X the
term |z| Phi(-|z|) is below X Phi(-X) ~ 6e-9 (X = 6).

Run as a script to print the coefficients and the errors of the FP32 evaluation
(FP32 rounding after every fused multiply-add, as the kernels do).
"""
from __future__ import annotations

import numpy as np

DEG = 6
X = 6.0


def fit(deg: int = DEG, x_max: float = X, iters: int = 300, samples: int = 60001) -> np.ndarray:
    """Monomial coefficients (increasing powers of x) of H."""
    from scipy.special import log_ndtr

    x = np.linspace(0.0, x_max, samples)
    target = log_ndtr(-x) / np.log(2.0)
    term = x * np.exp(log_ndtr(-x))  # x Phi(-x)
    t = 2.0 * x / x_max - 1.0
    V = np.polynomial.chebyshev.chebvander(t, deg)
    w = np.ones_like(x)
    best = (np.inf, None)
    for _ in range(iters):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(V * sw[:, None], target * sw, rcond=None)
        e = np.abs(term * (np.exp2(V @ c - target) - 1.0))
        if e.max() < best[0]:
            best = (e.max(), c)
        w = w * (e / e.max() + 1e-4)
        w /= w.max()
    cheb = np.polynomial.Chebyshev(best[1], domain=[0.0, x_max])
    return cheb.convert(kind=np.polynomial.Polynomial).coef


def gelu_fp32(z: np.ndarray, coef32: np.ndarray, x_max: float = X) -> np.ndarray:
    """The kernels' evaluation with FP32 rounding after each step (fma rounds once)."""
    z = np.asarray(z, dtype=np.float32)
    a = np.abs(z)
    x = np.minimum(a, np.float32(x_max))
    h = np.full(x.shape, coef32[-1], dtype=np.float32)
    for k in range(len(coef32) - 2, -1, -1):
        h = (h.astype(np.float64) * x.astype(np.float64) + np.float64(coef32[k])).astype(np.float32)
    e = np.exp2(h.astype(np.float64)).astype(np.float32)
    return (-(a.astype(np.float64)) * e.astype(np.float64) + np.maximum(z, 0).astype(np.float64)).astype(np.float32)


def gelu_exact(z: np.ndarray) -> np.ndarray:
    from scipy.special import ndtr

    z = np.asarray(z, dtype=np.float64)
    return z * ndtr(z)


if __name__ == "__main__":
    c = fit()
    c32 = c.astype(np.float32)
    z = np.linspace(-12.0, 12.0, 480001).astype(np.float32).astype(np.float64)  # FP32 inputs
    g = gelu_fp32(z, c32)
    err = np.abs(g.astype(np.float64) - gelu_exact(z))
    excess = err - 0.5 * np.spacing(np.abs(g))  # beyond the rounding of the FP32 result itself
    print("constexpr float kGeluH[%d] = {%s};" % (len(c32), ", ".join("%.9ef" % v for v in c32)))
    print(f"FP32 evaluation on [-12, 12]: max |error| {err.max():.3e}, "
          f"max |error| beyond half an ulp of the result {excess.max():.3e}")
