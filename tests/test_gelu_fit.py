"""The GELU evaluation of the MLP kernels (csrc/mlp.hpp): max(z, 0) - |z| 2^H(min(|z|, 6)).

The coefficients in the header are those gelu_fit.py fits, and the kernels' FP32
evaluation of them stays within 1e-7 of the exact erf form beyond half an ulp of
the FP32 result on [-12, 12] (exact form: z Phi(z) with scipy's normal distribution
function, an independent evaluation)."""
import os
import re

import numpy as np
import pytest

pytest.importorskip("scipy")
from paper_1505_06900_amd import gelu_fit as G  # noqa: E402

HEADER = os.path.join(os.path.dirname(__file__), "..", "paper_1505_06900_amd", "csrc", "mlp.hpp")


def header_coefficients():
    text = open(HEADER).read()
    m = re.search(r"kGeluH\[(\d+)\]\s*=\s*\{([^}]*)\}", text)
    vals = [float(v.strip().rstrip("f")) for v in m.group(2).split(",") if v.strip()]
    assert len(vals) == int(m.group(1))
    return np.array(vals, dtype=np.float32)


def test_header_holds_the_fitted_coefficients():
    c = header_coefficients()
    fit = G.fit().astype(np.float32)
    assert len(c) == G.DEG + 1
    np.testing.assert_allclose(c, fit, rtol=1e-5, atol=1e-9)


def test_fp32_evaluation_error():
    c = header_coefficients()
    z = np.linspace(-12.0, 12.0, 240001).astype(np.float32).astype(np.float64)
    g = G.gelu_fp32(z, c)
    err = np.abs(g.astype(np.float64) - G.gelu_exact(z))
    assert np.max(err - 0.5 * np.spacing(np.abs(g))) <= 1e-7
    # special points: gelu(0) = 0 exactly, odd-symmetric part, large |z|
    assert G.gelu_fp32(np.array([0.0]), c)[0] == 0.0
    big = np.array([-50.0, -8.0, 8.0, 50.0])
    np.testing.assert_allclose(G.gelu_fp32(big, c), G.gelu_exact(big), atol=1e-7 * 50)
