"""The FP32 erfc of the pair kernels: erfc(x) = exp(-x^2) Q(1 / (1 + 0.4 x)) with
the degree-9 polynomial Q whose coefficients csrc/bounce_device.hpp holds.
Checked here, on the CPU, against scipy's erfcx (an independent evaluation of
erfc(x) exp(x^2)) over the fitted range 0 <= x <= 8 and a little beyond, and
against the coefficients fit_erfc.py computes."""
import os
import re

import numpy as np
from scipy.special import erfc, erfcx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HPP = os.path.join(ROOT, "paper_2002_07109_amd", "csrc", "bounce_device.hpp")


def _coefficients():
    src = open(HPP).read()
    body = src[src.index("float erfcx_fit(float x)"):]
    body = body[:body.index("return q;")]
    lead = float(re.search(r"float q = ([-0-9.e]+)f;", body).group(1))
    rest = [float(v) for v in re.findall(r"q = fmaf\(q, t, ([-0-9.e]+)f\);", body)]
    p = float(re.search(r"fmaf\(([0-9.]+)f, x, 1\.0f\)", body).group(1))
    # Horner from the highest degree down: lead, then rest in order
    return p, np.array([lead] + rest)[::-1]          # lowest degree first


def _q(x, p, c):
    t = 1.0 / (1.0 + p * x)
    return np.polynomial.polynomial.polyval(t, c)


def test_fit_matches_erfcx_on_its_range():
    p, c = _coefficients()
    assert p == 0.4 and len(c) == 10
    x = np.linspace(0.0, 8.0, 200001)
    rel = np.abs(_q(x, p, c) / erfcx(x) - 1.0).max()
    assert rel < 3e-8, rel
    # erfc itself (the product with exp(-x^2)) where it is not negligible
    xs = np.linspace(0.0, 6.0, 60001)
    rel_e = np.abs(np.exp(-xs * xs) * _q(xs, p, c) / erfc(xs) - 1.0).max()
    assert rel_e < 3e-8, rel_e
    # at x = 0, erfc = 1: the coefficients sum to 1
    assert abs(c.sum() - 1.0) < 1e-7


def test_fit_beyond_its_range_stays_bounded():
    p, c = _coefficients()
    x = np.linspace(8.0, 12.0, 4001)
    rel = np.abs(_q(x, p, c) / erfcx(x) - 1.0).max()
    assert rel < 1e-3, rel          # the product with exp(-x^2) < 1.7e-28 there


def test_header_holds_the_coefficients_the_script_fits():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "fit_erfc", os.path.join(ROOT, "paper_2002_07109_amd", "fit_erfc.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    p, c = _coefficients()
    assert p == mod.P
    fitted = mod.fit().astype(np.float32).astype(np.float64)
    assert np.allclose(fitted, c, rtol=0, atol=1e-7), (fitted, c)
