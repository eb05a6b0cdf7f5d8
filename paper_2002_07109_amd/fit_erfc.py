"""Coefficients of the FP32 erfc in the pair kernels (csrc/bounce_device.hpp).

erfc(x) = exp(-x^2) Q(t), t = 1 / (1 + P x), where Q is a polynomial of degree
N in t fitted to erfcx(x) = erfc(x) exp(x^2) on 0 <= x <= X by iteratively
reweighted least squares on the relative error (Lawson's method towards the
minimax fit).  Running this prints the coefficients (lowest degree first, as
FP32 literals) and the relative error of the fit and of its FP32 Horner
evaluation.  Beyond X, exp(-x^2) < 1.7e-28 makes the term negligible.
"""
import numpy as np
from scipy.special import erfcx

P, N, X = 0.4, 9, 8.0


def fit(p=P, n=N, xmax=X, iters=40):
    x = np.linspace(0.0, xmax, 40001)
    t = 1.0 / (1.0 + p * x)
    y = erfcx(x)
    A = np.vander(t, n + 1, increasing=True)
    w = np.ones_like(x)
    for _ in range(iters):
        c, *_ = np.linalg.lstsq(A * (w / y)[:, None], w, rcond=None)
        e = (A @ c - y) / y
        w = w * (1.0 + 50.0 * np.abs(e) / np.abs(e).max())
        w /= w.mean()
    return c


def horner32(c, p, x):
    """Q(t) in FP32: t from an FP32 division, each step one fused multiply-add."""
    x = x.astype(np.float32)
    t = (np.float32(1) / (np.float32(1) + np.float32(p) * x)).astype(np.float32)
    c32 = c.astype(np.float32)
    q = np.full_like(t, c32[-1])
    for k in range(len(c32) - 2, -1, -1):
        q = (q.astype(np.float64) * t.astype(np.float64) + np.float64(c32[k])).astype(np.float32)
    return q


if __name__ == "__main__":
    c = fit()
    xs = np.linspace(0.0, X, 400001)
    t = 1.0 / (1.0 + P * xs)
    rel = np.abs(np.polynomial.polynomial.polyval(t, c) / erfcx(xs) - 1.0).max()
    rel32 = np.abs(horner32(c, P, xs) / erfcx(xs) - 1.0).max()
    print(f"P = {P}, degree {N}, 0 <= x <= {X}: fit {rel:.2e}, FP32 evaluation {rel32:.2e}")
    for k, v in enumerate(c.astype(np.float32)):
        print(f"c{k} = {float(v)!r}f")
