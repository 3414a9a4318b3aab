"""Coefficients of the binary32 complementary error function used by the effective-charge
kernel (effq.hip), and the check of its error.

Form (Numerical Recipes, "erfcc": a Chebyshev fit after factoring out the Gaussian):
    erfc(z) = t * exp(-z^2 + P(t)),   t = 1 / (1 + z / 2),   z >= 0,
with P a polynomial in t. Here P is a least-squares Chebyshev fit of degree 9 of
log(erfc(z) / t) + z^2 over z in [0, 10] (t in [1/6, 1]), converted to the power basis
and rounded to binary32; the fit is made here with scipy's erfc as the target, the
coefficients are not taken from any library. Run as a script to print them.
"""
from __future__ import annotations

import numpy as np

DEGREE = 9
ZMAX = 10.0
LOG2E = 1.4426950408889634


def fit(degree: int = DEGREE, zmax: float = ZMAX, n: int = 200001) -> np.ndarray:
    """Power-basis coefficients c[0..degree] of P(t) (binary64)."""
    from scipy.special import erfc
    z = np.linspace(0.0, zmax, n)
    t = 1.0 / (1.0 + 0.5 * z)
    y = np.log(erfc(z) / t) + z * z
    ch = np.polynomial.chebyshev.Chebyshev.fit(t, y, degree, domain=[t.min(), 1.0])
    return ch.convert(kind=np.polynomial.Polynomial, domain=[-1, 1], window=[-1, 1]).coef


def eval_f32(coef, z) -> np.ndarray:
    """The kernel's evaluation order in binary32: t by a reciprocal, Horner with fused
    multiply-adds on the coefficients times log2e (binary32 products), exp2 of
    fma(-z log2e, z, P log2e), times t."""
    f32 = np.float32
    z = np.asarray(z, np.float32)
    l2e = f32(LOG2E)
    c = [f32(f32(a) * l2e) for a in coef]
    t = (f32(1) / (f32(1) + f32(0.5) * z)).astype(f32)
    p = np.full_like(z, c[-1])
    for a in c[-2::-1]:
        p = (p.astype(np.float64) * t + a).astype(f32)            # one rounding per fma
    v = (-(z.astype(np.float64) * l2e)).astype(f32)
    arg = (v.astype(np.float64) * z + p).astype(f32)
    e = np.exp2(arg.astype(np.float64)).astype(f32)
    return (t * e).astype(f32)


def max_rel_error(coef, lo: float, hi: float, n: int = 100001) -> float:
    from scipy.special import erfc
    z = np.linspace(lo, hi, n).astype(np.float32)
    ref = erfc(z.astype(np.float64))
    return float(np.max(np.abs(eval_f32(coef, z).astype(np.float64) / ref - 1.0)))


def c_initializer(coef) -> str:
    return ", ".join(f"{float(np.float32(a)):.9e}f" for a in coef)


if __name__ == "__main__":
    c = fit()
    print("P(t) coefficients, t^0 first:")
    print("{" + c_initializer(c) + "}")
    for lo, hi in ((0, 2), (2, 4), (4, 9)):
        print(f"max relative error on [{lo}, {hi}]: {max_rel_error(c, lo, hi):.2e}")
