"""The binary32 erfc of the effective-charge kernel: its constants are the ones the fit
script produces, and its error (evaluated in the kernel's binary32 operation order)
stays within the bounds the kernel's comment states. scipy's erfc is the reference."""
import os
import re

import numpy as np

from paper_2602_12052_amd import erfc_fit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def kernel_constants():
    src = open(os.path.join(ROOT, "paper_2602_12052_amd", "csrc", "effq.hip")).read()
    body = src[src.index("float erfc_pos(float z)"):]
    arr = body[body.index("c[10] = {") + len("c[10] = {"):body.index("};")]
    return np.array([float(v.rstrip("f")) for v in re.findall(r"[-+0-9.e]+f", arr)])


def test_kernel_constants_are_the_fit():
    c = kernel_constants()
    f = erfc_fit.fit()
    assert len(c) == erfc_fit.DEGREE + 1
    np.testing.assert_allclose(c, f.astype(np.float32), rtol=1e-8, atol=0)


def test_error_bounds():
    c = kernel_constants()
    assert erfc_fit.max_rel_error(c, 0.0, 2.0) < 6e-7
    assert erfc_fit.max_rel_error(c, 2.0, 4.0) < 2e-6
    assert erfc_fit.max_rel_error(c, 4.0, 9.0) < 7e-6


def test_erf_differences():
    """erf(b) - erf(a) assembled from the two erfc values as the kernel does, against
    scipy in binary64, on the argument pairs of a line deposition (a = -kq s,
    b = kq (1 - s))."""
    from scipy.special import erf
    c = kernel_constants()
    rng = np.random.default_rng(0)
    kq = rng.uniform(0.05, 6.0, 20000).astype(np.float32)
    s = rng.uniform(-2.0, 3.0, 20000).astype(np.float32)
    a = (-kq * s).astype(np.float32)
    b = (kq * (np.float32(1) - s)).astype(np.float32)
    ea = erfc_fit.eval_f32(c, np.abs(a)).astype(np.float64)
    eb = erfc_fit.eval_f32(c, np.abs(b)).astype(np.float64)
    got = np.where(a >= 0, ea - eb, np.where(b <= 0, eb - ea, 2.0 - ea - eb))
    ref = erf(b.astype(np.float64)) - erf(a.astype(np.float64))
    # absolute error relative to the largest difference (the scale of a node charge)
    assert np.max(np.abs(got - ref)) < 2e-6 * np.max(ref)
    big = ref > 1e-3
    assert np.max(np.abs(got[big] / ref[big] - 1)) < 5e-5
