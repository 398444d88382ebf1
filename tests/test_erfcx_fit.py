"""The polynomial the FP32 split kernels use for erfcx(u) = exp(u^2)
erfc(u): its coefficients, evaluated in FP32 by Horner's rule (fused
multiply-add emulated exactly), match scipy's erfcx to 3e-7 relative on
the whole domain 0 <= u <= 2.5, and the header matches its generator."""
import os
import re

import numpy as np
from scipy import special

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1812_07313_amd", "csrc")


def _header():
    with open(os.path.join(CSRC, "erfcx_fit.h")) as f:
        text = f.read()
    dom = float(re.search(r"kErfcxDomain = ([0-9.]+)f", text).group(1))
    coef = [float(v) for v in re.findall(r"^\s+([-+0-9.e]+)f,$", text, re.M)]
    return dom, np.array(coef)


def test_fit_accuracy_fp32():
    dom, c = _header()
    assert dom == 2.5 and len(c) == 13
    u = np.linspace(0.0, dom, 200001).astype(np.float32)
    # s = fma(u, fl32(2/dom), -1): the product of two FP32 values and the
    # subtraction are exact in FP64, so one rounding to FP32 emulates it
    s = (u.astype(np.float64) * np.float64(np.float32(2 / dom)) - 1.0).astype(np.float32)
    c32 = c.astype(np.float32)
    acc = np.full_like(s, c32[-1])
    for k in range(len(c32) - 2, -1, -1):
        # a*b + c with a, b, c in FP32 is exact in FP64 up to one rounding
        acc = (acc.astype(np.float64) * s.astype(np.float64) +
               np.float64(c32[k])).astype(np.float32)
    ref = special.erfcx(u.astype(np.float64))
    assert np.max(np.abs(acc / ref - 1.0)) < 3e-7


def test_header_matches_generator():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "gen", os.path.join(CSRC, "gen_erfcx_fit.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    _, c = _header()
    np.testing.assert_allclose(c, gen.fit(), rtol=1e-8, atol=1e-12)
