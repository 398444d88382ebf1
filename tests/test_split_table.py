"""The table the FP32 split kernels use for the Gaussian-split radial
functions (csrc/split_table.h): its piecewise cubics, evaluated in FP32 as
the kernels do (interval q = floor(t), f = t - q, Horner's rule with fused
multiply-adds emulated exactly), match the functions computed from scipy's
erfc and numpy's exp to 3e-7 relative on 0 <= u <= 2.5, its first entries
reproduce erfc(0) = 1, g(0) = 1, G2(0) = 3, G3(0) = 15, and the header
matches its generator.  The FP64 kernels' table of exp(-u^2) and
erfcx(u) = exp(u^2) erfc(u) (csrc/split_table64.h), evaluated as they
evaluate it, matches both functions, and their product erfc, computed with
30 significant digits to a few 1e-16."""
import importlib.util
import os
import re

import numpy as np
from scipy import special

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1812_07313_amd", "csrc")


def _header():
    with open(os.path.join(CSRC, "split_table.h")) as f:
        text = f.read()
    dom = float(re.search(r"kSplitDomain = ([0-9.]+)f", text).group(1))
    n = int(re.search(r"kSplitIntervals = (\d+);", text).group(1))
    body = text[text.index("kSplitTable["):]
    vals = [float(v) for v in re.findall(r"([-+0-9.]+e[-+0-9]+)f", body)]
    return dom, n, np.array(vals, np.float32).reshape(4, n + 1, 4)


def _reference(u):
    """ec, g, G2, G3 written out from their definitions (FP64)."""
    c = 2.0 / np.sqrt(np.pi)
    E = np.exp(-u * u)
    ec = special.erfc(u)
    g = ec + c * u * E
    h = 2.0 * c * u ** 3 * E
    k = 2.0 * u * u * h
    return ec, g, 3.0 * g + h, 15.0 * g + 5.0 * h + k


def _fma32(a, b, c):
    # a*b + c of FP32 values is exact in FP64 up to one rounding
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def test_table_accuracy_fp32():
    dom, n, tab = _header()
    assert dom == 2.5 and n == 128
    t = np.linspace(0.0, n * (1.0 + 1e-6), 300001).astype(np.float32)
    q = np.floor(t).astype(np.int64)
    f = (t - q).astype(np.float32)  # exact in FP32
    u = t.astype(np.float64) * (dom / n)
    for j, ref in enumerate(_reference(u)):
        c = tab[j][q]
        acc = c[:, 3]
        for k in (2, 1, 0):
            acc = _fma32(acc, f, c[:, k])
        assert np.max(np.abs(acc / ref - 1.0)) < 3e-7, j


def test_table_at_zero():
    _, _, tab = _header()
    assert list(tab[:, 0, 0]) == [1.0, 1.0, 3.0, 15.0]


def test_header_matches_generator():
    spec = importlib.util.spec_from_file_location(
        "gen", os.path.join(CSRC, "gen_split_table.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    _, _, tab = _header()
    # the header holds the generator's FP64 coefficients rounded to FP32
    np.testing.assert_allclose(tab, gen.table(), rtol=1.2e-7, atol=0)


def test_pieces_join():
    """Neighbouring cubics meet in value and slope (cubic Hermite pieces
    share their end values and derivatives), up to FP32 rounding: a piece
    evaluated at f = 1 equals the next at f = 0, and so do their slopes."""
    dom, n, tab = _header()
    c = tab.astype(np.float64)
    end_val = c[:, :-1].sum(axis=2)                                   # f = 1
    end_slope = c[:, :-1, 1] + 2 * c[:, :-1, 2] + 3 * c[:, :-1, 3]   # dF/df at 1
    start_val, start_slope = c[:, 1:, 0], c[:, 1:, 1]
    scale = np.abs(c[:, :, 0]).max(axis=1)[:, None]
    assert np.max(np.abs(end_val - start_val) / scale) < 4e-7
    assert np.max(np.abs(end_slope - start_slope) / scale) < 1e-7


def test_generator_derivatives():
    """The exact derivatives the generator gives the Hermite pieces agree
    with central differences of its function values."""
    spec = importlib.util.spec_from_file_location(
        "gen", os.path.join(CSRC, "gen_split_table.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    u = np.linspace(0.05, 2.6, 200)
    h = 1e-5
    vp, _ = gen.funcs(u + h)
    vm, _ = gen.funcs(u - h)
    _, ders = gen.funcs(u)
    for j in range(4):
        num = (vp[j] - vm[j]) / (2 * h)
        assert np.max(np.abs(num - ders[j])) < 1e-8 * max(1.0, np.max(np.abs(ders[j]))), j


def _header64():
    with open(os.path.join(CSRC, "split_table64.h")) as f:
        text = f.read()
    dom = float(re.search(r"kTab64Domain = ([0-9.]+);", text).group(1))
    n = int(re.search(r"kTab64Intervals = (\d+);", text).group(1))
    de = int(re.search(r"kExpDegree = (\d+);", text).group(1))
    dx = int(re.search(r"kErfcxDegree = (\d+);", text).group(1))
    stride = int(re.search(r"kTab64Stride = (\d+);", text).group(1))
    assert stride == de + dx + 2
    body = text[text.index("kTab64["):]
    body = body[body.index("= {"):]
    vals = [float(v) for v in re.findall(r"([-+0-9.]+e[-+0-9]+)", body)]
    return dom, n, de, dx, np.array(vals).reshape(n, stride)


def _horner_fma(c, f):
    """Horner's rule with fused multiply-adds (emulated exactly: the
    rational result rounded once)."""
    from fractions import Fraction
    x = float(c[-1])
    for k in range(len(c) - 2, -1, -1):
        x = float(Fraction(x) * Fraction(f) + Fraction(float(c[k])))
    return x


def _tab64_kernel(u, dom, n, de, tab):
    """The FP64 kernels' evaluation: t = u n / dom (exact: a power-of-two
    scale), q = floor(t), f = t - q; exp(-u^2) and erfcx(u) from row q."""
    t = u * (n / dom)
    q = int(t)
    f = t - q
    return _horner_fma(tab[q, :de + 1], f), _horner_fma(tab[q, de + 1:], f)


def test_fp64_exp_erfcx_table():
    import mpmath as mp
    dom, n, de, dx, tab = _header64()
    assert (dom, n, de, dx) == (4.0, 64, 9, 7)
    # exp(0) = 1 exactly; erfcx(0) = 1 within one unit in the last place (the
    # degree-7 interpolant's error at the interval's end)
    assert tab[0, 0] == 1.0
    assert abs(tab[0, de + 1] - 1.0) <= 2.0 ** -52
    u = np.concatenate([np.linspace(0.0, dom, 1601, endpoint=False),
                        np.nextafter(np.arange(1, n + 1) * (dom / n), 0.0)])
    worst_e = worst_x = worst_c = 0.0
    with mp.workdps(30):
        for v in u:
            e, x = _tab64_kernel(float(v), dom, n, de, tab)
            w = mp.mpf(float(v))
            worst_e = max(worst_e, abs(float(e / mp.exp(-w * w) - 1)))
            worst_x = max(worst_x, abs(float(x / (mp.exp(w * w) * mp.erfc(w)) - 1)))
            # the kernels' erfc: the two table values multiplied in FP64
            worst_c = max(worst_c, abs(float((e * x) / mp.erfc(w) - 1)))
    assert worst_e < 1e-15, worst_e
    assert worst_x < 1e-15, worst_x
    assert worst_c < 2e-15, worst_c


def test_fp64_header_matches_generator():
    spec = importlib.util.spec_from_file_location(
        "gen64", os.path.join(CSRC, "gen_split_table64.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    _, _, _, _, tab = _header64()
    assert np.array_equal(tab, np.array(gen.table()))
