"""CPU-side checks of libbhq: the library loads, exports every symbol that
include/bhq.h declares, and reports the failures that can be forced without
a GPU (no device, bad arguments)."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from paper_1812_07313_amd import bhq


def _declared_symbols():
    with open(os.path.join(ROOT, "include", "bhq.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bhq_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = bhq.lib()
    names = _declared_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
        assert name in bhq.SIGNATURES, name


def _have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(_have_gpu(), reason="checks the no-device path")
def test_create_without_gpu_reports_nodev():
    with pytest.raises(bhq.BhqError) as ei:
        bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    assert ei.value.code == bhq.E_NODEV
    assert "GPU" in bhq.bhq_last_error(None)


def test_create_argument_errors():
    L = bhq.lib()
    assert L.bhq_create(None, 0, bhq.QUAD, bhq.FP32_OFS64) == bhq.E_ARG
    h = ctypes.c_void_p()
    assert L.bhq_create(ctypes.byref(h), 0, 9, bhq.FP32_OFS64) == bhq.E_ARG
    assert L.bhq_create(ctypes.byref(h), 0, bhq.QUAD, 5) == bhq.E_ARG
    assert h.value is None


def test_null_context_calls_are_rejected():
    L = bhq.lib()
    assert L.bhq_set_eps(None, 0.1) == bhq.E_ARG
    assert L.bhq_compute(None, None) == bhq.E_ARG
    assert L.bhq_get_result(None, None, None) == bhq.E_ARG
    assert L.bhq_destroy(None) == bhq.OK
    assert L.bhq_lists_free(None) == bhq.OK


def test_build_lists_argument_errors():
    x = np.random.default_rng(0).random((100, 3))
    m = np.full(100, 0.01)
    for kw in (dict(theta=-0.1, ncrit=16), dict(theta=0.5, ncrit=0),
               dict(theta=0.5, ncrit=16, nleaf=32),
               dict(theta=0.5, ncrit=16, box=-1.0)):
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_build_lists(x, m, **kw)
        assert ei.value.code == bhq.E_ARG
    xb = x.copy()
    xb[3, 1] = np.nan
    with pytest.raises(bhq.BhqError) as ei:
        bhq.bhq_build_lists(xb, m, 0.5, 16)
    assert ei.value.code == bhq.E_NONFINITE


def test_bench_refuses_several_gpus():
    """bench.py --gpus N with N > 1 exits with a message before touching a
    GPU (one GPU only)."""
    import subprocess
    import sys
    from conftest import ROOT
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_bench_lane_slot_fraction():
    """The slicing model behind bench.py's lane_slot_fraction, on cases
    counted by hand."""
    import bench
    # 64 i-particles, 2 per thread: 32 threads a slice, 8 slices fill the
    # 256 threads; 256 entries are 32 steps of every slice: no empty slot
    assert bench.lane_slot_fraction([0, 64], [0, 256], [0, 0], 256, 2) == 1.0
    # 3 i-particles: 2 threads a slice, 128 slices (4 waves, 512 slots a
    # step); 5 particle entries take one step: 15 of 512 slots
    assert bench.lane_slot_fraction([0, 3], [0, 5], [0, 0], 256, 2) == 15 / 512
    # cells weigh 34 operations against 14: 64 i-particles over 256 entries
    # of each kind (1.0) plus a group of 3 with 5 cells (15 / 512)
    f = bench.lane_slot_fraction([0, 64, 67], [0, 256, 256], [0, 256, 261], 256, 2)
    useful = 64 * 256 * 14 + 64 * 256 * 34 + 3 * 5 * 34
    issued = 64 * 256 * 14 + 64 * 256 * 34 + 512 * 34
    assert f == pytest.approx(useful / issued, rel=1e-15)
    # 600 i-particles in two passes: 512 (256 threads, one slice, 256-entry
    # tiles of 256 steps) and 88 (44 threads a slice, 5 slices in 4 waves,
    # 255-entry tiles of 51 steps); 300 entries: 256 + 44 steps in the
    # first pass, 51 + 9 in the second
    f = bench.lane_slot_fraction([0, 600], [0, 300], [0, 0], 256, 2)
    assert f == pytest.approx(600 * 300 / (512 * (256 + 44) + 512 * (51 + 9)), rel=1e-15)


def test_bench_split_pricing():
    """The split kernels are priced per term inside the cutoff with the
    counts of their own precision (FP32 cubics, FP64 polynomials)."""
    import bench
    n_pp, n_pc = 10 ** 12, 10 ** 11
    r32 = bench._priced(bhq.SPLIT_QUAD, n_pp, n_pc, 1000.0, 100.0)
    r64 = bench._priced(bhq.SPLIT_QUAD, n_pp, n_pc, 1000.0, 100.0, fp64=True)
    assert r32["tflops"] == round((36 * n_pp + 97 * n_pc) / 1e12, 3)
    assert r64["tflops"] == round((62 * n_pp + 123 * n_pc) / 1e12, 3)
    # the non-split kernels ignore the flag
    assert bench._priced(bhq.QUAD, n_pp, n_pc, 1000.0, 100.0, fp64=True) == \
        bench._priced(bhq.QUAD, n_pp, n_pc, 1000.0, 100.0)
