"""bhq_compute_noalloc (the entry point for callers that cannot allocate)
against bhq_compute on the same context: results written straight to
caller GPU arrays, bitwise equal to bhq_compute's, for two inputs in a row
(the second smaller), with the j-split parts and the persistent queue
counters in the library's static working memory; inputs whose parts exceed
that memory are refused."""
import numpy as np
import pytest

from _parity import log
from paper_1812_07313_amd import bhq, synth

pytestmark = pytest.mark.gpu


def _lists(ctx, x, m, theta, ncrit, eps):
    L = bhq.bhq_build_lists(x, m, theta, ncrit)
    try:
        bhq.bhq_set_lists_indexed(ctx, L, x, m)
    finally:
        bhq.bhq_lists_free(L)
    bhq.bhq_set_eps(ctx, eps)


@pytest.mark.parametrize("precision", [bhq.FP32_OFS64, bhq.FP64])
def test_noalloc_matches_compute(precision):
    torch = pytest.importorskip("torch")
    ctx = bhq.bhq_create(0, bhq.QUAD, precision)
    try:
        for n in (16384, 4096):   # the second input is smaller
            x, m = synth.plummer(n, synth.rng(40 + n))
            _lists(ctx, x, m, 0.5, 64, 1.0 / 64)
            for shape in ((256, 2, 0, 1, 0, 4), (256, 1, 0, 0, 0, 8), (256, 2, 0, 0, 0, 1),
                          (128, 2, 0, 1, 0, 1)):
                log("case noalloc n=%d precision=%s shape=%s"
                    % (n, bhq.PRECISION_NAMES[precision], shape))
                bhq.bhq_set_tuning(ctx, *shape)
                bhq.bhq_set_kernel(ctx, bhq.QUAD, precision)
                bhq.bhq_compute(ctx)
                a_ref, p_ref = bhq.bhq_get_result(ctx, n)
                a = torch.full((n, 3), float("nan"), dtype=torch.float64, device="cuda")
                p = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
                bhq.bhq_compute_noalloc(ctx, a, p)
                torch.cuda.synchronize()
                assert bhq.bhq_get_kernel_ms(ctx) > 0.0
                assert np.array_equal(a.cpu().numpy(), a_ref), shape
                assert np.array_equal(p.cpu().numpy(), p_ref), shape
                # without the potential
                a2 = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
                bhq.bhq_compute_noalloc(ctx, a2, None)
                torch.cuda.synchronize()
                assert np.array_equal(a2.cpu().numpy(), a_ref), shape
    finally:
        bhq.bhq_destroy(ctx)


def test_noalloc_refuses_parts_beyond_its_memory():
    torch = pytest.importorskip("torch")
    n = 1 << 18
    x, m = synth.plummer(n, synth.rng(47))
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        _lists(ctx, x, m, 0.7, 256, 0.01)
        a = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
        # 8 parts x 2^18 particles x 16 B = 32 MiB > 16 MiB
        bhq.bhq_set_tuning(ctx, 256, 2, 0, 0, 0, 8)
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_compute_noalloc(ctx, a)
        assert ei.value.code == bhq.E_RANGE
        assert "16777216" in bhq.bhq_last_error(ctx)
        # 4 parts fit exactly (16 MiB) and give bhq_compute's result
        bhq.bhq_set_tuning(ctx, 256, 2, 0, 0, 0, 4)
        bhq.bhq_compute(ctx)
        a_ref, _ = bhq.bhq_get_result(ctx, n)
        bhq.bhq_compute_noalloc(ctx, a)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), a_ref)
        # host memory is refused before anything is launched
        h = np.zeros((n, 3))
        assert bhq.lib().bhq_compute_noalloc(ctx, h.ctypes.data, None, None) == bhq.E_ARG
        assert bhq.lib().bhq_compute_noalloc(ctx, None, None, None) == bhq.E_ARG
    finally:
        bhq.bhq_destroy(ctx)


@pytest.mark.parametrize("precision", [bhq.FP32_OFS64, bhq.FP64])
def test_noalloc_split_kernel(precision):
    """The periodic split kernel through bhq_compute_noalloc equals
    bhq_compute, whole lists and cut into parts, for two inputs in a row
    (the second smaller)."""
    torch = pytest.importorskip("torch")
    ctx = bhq.bhq_create(0, bhq.SPLIT_QUAD, precision)
    try:
        for nside in (24, 16):
            x, m = synth.perturbed_lattice(nside, synth.rng(50 + nside))
            rs = 1.25 / nside
            rcut = 4.5 * rs
            L = bhq.bhq_build_lists(x, m, 0.5, 64, box=1.0, rcut=rcut)
            try:
                bhq.bhq_set_lists_indexed(ctx, L, x, m)
            finally:
                bhq.bhq_lists_free(L)
            bhq.bhq_set_split(ctx, rs, rcut, 1.0)
            n = len(m)
            for shape in ((256, 2, 0, 0, 0, 1), (256, 2, 0, 1, 0, 4)):
                log("case noalloc split n=%d precision=%s shape=%s"
                    % (n, bhq.PRECISION_NAMES[precision], shape))
                bhq.bhq_set_tuning(ctx, *shape)
                bhq.bhq_set_kernel(ctx, bhq.SPLIT_QUAD, precision)
                bhq.bhq_compute(ctx)
                a_ref, p_ref = bhq.bhq_get_result(ctx, n)
                a = torch.full((n, 3), float("nan"), dtype=torch.float64, device="cuda")
                p = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
                bhq.bhq_compute_noalloc(ctx, a, p)
                torch.cuda.synchronize()
                assert np.array_equal(a.cpu().numpy(), a_ref), shape
                assert np.array_equal(p.cpu().numpy(), p_ref), shape
    finally:
        bhq.bhq_destroy(ctx)
