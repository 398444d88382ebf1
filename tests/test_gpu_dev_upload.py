"""The device-pointer set calls (bhq_set_*_dev) against the host set calls:
the same lists handed over as torch tensors give bit for bit the forces of
the host upload (materialised lists, and index lists into pools), which
match the oracle; invalid device arrays are refused with the host calls'
error codes and leave the context as it was."""
import numpy as np
import pytest

import oracle as orc
from _parity import assert_parity, errors, log, run, upload
from paper_1812_07313_amd import bhq, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    x, m = synth.plummer(6000, synth.rng(21))
    T = orc.Tree(x, m, 0.5, 64)
    mat = orc.materialise(T, x, m)
    e2 = np.full(len(m), (1.0 / 64) ** 2)
    e2[::3] *= 1.5   # per-particle softening
    ref = orc.eval_lists(orc.QUAD_SOFT, mat, x, e2)
    return x, m, T, mat, e2, ref


def _t(torch, a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _upload_dev(torch, ctx, mat, x, e2, stream=None):
    i_idx = mat["i_idx"]
    bhq.bhq_set_groups_dev(ctx, _t(torch, mat["i_off"], np.int64), _t(torch, mat["gcenter"]),
                           _t(torch, mat["jp_off"], np.int64), _t(torch, mat["jc_off"], np.int64),
                           stream)
    bhq.bhq_set_i_dev(ctx, _t(torch, x[i_idx]), stream)
    bhq.bhq_set_eps2_i_dev(ctx, _t(torch, e2[i_idx]), stream)
    bhq.bhq_set_jp_dev(ctx, 0, _t(torch, mat["jp_x"]), _t(torch, mat["jp_m"]), stream)
    bhq.bhq_set_jc_dev(ctx, 0, _t(torch, mat["jc_x"]), _t(torch, mat["jc_m"]),
                       _t(torch, mat["jc_q"]), _t(torch, mat["jc_t"]), stream)


def test_dev_materialised_equals_host(case):
    torch = pytest.importorskip("torch")
    x, m, T, mat, e2, (a_ref, p_ref) = case
    ctx = bhq.bhq_create(0, bhq.QUAD_SOFT, bhq.FP32_OFS64)
    ctx2 = bhq.bhq_create(0, bhq.QUAD_SOFT, bhq.FP32_OFS64)
    try:
        upload(ctx, mat, x, eps2=e2)
        s = torch.cuda.Stream()
        log("case dev upload materialised (torch stream)")
        _upload_dev(torch, ctx2, mat, x, e2, stream=s)
        for prec in (bhq.FP32_OFS64, bhq.FP64):
            a0, p0 = run(ctx, mat, len(m), bhq.QUAD_SOFT, prec)
            a1, p1 = run(ctx2, mat, len(m), bhq.QUAD_SOFT, prec)
            assert np.array_equal(a0, a1) and np.array_equal(p0, p1), prec
            assert_parity(errors(a1, p1, a_ref, p_ref), prec, "dev upload")
        # chunked j-cells, as the host call allows
        njc = len(mat["jc_m"])
        h = njc // 3
        for lo, hi in ((0, h), (h, njc)):
            bhq.bhq_set_jc_dev(ctx2, lo, _t(torch, mat["jc_x"][lo:hi]), _t(torch, mat["jc_m"][lo:hi]),
                               _t(torch, mat["jc_q"][lo:hi]), _t(torch, mat["jc_t"][lo:hi]))
        a2, p2 = run(ctx2, mat, len(m), bhq.QUAD_SOFT, bhq.FP64)
        a0, p0 = run(ctx, mat, len(m), bhq.QUAD_SOFT, bhq.FP64)
        assert np.array_equal(a0, a2) and np.array_equal(p0, p2)
    finally:
        bhq.bhq_destroy(ctx)
        bhq.bhq_destroy(ctx2)


def test_dev_index_lists_equal_host(case):
    torch = pytest.importorskip("torch")
    x, m, T, mat, e2, _ = case
    i_idx = mat["i_idx"]
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    ctx2 = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        for c in (ctx, ctx2):
            bhq.bhq_set_groups(c, mat["i_off"], mat["gcenter"], mat["jp_off"], mat["jc_off"])
            bhq.bhq_set_i(c, x[i_idx])
            bhq.bhq_set_eps2_i(c, e2[i_idx])
        bhq.bhq_set_pool_particles(ctx, x, m)
        bhq.bhq_set_pool_cells(ctx, T.com, T.mass, T.q, T.trace)
        bhq.bhq_set_jp_idx(ctx, 0, T.jp_idx)
        bhq.bhq_set_jc_idx(ctx, 0, T.jc_node)
        log("case dev upload index lists")
        bhq.bhq_set_pool_particles_dev(ctx2, _t(torch, x), _t(torch, m))
        bhq.bhq_set_pool_cells_dev(ctx2, _t(torch, T.com), _t(torch, T.mass), _t(torch, T.q),
                                   _t(torch, T.trace))
        bhq.bhq_set_jp_idx_dev(ctx2, 0, _t(torch, T.jp_idx, np.int32))
        bhq.bhq_set_jc_idx_dev(ctx2, 0, _t(torch, T.jc_node, np.int32))
        for prec in (bhq.FP32_OFS64, bhq.FP64):
            a0, p0 = run(ctx, mat, len(m), bhq.QUAD, prec)
            a1, p1 = run(ctx2, mat, len(m), bhq.QUAD, prec)
            assert np.array_equal(a0, a1) and np.array_equal(p0, p1), prec
    finally:
        bhq.bhq_destroy(ctx)
        bhq.bhq_destroy(ctx2)


def test_dev_upload_errors_leave_context(case):
    torch = pytest.importorskip("torch")
    x, m, T, mat, e2, _ = case
    i_idx = mat["i_idx"]
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        _upload_dev(torch, ctx, mat, x, e2)
        a0, p0 = run(ctx, mat, len(m), bhq.QUAD, bhq.FP32_OFS64)
        log("case dev upload errors")

        def expect(code, fn, *args):
            with pytest.raises(bhq.BhqError) as ei:
                fn(ctx, *args)
            assert ei.value.code == code, (fn.__name__, ei.value)

        xb = x[i_idx].copy()
        xb[7, 1] = np.nan
        expect(bhq.E_NONFINITE, bhq.bhq_set_i_dev, _t(torch, xb))
        for bad in (0.0, 2.0 ** -127):
            eb = e2[i_idx].copy()
            eb[3] = bad
            expect(bhq.E_ARG, bhq.bhq_set_eps2_i_dev, _t(torch, eb))
        qb = mat["jc_q"].copy()
        qb[5, 2] = np.inf
        expect(bhq.E_NONFINITE, bhq.bhq_set_jc_dev, 0, _t(torch, mat["jc_x"]),
               _t(torch, mat["jc_m"]), _t(torch, qb))
        ob = mat["jp_off"].copy()
        ob[4], ob[5] = ob[5], ob[4] - 1
        expect(bhq.E_RANGE, bhq.bhq_set_groups_dev, _t(torch, mat["i_off"], np.int64),
               _t(torch, mat["gcenter"]), _t(torch, ob, np.int64),
               _t(torch, mat["jc_off"], np.int64))
        # a host pointer where device memory is required
        assert bhq.lib().bhq_set_i_dev(ctx, len(m), x[i_idx].ctypes.data, None) == bhq.E_ARG
        # the refused calls left the context as it was
        a1, p1 = run(ctx, mat, len(m), bhq.QUAD, bhq.FP32_OFS64)
        assert np.array_equal(a0, a1) and np.array_equal(p0, p1)
        # index lists: an index outside the pool
        bhq.bhq_set_pool_particles_dev(ctx, _t(torch, x), _t(torch, m))
        bad = T.jp_idx.astype(np.int32).copy()
        bad[-1] = len(m)
        expect(bhq.E_RANGE, bhq.bhq_set_jp_idx_dev, 0, _t(torch, bad))
    finally:
        bhq.bhq_destroy(ctx)
