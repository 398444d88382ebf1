"""GPU: batched independent systems in one launch, the persistent group
queue, block sizes and HIP-graph replay, all through the C ABI and checked
against the FP64 oracle (or bitwise against the one-block-per-group launch,
which runs the same per-group arithmetic)."""
import numpy as np
import pytest

import oracle as orc
from _parity import assert_parity, errors, log, run, upload
from paper_1812_07313_amd import bhq, synth

pytestmark = pytest.mark.gpu

PRECS = [bhq.FP32_OFS64, bhq.FP64]


@pytest.fixture(scope="module")
def ctx():
    c = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    yield c
    bhq.bhq_destroy(c)


@pytest.fixture(scope="module")
def cube_case(ctx):
    x, m = synth.uniform_cube(1 << 16, synth.rng(1))
    T = orc.Tree(x, m, 0.5, 256)
    mat = orc.materialise(T, x, m)
    ref = orc.eval_lists(orc.QUAD, mat, x, 1e-6)
    return x, m, mat, ref


def test_launch_shapes(ctx, cube_case):
    x, m, mat, (a_ref, p_ref) = cube_case
    upload(ctx, mat, x, eps2=1e-6)
    for prec in PRECS:
        for block in (256, 128):
            for ipt in (1, 2):
                bhq.bhq_set_tuning(ctx, block, ipt)
                log("case shapes block=%d i_per_thread=%d precision=%s"
                    % (block, ipt, bhq.PRECISION_NAMES[prec]))
                a0, p0 = run(ctx, mat, len(m), bhq.QUAD, prec)
                assert_parity(errors(a0, p0, a_ref, p_ref), prec,
                              "block %d ipt %d" % (block, ipt))
                for bpc in (0, 1, 3):
                    log("  persistent blocks_per_cu=%d" % bpc)
                    bhq.bhq_set_tuning(ctx, block, ipt, bpc, 1)
                    a1, p1 = run(ctx, mat, len(m), bhq.QUAD, prec)
                    assert np.array_equal(a0, a1) and np.array_equal(p0, p1)
                if block == 256:
                    # capped register allocation: the same arithmetic
                    for w in (6, 8):
                        log("  waves_per_eu=%d" % w)
                        bhq.bhq_set_tuning(ctx, block, ipt, 0, 0, 0, 1, w)
                        aw, pw = run(ctx, mat, len(m), bhq.QUAD, prec)
                        assert np.array_equal(a0, aw) and np.array_equal(p0, pw)
                        bhq.bhq_set_tuning(ctx, block, ipt, 0, 1, 0, 1, w)
                        aw, pw = run(ctx, mat, len(m), bhq.QUAD, prec)
                        assert np.array_equal(a0, aw) and np.array_equal(p0, pw)
                for js in (2, 4, 8):
                    # cross-block j-split: parts of the lists in different
                    # blocks, added in part order; the persistent queue
                    # hands out the same parts
                    log("  jsplit=%d" % js)
                    bhq.bhq_set_tuning(ctx, block, ipt, 0, 0, 0, js)
                    a2, p2 = run(ctx, mat, len(m), bhq.QUAD, prec)
                    assert_parity(errors(a2, p2, a_ref, p_ref), prec,
                                  "block %d ipt %d jsplit %d" % (block, ipt, js))
                    bhq.bhq_set_tuning(ctx, block, ipt, 2, 1, 0, js)
                    a3, p3 = run(ctx, mat, len(m), bhq.QUAD, prec)
                    assert np.array_equal(a2, a3) and np.array_equal(p2, p3)
        t = bhq.bhq_get_tuning(ctx)
        assert t["persistent"] == 1 and t["i_per_thread"] == 2 and t["jsplit"] == 8
        assert t["waves_per_eu"] == 0
    bhq.bhq_set_tuning(ctx)


ORDERS = [(bhq.ORDER_COST, 256, 1024), (bhq.ORDER_XCD, 256, 1024),
          (bhq.ORDER_XCD, 1, 0), (bhq.ORDER_XCD, 64, 3000),
          (bhq.ORDER_XCD, 1 << 24, 0)]


def test_group_orders_bitwise(ctx, cube_case):
    """Every dispatch order, eager and persistent, gives the same bits (the
    per-group arithmetic does not depend on which block runs a group), and
    matches the oracle."""
    x, m, mat, (a_ref, p_ref) = cube_case
    upload(ctx, mat, x, eps2=1e-6)
    for prec in PRECS:
        first = None
        for mode, window, tail in ORDERS:
            bhq.bhq_set_group_order(ctx, mode, window, tail)
            assert bhq.bhq_get_group_order(ctx) == dict(mode=mode, window=window,
                                                        tail=tail)
            for pers in (0, 1):
                bhq.bhq_set_tuning(ctx, 256, 2, 0, pers, 0)
                log("case order mode=%d window=%d tail=%d persistent=%d %s"
                    % (mode, window, tail, pers, bhq.PRECISION_NAMES[prec]))
                a, p = run(ctx, mat, len(m), bhq.QUAD, prec)
                if first is None:
                    first = (a, p)
                    assert_parity(errors(a, p, a_ref, p_ref), prec, "orders")
                else:
                    assert np.array_equal(a, first[0]) and np.array_equal(p, first[1])
    bhq.bhq_set_group_order(ctx)
    bhq.bhq_set_tuning(ctx)


def test_tuning_argument_errors(ctx):
    for args in ((64, 1, 0, 0, 0), (256, 3, 0, 0, 0), (256, 1, -1, 0, 0),
                 (256, 1, 0, 2, 0), (256, 1, 0, 0, 3), (256, 1, 0, 0, 0, 3),
                 (256, 1, 0, 0, 0, 16), (256, 1, 0, 0, 0, -1), (256, 1, 0, 0, 0, 1, 4),
                 (256, 1, 0, 0, 0, 1, 7), (128, 1, 0, 0, 0, 1, 6)):
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_set_tuning(ctx, *args)
        assert ei.value.code == bhq.E_ARG
    for args in ((2, 256, 0), (1, 0, 0), (1, 256, -1)):
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_set_group_order(ctx, *args)
        assert ei.value.code == bhq.E_ARG
    assert bhq.bhq_get_group_order(ctx) == dict(mode=bhq.ORDER_XCD,
                                                window=bhq.ORDER_WINDOW,
                                                tail=bhq.ORDER_TAIL)


def test_graph_replays_match_eager(ctx, cube_case):
    """Graph mode: several replays, with other GPU work and synchronizations
    between them, each equal to the eager launch; a data change re-records."""
    torch = pytest.importorskip("torch")
    x, m, mat, (a_ref, p_ref) = cube_case
    upload(ctx, mat, x, eps2=1e-6)
    for persistent in (0, 1):
        bhq.bhq_set_tuning(ctx, 256, 1, 0, persistent, 0)
        a_e, p_e = run(ctx, mat, len(m), bhq.QUAD, bhq.FP32_OFS64)
        bhq.bhq_set_tuning(ctx, 256, 1, 0, persistent, 1)
        for rep in range(4):
            log("case graph persistent=%d replay %d" % (persistent, rep))
            a, p = run(ctx, mat, len(m), bhq.QUAD, bhq.FP32_OFS64)
            assert np.array_equal(a, a_e) and np.array_equal(p, p_e)
            y = torch.ones(1 << 20, device="cuda") * (rep + 1)
            torch.cuda.synchronize()
            assert float(y.sum()) == float((rep + 1) << 20)
    # a new order re-records the graph; results unchanged
    bhq.bhq_set_tuning(ctx, 256, 1, 0, 1, 1)
    a0, p0 = run(ctx, mat, len(m), bhq.QUAD, bhq.FP32_OFS64)
    for mode in (bhq.ORDER_COST, bhq.ORDER_XCD):
        bhq.bhq_set_group_order(ctx, mode)
        for rep in range(2):
            log("case graph order=%d replay %d" % (mode, rep))
            a, p = run(ctx, mat, len(m), bhq.QUAD, bhq.FP32_OFS64)
            assert np.array_equal(a, a0) and np.array_equal(p, p0)
    # new data -> the graph is recorded again
    x2, m2 = synth.plummer(5000, synth.rng(12))
    T2 = orc.Tree(x2, m2, 0.5, 64)
    mat2 = orc.materialise(T2, x2, m2)
    upload(ctx, mat2, x2, eps2=1e-4)
    a_ref2, p_ref2 = orc.eval_lists(orc.QUAD, mat2, x2, 1e-4)
    for rep in range(2):
        a, p = run(ctx, mat2, len(m2), bhq.QUAD, bhq.FP32_OFS64)
        assert_parity(errors(a, p, a_ref2, p_ref2), bhq.FP32_OFS64, "graph new data")
    bhq.bhq_set_tuning(ctx)


def test_jsplit_across_launches(ctx, cube_case):
    """Cross-block j-split over repeated launches: eager launches, graph
    replays (the force kernel and the parts' reduction recorded together)
    and the persistent queue give the first launch's bits, also after an
    input with more groups and particles has grown the parts buffer, and
    back."""
    torch = pytest.importorskip("torch")
    x, m, mat, (a_ref, p_ref) = cube_case
    x2, m2 = synth.uniform_cube(1 << 15, synth.rng(13))
    T2 = orc.Tree(x2, m2, 0.5, 16)
    mat2 = orc.materialise(T2, x2, m2)
    assert len(mat2["i_off"]) > len(mat["i_off"])
    ref2 = orc.eval_lists(orc.QUAD, mat2, x2, 1e-6)
    try:
        for prec in PRECS:
            for js in (2, 8):
                upload(ctx, mat, x, eps2=1e-6)
                bhq.bhq_set_tuning(ctx, 256, 2, 0, 0, 0, js)
                a0, p0 = run(ctx, mat, len(m), bhq.QUAD, prec)
                assert_parity(errors(a0, p0, a_ref, p_ref), prec, "jsplit %d" % js)
                for pers, graph in ((0, 0), (0, 1), (1, 0), (1, 1)):
                    bhq.bhq_set_tuning(ctx, 256, 2, 2 if pers else 0, pers, graph, js)
                    for rep in range(3):
                        log("case jsplit launches precision=%s jsplit=%d persistent=%d graph=%d "
                            "launch %d" % (bhq.PRECISION_NAMES[prec], js, pers, graph, rep))
                        a, p = run(ctx, mat, len(m), bhq.QUAD, prec)
                        assert np.array_equal(a, a0) and np.array_equal(p, p0)
                        y = torch.ones(1 << 16, device="cuda")
                        torch.cuda.synchronize()
                        assert float(y.sum()) == float(1 << 16)
                # more groups, then the first input again
                log("case jsplit launches: %d groups, then %d"
                    % (len(mat2["i_off"]) - 1, len(mat["i_off"]) - 1))
                upload(ctx, mat2, x2, eps2=1e-6)
                a2, p2 = run(ctx, mat2, len(m2), bhq.QUAD, prec)
                assert_parity(errors(a2, p2, *ref2), prec, "jsplit %d, more groups" % js)
                upload(ctx, mat, x, eps2=1e-6)
                a, p = run(ctx, mat, len(m), bhq.QUAD, prec)
                assert np.array_equal(a, a0) and np.array_equal(p, p0)
    finally:
        bhq.bhq_set_tuning(ctx)


@pytest.mark.parametrize("persistent", [0, 1])
def test_batched_systems_one_launch(ctx, persistent):
    """Independent Plummer systems (sizes log-uniform in [2^10, 2^13] here),
    each with eps = 1/(4 N^(1/3)) and theta = 0.6, built together by
    bhq_build_lists_batch and evaluated in one launch."""
    systems = synth.batched_plummer(24, lo=10.0, hi=13.0)
    sizes = np.array([len(s[1]) for s in systems])
    off = np.concatenate([[0], np.cumsum(sizes)])
    X = np.concatenate([s[0] for s in systems])
    M = np.concatenate([s[1] for s in systems])
    E2 = np.concatenate([np.full(len(s[1]), s[2] ** 2) for s in systems])
    log("case batched %d systems, %d particles, persistent=%d"
        % (len(systems), len(M), persistent))
    a_ref = np.zeros((len(M), 3))
    p_ref = np.zeros(len(M))
    for s, (x, m, eps) in enumerate(systems):
        T = orc.Tree(x, m, 0.6, 64)
        mat = orc.materialise(T, x, m)
        a, p = orc.eval_lists(orc.QUAD, mat, x, eps * eps)
        a_ref[off[s]:off[s + 1]] = a
        p_ref[off[s]:off[s + 1]] = p
    L = bhq.bhq_build_lists_batch(off, X, M, 0.6, 64)
    try:
        bhq.bhq_set_lists(ctx, L, X, M)
        idx = bhq.bhq_lists_export(L, len(M))["i_idx"]
    finally:
        bhq.bhq_lists_free(L)
    bhq.bhq_set_eps2_i(ctx, E2[idx])
    bhq.bhq_set_tuning(ctx, 256, 2, 0, persistent, 1)
    for prec in PRECS:
        bhq.bhq_set_kernel(ctx, bhq.QUAD, prec)
        bhq.bhq_compute(ctx)
        a_g, p_g = bhq.bhq_get_result(ctx, len(M))
        a = np.zeros_like(a_g)
        p = np.zeros_like(p_g)
        a[idx] = a_g
        p[idx] = p_g
        err = errors(a, p, a_ref, p_ref)
        log("  precision=%s %s" % (bhq.PRECISION_NAMES[prec], err))
        assert_parity(err, prec, "batched")
    bhq.bhq_set_tuning(ctx)
