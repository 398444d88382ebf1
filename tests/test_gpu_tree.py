"""GPU: tree, groups and interaction lists built on the device
(bhq_build_lists_device) against the host builder (bhq_build_lists), whose
lists the CPU tests tie to the oracle's tree walk.  Index work is compared
bit for bit: particle order, group offsets, every list entry in order, and
the cell moments (the device computes them with the host's operations in
the host's order).  Forces from device-built lists then equal, bit for bit,
forces from the host-built lists, and match the FP64 oracle."""
import ctypes

import numpy as np
import pytest

import oracle as orc
from _parity import assert_parity, errors, log
from paper_1812_07313_amd import bhq, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(x, m):
    xt = torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()
    mt = torch.from_numpy(np.ascontiguousarray(m, np.float64)).cuda()
    return xt, mt


def _host(x, m, theta, ncrit, nleaf=8, box=0.0, rcut=0.0):
    L = bhq.bhq_build_lists(x, m, theta, ncrit, nleaf=nleaf, box=box, rcut=rcut)
    try:
        out = bhq.bhq_lists_export(L, len(m))
        out["cells"] = bhq.bhq_lists_cells(L)
        out["sizes"] = bhq.bhq_lists_sizes(L)
    finally:
        bhq.bhq_lists_free(L)
    return out


def _device(ctx, x, m, theta, ncrit, nleaf=8, box=0.0, rcut=0.0):
    xt, mt = _dev(x, m)
    bhq.bhq_build_lists_device(ctx, xt, mt, theta, ncrit, nleaf, box, rcut)
    torch.cuda.synchronize()
    out = bhq.bhq_get_lists(ctx, len(m))
    out["cells"] = bhq.bhq_get_cells(ctx)
    out["sizes"] = bhq.bhq_get_lists_sizes(ctx)
    return out


def _same(h, d, name):
    assert h["sizes"] == d["sizes"], (name, h["sizes"], d["sizes"])
    for k in ("i_idx", "i_off", "jp_off", "jp_idx", "jc_off"):
        assert np.array_equal(h[k], d[k]), (name, k)
    assert np.array_equal(h["jc_cell"], d["jc_cell"]), (name, "jc_cell")
    for k in ("com", "mass", "q", "trace"):
        a, b = h["cells"][k], d["cells"][k]
        assert np.array_equal(a.view(np.int64), b.view(np.int64)), (name, k)


CASES = [
    ("cube 65536", lambda: synth.uniform_cube(1 << 16, synth.rng(1)), 0.5, 256, 8, 0.0, 0.0),
    ("plummer 16384", lambda: synth.plummer(16384, synth.rng(0)), 0.5, 64, 8, 0.0, 0.0),
    ("clustered 32768", lambda: synth.clustered(1 << 15, synth.rng(2)), 0.6, 128, 8, 0.0, 0.0),
    ("cube theta 0", lambda: synth.uniform_cube(3000, synth.rng(5)), 0.0, 64, 8, 0.0, 0.0),
    ("cube ncrit=nleaf=1", lambda: synth.uniform_cube(2000, synth.rng(6)), 0.7, 1, 1, 0.0, 0.0),
    ("lattice 32^3 periodic", lambda: synth.perturbed_lattice(32, synth.rng(4)), 0.5, 64, 8,
     1.0, 4.5 * 1.25 / 32),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_device_lists_equal_host(case):
    name, gen, theta, ncrit, nleaf, box, rcut = case
    x, m = gen()
    log("case device lists %s (n=%d)" % (name, len(m)))
    h = _host(x, m, theta, ncrit, nleaf, box, rcut)
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        d = _device(ctx, x, m, theta, ncrit, nleaf, box, rcut)
    finally:
        bhq.bhq_destroy(ctx)
    log("  sizes %s" % (d["sizes"],))
    _same(h, d, name)


def test_degenerate_inputs():
    """One particle; two; coincident particles (a chain of cells down to
    depth 21 holding more than nleaf); a flat (2-d) distribution."""
    g = np.random.default_rng(9)
    cases = [
        ("one", np.array([[0.3, 0.2, 0.1]]), np.array([1.0])),
        ("two", np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 3.0]]), np.array([1.0, 2.0])),
        ("coincident", np.vstack([np.full((20, 3), 0.25), g.random((50, 3))]),
         np.full(70, 1.0 / 70)),
        ("flat", np.column_stack([g.random(500), g.random(500), np.zeros(500)]),
         np.full(500, 0.002)),
    ]
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        for name, x, m in cases:
            log("case device lists degenerate %s" % name)
            for ncrit, nleaf in ((8, 8), (16, 2)):
                h = _host(x, m, 0.5, ncrit, nleaf)
                d = _device(ctx, x, m, 0.5, ncrit, nleaf)
                _same(h, d, name)
    finally:
        bhq.bhq_destroy(ctx)


@pytest.mark.parametrize("prec", [bhq.FP32_OFS64, bhq.FP64])
def test_forces_from_device_lists(prec):
    """Device-built lists: the same force bits as host-built index lists,
    and parity with the FP64 oracle's own tree and lists."""
    x, m = synth.plummer(16384, synth.rng(0))
    eps = 1.0 / 64.0
    ctx_d = bhq.bhq_create(0, bhq.QUAD, prec)
    ctx_h = bhq.bhq_create(0, bhq.QUAD, prec)
    try:
        xt, mt = _dev(x, m)
        bhq.bhq_build_lists_device(ctx_d, xt, mt, 0.5, 64)
        bhq.bhq_set_eps(ctx_d, eps)
        L = bhq.bhq_build_lists(x, m, 0.5, 64)
        bhq.bhq_set_lists_indexed(ctx_h, L, x, m)
        bhq.bhq_lists_free(L)
        bhq.bhq_set_eps(ctx_h, eps)
        res = []
        for ctx in (ctx_d, ctx_h):
            bhq.bhq_compute(ctx)
            res.append(bhq.bhq_get_result(ctx, len(m)))
        assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
        idx = bhq.bhq_get_lists(ctx_d, len(m))["i_idx"]
        a = np.zeros_like(res[0][0])
        p = np.zeros_like(res[0][1])
        a[idx] = res[0][0]
        p[idx] = res[0][1]
        T = orc.Tree(x, m, 0.5, 64)
        a_ref, p_ref = orc.eval_lists(orc.QUAD, orc.materialise(T, x, m), x, eps * eps)
        err = errors(a, p, a_ref, p_ref)
        log("case device-list forces %s: %s" % (bhq.PRECISION_NAMES[prec], err))
        assert_parity(err, prec, "device lists")
        # a rebuild leaves each group's entries in a slot of its own; the
        # j-split parts and the persistent queue read them there, and give
        # the host-built lists' bits at the same launch shape
        bhq.bhq_build_lists_device(ctx_d, xt, mt, 0.5, 64)
        bhq.bhq_set_eps(ctx_d, eps)
        for shape in ((256, 2, 0, 0, 0, 1), (256, 1, 0, 0, 0, 2, 6), (256, 2, 2, 1, 0, 4)):
            log("case device-list rebuild %s shape %s" % (bhq.PRECISION_NAMES[prec], shape))
            out = []
            for ctx in (ctx_d, ctx_h):
                bhq.bhq_set_tuning(ctx, *shape)
                bhq.bhq_compute(ctx)
                out.append(bhq.bhq_get_result(ctx, len(m)))
                bhq.bhq_set_tuning(ctx)
            assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    finally:
        bhq.bhq_destroy(ctx_d)
        bhq.bhq_destroy(ctx_h)


def test_split_forces_from_device_lists():
    """Periodic split kernel on device-built lists equals host-built."""
    x, m = synth.perturbed_lattice(24, synth.rng(4))
    rs = 1.25 / 24
    rcut = 4.5 * rs
    ctx_d = bhq.bhq_create(0, bhq.SPLIT_QUAD, bhq.FP32_OFS64)
    ctx_h = bhq.bhq_create(0, bhq.SPLIT_QUAD, bhq.FP32_OFS64)
    try:
        xt, mt = _dev(x, m)
        bhq.bhq_build_lists_device(ctx_d, xt, mt, 0.5, 64, 8, 1.0, rcut)
        L = bhq.bhq_build_lists(x, m, 0.5, 64, box=1.0, rcut=rcut)
        bhq.bhq_set_lists_indexed(ctx_h, L, x, m)
        bhq.bhq_lists_free(L)
        res = []
        for ctx in (ctx_d, ctx_h):
            bhq.bhq_set_split(ctx, rs, rcut, 1.0)
            bhq.bhq_compute(ctx)
            res.append(bhq.bhq_get_result(ctx, len(m)))
        assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
        # after a rebuild (entries in per-group slots), in both precisions and
        # the launch shapes the bench times for the lattice, plus the j-split
        bhq.bhq_build_lists_device(ctx_d, xt, mt, 0.5, 64, 8, 1.0, rcut)
        bhq.bhq_set_split(ctx_d, rs, rcut, 1.0)
        for prec in (bhq.FP32_OFS64, bhq.FP64):
            for shape in ((256, 2, 0, 0, 0, 1, 6), (256, 2, 0, 1, 0, 1, 6), (256, 2, 0, 0, 0, 4)):
                log("case split device-list rebuild %s shape %s"
                    % (bhq.PRECISION_NAMES[prec], shape))
                out = []
                for ctx in (ctx_d, ctx_h):
                    bhq.bhq_set_kernel(ctx, bhq.SPLIT_QUAD, prec)
                    bhq.bhq_set_tuning(ctx, *shape)
                    bhq.bhq_compute(ctx)
                    out.append(bhq.bhq_get_result(ctx, len(m)))
                    bhq.bhq_set_tuning(ctx)
                assert np.array_equal(out[0][0], out[1][0])
                assert np.array_equal(out[0][1], out[1][1])
    finally:
        bhq.bhq_destroy(ctx_d)
        bhq.bhq_destroy(ctx_h)


def test_device_build_errors():
    x, m = synth.uniform_cube(1000, synth.rng(3))
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        xt, mt = _dev(x, m)
        lib = bhq.lib()
        # host memory instead of device memory
        rc = lib.bhq_build_lists_device(ctx, len(m), x.ctypes.data, m.ctypes.data, 0.5, 64,
                                        8, 0.0, 0.0, None)
        assert rc == bhq.E_ARG, rc
        # a count far beyond the allocation
        rc = lib.bhq_build_lists_device(ctx, 1 << 30, xt.data_ptr(), mt.data_ptr(), 0.5, 64,
                                        8, 0.0, 0.0, None)
        assert rc == bhq.E_RANGE, rc
        for args in ((-0.1, 64, 8, 0.0, 0.0), (0.5, 0, 8, 0.0, 0.0), (0.5, 8, 16, 0.0, 0.0),
                     (0.5, 64, 8, -1.0, 0.0), (0.5, 64, 8, 0.0, -1.0)):
            with pytest.raises(bhq.BhqError) as ei:
                bhq.bhq_build_lists_device(ctx, xt, mt, *args)
            assert ei.value.code == bhq.E_ARG
        # a non-finite position: error, and no lists left in the context
        bhq.bhq_build_lists_device(ctx, xt, mt, 0.5, 64)
        bhq.bhq_set_eps(ctx, 0.01)
        bhq.bhq_compute(ctx)
        xt[17, 1] = float("nan")
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_build_lists_device(ctx, xt, mt, 0.5, 64)
        assert ei.value.code == bhq.E_NONFINITE
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_compute(ctx)
        assert ei.value.code == bhq.E_STATE
        with pytest.raises(TypeError):
            bhq.bhq_build_lists_device(ctx, torch.from_numpy(x), torch.from_numpy(m), 0.5, 64)
    finally:
        bhq.bhq_destroy(ctx)


def test_rebuild_reuses_context():
    """Builds of different sizes in a row on one context, each equal to the
    host builder's lists: a smaller one (its levels built without host
    synchronisation from the first build's depth), a larger one (whose
    cells overflow that capacity, so its levels are built again one at a
    time), and the same again; the last evaluates correctly."""
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        for n, seed in ((40000, 11), (7000, 12), (60000, 13), (60000, 13)):
            x, m = synth.plummer(n, synth.rng(seed))
            log("case device rebuild n=%d" % n)
            h = _host(x, m, 0.6, 64)
            d = _device(ctx, x, m, 0.6, 64)
            _same(h, d, "rebuild %d" % n)
        bhq.bhq_set_eps(ctx, 0.01)
        bhq.bhq_compute(ctx)
        a, p = bhq.bhq_get_result(ctx, len(m))
        idx = bhq.bhq_get_lists(ctx, len(m))["i_idx"]
        aa = np.zeros_like(a)
        pp = np.zeros_like(p)
        aa[idx] = a
        pp[idx] = p
        T = orc.Tree(x, m, 0.6, 64)
        a_ref, p_ref = orc.eval_lists(orc.QUAD, orc.materialise(T, x, m), x, 1e-4)
        assert_parity(errors(aa, pp, a_ref, p_ref), bhq.FP32_OFS64, "rebuild")
    finally:
        bhq.bhq_destroy(ctx)


def test_rebuild_one_walk_and_overflow():
    """Rebuilds on one context: the second build of the same particles walks
    once (slots sized from the first); a build with longer lists (smaller
    theta) overflows its slots and counts first; the next one walks once
    again.  Every build equals the host builder's lists."""
    x, m = synth.plummer(30000, synth.rng(21))
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        expect = []
        for theta, one_walk in ((0.7, False), (0.7, True), (0.4, False), (0.4, True)):
            log("case device rebuild theta=%g" % theta)
            h = _host(x, m, theta, 64)
            d = _device(ctx, x, m, theta, 64)
            _same(h, d, "rebuild theta %g" % theta)
            info = bhq.bhq_get_build_info(ctx)
            ni = np.diff(h["jp_off"]).max(), np.diff(h["jc_off"]).max()
            assert info == (one_walk, int(ni[0]), int(ni[1])), (theta, info)
            expect.append(info)
    finally:
        bhq.bhq_destroy(ctx)


def test_partial_list_update_after_rebuild():
    """bhq_set_jp_idx and bhq_set_jc_idx after a rebuild (whose lists stay in
    per-group slots) write at compact list addresses, as after a first
    build: the lists and the forces equal, bit for bit, those of a context
    built once with the same entries overwritten."""
    x, m = synth.plummer(20000, synth.rng(31))
    xt, mt = _dev(x, m)
    got = []
    for builds in (1, 2):
        log("case partial list update after %d device builds" % builds)
        ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
        try:
            for _ in range(builds):
                bhq.bhq_build_lists_device(ctx, xt, mt, 0.6, 64, 8, 0.0, 0.0)
            assert bhq.bhq_get_build_info(ctx)[0] == (builds == 2)
            ng, njp, njc, _ = bhq.bhq_get_lists_sizes(ctx)
            # pool indices 0..k-1 into the middle of the lists, across groups
            bhq.bhq_set_jp_idx(ctx, njp // 3, np.arange(200, dtype=np.int32))
            bhq.bhq_set_jc_idx(ctx, njc // 2, np.arange(150, dtype=np.int32)[::-1].copy())
            bhq.bhq_set_eps(ctx, 0.01)
            bhq.bhq_compute(ctx)
            a, p = bhq.bhq_get_result(ctx, len(m))
            got.append((bhq.bhq_get_lists(ctx, len(m)), a, p))
        finally:
            bhq.bhq_destroy(ctx)
    (l1, a1, p1), (l2, a2, p2) = got
    for k in ("i_idx", "i_off", "jp_off", "jp_idx", "jc_off", "jc_cell"):
        assert np.array_equal(l1[k], l2[k]), k
    assert np.array_equal(l2["jc_cell"][njc // 2:njc // 2 + 150], np.arange(150)[::-1])
    assert np.array_equal(a1.view(np.int64), a2.view(np.int64))
    assert np.array_equal(p1.view(np.int64), p2.view(np.int64))


def test_host_views_after_rebuild():
    """After a one-walk rebuild the group offsets stay on the device until
    the host asks: bhq_get_counts gives the host builder's interaction
    counts, and the host order planner (cost order), which reads the
    offsets on the host, gives the forces of the device-planned XCD order
    bit for bit (a group's forces do not depend on the launch order)."""
    x, m = synth.plummer(25000, synth.rng(41))
    xt, mt = _dev(x, m)
    h = _host(x, m, 0.6, 64)
    ni = np.diff(h["i_off"])
    n_pp = int((ni * np.diff(h["jp_off"])).sum())
    n_pc = int((ni * np.diff(h["jc_off"])).sum())
    got = []
    for mode in (bhq.ORDER_XCD, bhq.ORDER_COST):
        log("case host views after rebuild, order mode %d" % mode)
        ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
        try:
            bhq.bhq_set_group_order(ctx, mode)
            for _ in range(2):
                bhq.bhq_build_lists_device(ctx, xt, mt, 0.6, 64, 8, 0.0, 0.0)
            assert bhq.bhq_get_build_info(ctx)[0]
            assert bhq.bhq_get_counts(ctx) == (n_pp, n_pc)
            bhq.bhq_set_eps(ctx, 0.01)
            bhq.bhq_compute(ctx)
            got.append(bhq.bhq_get_result(ctx, len(m)))
        finally:
            bhq.bhq_destroy(ctx)
    (a1, p1), (a2, p2) = got
    assert np.array_equal(a1.view(np.int64), a2.view(np.int64))
    assert np.array_equal(p1.view(np.int64), p2.view(np.int64))


def _batch(systems):
    sizes = np.array([len(s[1]) for s in systems])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    X = np.concatenate([s[0] for s in systems])
    M = np.concatenate([s[1] for s in systems])
    E2 = np.concatenate([np.full(len(s[1]), s[2] ** 2) for s in systems])
    return off, X, M, E2


def _host_batch(off, X, M, theta, ncrit, nleaf=8):
    L = bhq.bhq_build_lists_batch(off, X, M, theta, ncrit, nleaf=nleaf)
    try:
        out = bhq.bhq_lists_export(L, len(M))
        out["cells"] = bhq.bhq_lists_cells(L)
        out["sizes"] = bhq.bhq_lists_sizes(L)
    finally:
        bhq.bhq_lists_free(L)
    return out


def test_device_batch_equals_host():
    """Independent systems in one build, including one- and two-particle
    systems: the device batch build equals bhq_build_lists_batch entry for
    entry (cells numbered system by system)."""
    systems = synth.batched_plummer(20, lo=8.0, hi=12.0)
    systems.insert(3, (np.array([[0.1, 0.2, 0.3]]), np.array([1.0]), 0.1))
    systems.insert(7, (np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]]), np.array([0.5, 0.5]), 0.1))
    off, X, M, E2 = _batch(systems)
    log("case device batch: %d systems, %d particles" % (len(systems), len(M)))
    h = _host_batch(off, X, M, 0.6, 64)
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        xt, mt = _dev(X, M)
        bhq.bhq_build_lists_device_batch(ctx, off, xt, mt, 0.6, 64)
        torch.cuda.synchronize()
        d = bhq.bhq_get_lists(ctx, len(M))
        d["cells"] = bhq.bhq_get_cells(ctx)
        d["sizes"] = bhq.bhq_get_lists_sizes(ctx)
    finally:
        bhq.bhq_destroy(ctx)
    _same(h, d, "batch")


def test_device_batch_forces_with_softening():
    """Per-system softening given to the device build: forces equal those
    of host-built lists with bhq_set_eps2_i (bitwise) and match the oracle
    system by system."""
    systems = synth.batched_plummer(12, lo=9.0, hi=11.0)
    off, X, M, E2 = _batch(systems)
    ctx_d = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    ctx_h = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        xt, mt = _dev(X, M)
        e2t = torch.from_numpy(E2).cuda()
        bhq.bhq_build_lists_device_batch(ctx_d, off, xt, mt, 0.6, 64, eps2=e2t)
        L = bhq.bhq_build_lists_batch(off, X, M, 0.6, 64)
        bhq.bhq_set_lists_indexed(ctx_h, L, X, M)
        idx = bhq.bhq_lists_export(L, len(M))["i_idx"]
        bhq.bhq_lists_free(L)
        bhq.bhq_set_eps2_i(ctx_h, E2[idx])
        res = []
        for c in (ctx_d, ctx_h):
            bhq.bhq_compute(c)
            res.append(bhq.bhq_get_result(c, len(M)))
        assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
        a = np.zeros_like(res[0][0])
        p = np.zeros_like(res[0][1])
        a[idx] = res[0][0]
        p[idx] = res[0][1]
        for s, (x, m, eps) in enumerate(systems):
            T = orc.Tree(x, m, 0.6, 64)
            ar, pr = orc.eval_lists(orc.QUAD, orc.materialise(T, x, m), x, eps * eps)
            sl = slice(off[s], off[s + 1])
            assert_parity(errors(a[sl], p[sl], ar, pr), bhq.FP32_OFS64, "batch system %d" % s)
        # a softening below 2^-126 in eps^2 is refused, and the context then
        # holds no lists
        e2t[5] = 2.0 ** -127
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_build_lists_device_batch(ctx_d, off, xt, mt, 0.6, 64, eps2=e2t)
        assert ei.value.code == bhq.E_ARG
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_compute(ctx_d)
        assert ei.value.code == bhq.E_STATE
        for bad in ([0, 5, 5, len(M)], [1, len(M)]):
            with pytest.raises(bhq.BhqError) as ei:
                bhq.bhq_build_lists_device_batch(ctx_d, np.array(bad), xt, mt, 0.6, 64)
            assert ei.value.code in (bhq.E_RANGE, bhq.E_ARG)
    finally:
        bhq.bhq_destroy(ctx_d)
        bhq.bhq_destroy(ctx_h)


@pytest.mark.parametrize("window,tail", [(256, 1024), (100, 333), (1, 0), (1024, 7),
                                         (2000, 1024)])
def test_device_order_equals_host_plan(window, tail):
    """The slot table planned on the device for device-built lists equals
    bhq_plan_order on the same offsets, entry for entry (the last case,
    window 2000, is planned on the host)."""
    x, m = synth.clustered(1 << 16, synth.rng(9))
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        bhq.bhq_set_group_order(ctx, bhq.ORDER_XCD, window, tail)
        xt, mt = torch.from_numpy(x).cuda(), torch.from_numpy(m).cuda()
        bhq.bhq_build_lists_device(ctx, xt, mt, 0.5, 32, 8)
        dev = bhq.bhq_get_order(ctx)
        L = bhq.bhq_get_lists(ctx)
    finally:
        bhq.bhq_destroy(ctx)
    host = bhq.bhq_plan_order(L["i_off"], L["jp_off"], L["jc_off"], bhq.ORDER_XCD, window,
                              tail)
    log("case device order window %d tail %d: %d groups, %d slots"
        % (window, tail, len(L["i_off"]) - 1, len(dev)))
    assert np.array_equal(dev, host)


def test_order_and_build_info_queries():
    """bhq_get_order before any groups is a state error; bhq_get_build_info
    is all zero before the first device build; a host-built upload keeps
    the last device build's record."""
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_get_order(ctx)
        assert ei.value.code == bhq.E_STATE
        assert bhq.bhq_get_build_info(ctx) == (False, 0, 0)
        assert bhq.lib().bhq_get_build_info(ctx, None) == bhq.E_ARG
        x, m = synth.uniform_cube(5000, synth.rng(3))
        d = _device(ctx, x, m, 0.6, 64)
        info = bhq.bhq_get_build_info(ctx)
        assert info == (False, int(np.diff(d["jp_off"]).max()), int(np.diff(d["jc_off"]).max()))
        o = bhq.bhq_get_order(ctx)
        assert sorted(o[o >= 0].tolist()) == list(range(len(d["i_off"]) - 1))
        n = ctypes.c_int64()
        small = np.zeros(1, np.int32)
        rc = bhq.lib().bhq_get_order(ctx, small.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     1, ctypes.byref(n))
        assert rc == bhq.E_RANGE and n.value == len(o)
        L = bhq.bhq_build_lists(x, m, 0.6, 64)
        try:
            bhq.bhq_set_lists_indexed(ctx, L, x, m)
        finally:
            bhq.bhq_lists_free(L)
        assert bhq.bhq_get_build_info(ctx) == info
    finally:
        bhq.bhq_destroy(ctx)


def test_rebuild_deeper_tree():
    """A rebuild whose tree is much deeper than the previous one (the key
    sort of the rebuild covers only the previous depth's bits): the build
    sorts again on all bits and still equals the host builder's lists."""
    g = np.random.default_rng(31)
    x1 = g.random((2000, 3))
    m1 = np.full(2000, 1.0 / 2000)
    x2 = np.vstack([g.random((3000, 3)), np.full((40, 3), 0.3) + g.random((40, 3)) * 1e-9])
    m2 = np.full(len(x2), 1.0 / len(x2))
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        for x, m in ((x1, m1), (x1, m1), (x2, m2), (x2, m2), (x1, m1)):
            log("case device rebuild deeper n=%d" % len(m))
            _same(_host(x, m, 0.6, 32), _device(ctx, x, m, 0.6, 32), "deeper %d" % len(m))
    finally:
        bhq.bhq_destroy(ctx)
