"""GPU parity: libbhq's HIP kernels against the FP64 oracle on the same
interaction lists, element by element, through the C ABI.

Bars (per-particle relative error of the acceleration, and of the
potential): FP32 with FP64 group offsets <= 2e-6 rms and <= 1e-4 max;
FP64 <= 1e-12 rms and <= 1e-10 max (summation order and the last bits of
rsqrt and erfc).
"""
import numpy as np
import pytest

import oracle as orc
from _parity import assert_parity, errors, log, run, upload
from paper_1812_07313_amd import bhq, synth

pytestmark = pytest.mark.gpu

KINDS = [(bhq.QUAD, orc.QUAD), (bhq.MONO, orc.MONO),
         (bhq.QUAD_SOFT, orc.QUAD_SOFT)]
PRECS = [bhq.FP32_OFS64, bhq.FP64]


@pytest.fixture(scope="module")
def ctx():
    c = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    yield c
    bhq.bhq_destroy(c)


def _check_case(ctx, name, x, m, eps, theta, ncrit, kinds=KINDS, precs=PRECS,
                box=0.0):
    log("case %s: n=%d theta=%g ncrit=%d" % (name, len(m), theta, ncrit))
    T = orc.Tree(x, m, theta, ncrit)
    mat = orc.materialise(T, x, m)
    eps2 = np.broadcast_to(np.asarray(eps, np.float64) ** 2, (len(m),))
    upload(ctx, mat, x, eps2=eps2)
    out = {}
    for bk, ok in kinds:
        a_ref, p_ref = orc.eval_lists(ok, mat, x, eps2)
        for prec in precs:
            log("  kernel=%s precision=%s" % (bhq.KERNEL_NAMES[bk],
                                               bhq.PRECISION_NAMES[prec]))
            a, p = run(ctx, mat, len(m), bk, prec)
            err = errors(a, p, a_ref, p_ref)
            log("    %s" % err)
            assert_parity(err, prec, "%s %s %s" % (name, bk, prec))
            out[(bk, prec)] = (a, p)
    return T, mat, out


def test_plummer_16k(ctx):
    c = synth.config_plummer_16k()
    _check_case(ctx, "plummer16k", c["x"], c["m"], c["eps"], c["theta"],
                c["ncrit"])


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.7])
def test_uniform_cube_64k(ctx, theta):
    x, m = synth.uniform_cube(1 << 16, synth.rng(1))
    _check_case(ctx, "cube64k", x, m, 1e-3, theta, 256)


def test_clustered_32k(ctx):
    x, m = synth.clustered(1 << 15, synth.rng(2))
    _check_case(ctx, "clustered32k", x, m, 2e-4, 0.5, 64)


def test_large_groups_and_ragged_tiles(ctx):
    """ncrit above the block size: groups of up to 600 i-particles are
    processed in chunks of 256; list lengths are not tile multiples."""
    x, m = synth.plummer(5000, synth.rng(5))
    T, mat, _ = _check_case(ctx, "biggroups", x, m, 0.02, 0.6, 600)
    assert np.diff(T.i_off).max() > 256


def test_theta_zero_single_group_and_tiny(ctx):
    # theta = 0: no cells, all particles direct; one group when n <= ncrit
    x, m = synth.plummer(300, synth.rng(6))
    _check_case(ctx, "theta0", x, m, 0.05, 0.0, 64)
    _check_case(ctx, "onegroup", x, m, 0.05, 0.5, 512)
    # a single particle: only the self term, phi = -m / eps, a = 0
    x1 = np.array([[0.25, -0.5, 2.0]])
    m1 = np.array([1.0])
    _, _, out = _check_case(ctx, "single", x1, m1, 0.125, 0.5, 8)
    for (bk, prec), (a, p) in out.items():
        assert np.all(a == 0.0)
        assert p[0] == pytest.approx(-8.0, rel=1e-6 if prec == 0 else 1e-15)


@pytest.mark.parametrize("js", [2, 4, 8])
def test_jsplit_short_lists(ctx, js):
    """Cross-block j-split on lists shorter than the part count: most parts
    of a group hold no entry and add exact zeros in the part sum.  The
    persistent queue hands out the same parts (bitwise the same sums)."""
    x1 = np.array([[0.25, -0.5, 2.0]])
    m1 = np.array([1.0])
    x, m = synth.plummer(40, synth.rng(7))
    try:
        for pers in (0, 1):
            bhq.bhq_set_tuning(ctx, 256, 2, 2 if pers else 0, pers, 0, js)
            log("case jsplit=%d persistent=%d" % (js, pers))
            _, _, out = _check_case(ctx, "single js%d" % js, x1, m1, 0.125, 0.5, 8)
            for (bk, prec), (a, p) in out.items():
                assert np.all(a == 0.0)
                assert p[0] == pytest.approx(-8.0, rel=1e-6 if prec == 0 else 1e-15)
            T, _, out = _check_case(ctx, "short js%d" % js, x, m, 0.05, 0.7, 4)
            assert T.ngroups > 1
            if pers == 0:
                eager = out
            else:
                for key, (a, p) in out.items():
                    assert np.array_equal(a, eager[key][0])
                    assert np.array_equal(p, eager[key][1])
    finally:
        bhq.bhq_set_tuning(ctx)


def test_per_particle_softening(ctx):
    """Several independent Plummer systems, each with its own eps, in one
    launch (per-i eps^2; the batched configuration in miniature)."""
    systems = synth.batched_plummer(6, lo=9.0, hi=11.0)
    log("case batched: sizes %s" % [len(s[1]) for s in systems])
    mats, xs, e2s, refs = [], [], [], []
    base = 0
    i_off, jp_off, jc_off, cen = [0], [0], [0], []
    i_idx, jp_x, jp_m, jc_x, jc_m, jc_q, jc_t = [], [], [], [], [], [], []
    for (x, m, eps) in systems:
        T = orc.Tree(x, m, 0.6, 64)
        mat = orc.materialise(T, x, m)
        e2 = np.full(len(m), eps * eps)
        refs.append((orc.eval_lists(orc.QUAD, mat, x, e2),
                     orc.eval_lists(orc.QUAD_SOFT, mat, x, e2)))
        i_idx.append(mat["i_idx"] + base)
        i_off += list(mat["i_off"][1:] + i_off[-1])
        jp_off += list(mat["jp_off"][1:] + jp_off[-1])
        jc_off += list(mat["jc_off"][1:] + jc_off[-1])
        cen.append(mat["gcenter"])
        jp_x.append(mat["jp_x"]); jp_m.append(mat["jp_m"])
        jc_x.append(mat["jc_x"]); jc_m.append(mat["jc_m"])
        jc_q.append(mat["jc_q"]); jc_t.append(mat["jc_t"])
        xs.append(x)
        e2s.append(e2)
        base += len(m)
    big = dict(i_idx=np.concatenate(i_idx), i_off=np.array(i_off),
               gcenter=np.concatenate(cen), jp_off=np.array(jp_off),
               jc_off=np.array(jc_off), jp_x=np.concatenate(jp_x),
               jp_m=np.concatenate(jp_m), jc_x=np.concatenate(jc_x),
               jc_m=np.concatenate(jc_m), jc_q=np.concatenate(jc_q),
               jc_t=np.concatenate(jc_t))
    X = np.concatenate(xs)
    E2 = np.concatenate(e2s)
    upload(ctx, big, X, eps2=E2)
    for which, kern in ((0, bhq.QUAD), (1, bhq.QUAD_SOFT)):
        a_ref = np.concatenate([r[which][0] for r in refs])
        p_ref = np.concatenate([r[which][1] for r in refs])
        for prec in PRECS:
            a, p = run(ctx, big, len(X), kern, prec)
            err = errors(a, p, a_ref, p_ref)
            log("  kernel=%s precision=%s %s" % (bhq.KERNEL_NAMES[kern],
                                                 bhq.PRECISION_NAMES[prec], err))
            assert_parity(err, prec, "batched")


def test_deterministic_and_zero_quadrupole(ctx):
    """Bitwise identical results run to run; Q = 0 makes the quadrupole
    kernel's cell terms the monopole ones (to rounding)."""
    x, m = synth.uniform_cube(20000, synth.rng(8))
    T = orc.Tree(x, m, 0.5, 128)
    mat = orc.materialise(T, x, m)
    upload(ctx, mat, x, eps2=1e-6)
    for prec in PRECS:
        log("case determinism precision=%s" % bhq.PRECISION_NAMES[prec])
        a1, p1 = run(ctx, mat, len(m), bhq.QUAD, prec)
        a2, p2 = run(ctx, mat, len(m), bhq.QUAD, prec)
        assert np.array_equal(a1, a2) and np.array_equal(p1, p2)
    mat0 = dict(mat)
    mat0["jc_q"] = np.zeros_like(mat["jc_q"])
    upload(ctx, mat0, x, eps2=1e-6)
    aq, pq = run(ctx, mat0, len(m), bhq.QUAD, bhq.FP64)
    am, pm = run(ctx, mat0, len(m), bhq.MONO, bhq.FP64)
    np.testing.assert_allclose(aq, am, rtol=1e-12, atol=1e-12 * np.abs(am).max())
    np.testing.assert_allclose(pq, pm, rtol=1e-13)


def test_product_lists_path(ctx):
    """bhq_build_lists + bhq_set_lists (the benchmark's input path) gives the
    oracle's result on the oracle's lists."""
    x, m = synth.uniform_cube(1 << 15, synth.rng(9))
    T = orc.Tree(x, m, 0.5, 256)
    mat = orc.materialise(T, x, m)
    a_ref, p_ref = orc.eval_lists(orc.QUAD, mat, x, 1e-6)
    log("case product lists n=%d" % len(m))
    L = bhq.bhq_build_lists(x, m, 0.5, 256)
    try:
        bhq.bhq_set_lists(ctx, L, x, m)
        idx = bhq.bhq_lists_export(L, len(m))["i_idx"]
    finally:
        bhq.bhq_lists_free(L)
    bhq.bhq_set_eps(ctx, 1e-3)
    for prec in PRECS:
        bhq.bhq_set_kernel(ctx, bhq.QUAD, prec)
        bhq.bhq_compute(ctx)
        a_g, p_g = bhq.bhq_get_result(ctx, len(m))
        a = np.zeros_like(a_g)
        p = np.zeros_like(p_g)
        a[idx] = a_g
        p[idx] = p_g
        err = errors(a, p, a_ref, p_ref)
        log("  precision=%s %s" % (bhq.PRECISION_NAMES[prec], err))
        assert_parity(err, prec, "product lists")


def test_stream_and_timing(ctx):
    torch = pytest.importorskip("torch")
    x, m = synth.plummer(4096, synth.rng(10))
    T = orc.Tree(x, m, 0.5, 64)
    mat = orc.materialise(T, x, m)
    upload(ctx, mat, x, eps2=1e-4)
    s = torch.cuda.Stream()
    a0, p0 = run(ctx, mat, len(m), bhq.QUAD, bhq.FP32_OFS64)
    a1, p1 = run(ctx, mat, len(m), bhq.QUAD, bhq.FP32_OFS64, stream=s)
    assert np.array_equal(a0, a1) and np.array_equal(p0, p1)
    assert bhq.bhq_get_kernel_ms(ctx) > 0.0
    n_pp, n_pc = bhq.bhq_get_counts(ctx)
    assert (n_pp, n_pc) == T.interaction_counts()


def test_upload_waits_for_compute_on_stream(ctx):
    """Host uploads after a compute on a non-blocking stream wait for it:
    the result is that of the data the compute was launched with."""
    torch = pytest.importorskip("torch")
    x, m = synth.plummer(65536, synth.rng(12))
    T = orc.Tree(x, m, 0.3, 64)
    mat = orc.materialise(T, x, m)
    upload(ctx, mat, x, eps2=1e-4)
    a0, p0 = run(ctx, mat, len(m), bhq.QUAD, bhq.FP32_OFS64)
    s = torch.cuda.Stream()
    for _ in range(3):
        bhq.bhq_compute(ctx, s)
        # new positions and a new particle list while the kernel may run
        bhq.bhq_set_i(ctx, x[mat["i_idx"]] + 0.25)
        bhq.bhq_set_jp(ctx, 0, mat["jp_x"] + 0.5, mat["jp_m"])
        a_g, p_g = bhq.bhq_get_result(ctx, len(m))
        a1 = np.zeros_like(a0)
        p1 = np.zeros_like(p0)
        a1[mat["i_idx"]] = a_g
        p1[mat["i_idx"]] = p_g
        assert np.array_equal(a0, a1) and np.array_equal(p0, p1)
        upload(ctx, mat, x, eps2=1e-4)


def test_state_errors(ctx):
    c2 = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_compute(c2)
        assert ei.value.code == bhq.E_STATE
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_set_i(c2, np.zeros((3, 3)))
        assert ei.value.code == bhq.E_STATE
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_set_groups(c2, [0, 2, 1], np.zeros((2, 3)), [0, 0, 0],
                               [0, 0, 0])
        assert ei.value.code == bhq.E_RANGE
        bhq.bhq_set_groups(c2, [0, 2], np.zeros((1, 3)), [0, 2], [0, 0])
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_set_i(c2, np.zeros((3, 3)))
        assert ei.value.code == bhq.E_RANGE
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_set_i(c2, np.array([[0.0, np.nan, 0.0], [0, 0, 0]]))
        assert ei.value.code == bhq.E_NONFINITE
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_set_jp(c2, 1, np.zeros((2, 3)), np.ones(2))
        assert ei.value.code == bhq.E_RANGE
        bhq.bhq_set_i(c2, np.array([[0.0, 0, 0], [1.0, 0, 0]]))
        bhq.bhq_set_jp(c2, 0, np.array([[0.0, 0, 0], [1.0, 0, 0]]), np.ones(2))
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_compute(c2)  # no softening yet
        assert ei.value.code == bhq.E_STATE
        for bad in (0.0, -1.0, 1e-20):
            with pytest.raises(bhq.BhqError) as ei:
                bhq.bhq_set_eps(c2, bad)   # the self pair needs eps^2 >= 2^-126
            assert ei.value.code == bhq.E_ARG
        for bad in (0.0, 2.0 ** -127):
            with pytest.raises(bhq.BhqError) as ei:
                bhq.bhq_set_eps2_i(c2, [1.0, bad])
            assert ei.value.code == bhq.E_ARG
        bhq.bhq_set_eps2_i(c2, [1.0, 2.0 ** -126])  # the smallest accepted value
        bhq.bhq_set_eps(c2, 1.0)
        bhq.bhq_compute(c2)
        a, p = bhq.bhq_get_result(c2, 2)
        # two unit masses one apart with eps = 1: |a| = 1 / 2^1.5
        assert a[0, 0] == pytest.approx(2 ** -1.5, rel=1e-6)
        assert p[0] == pytest.approx(-1.0 - 2 ** -0.5, rel=1e-6)
    finally:
        bhq.bhq_destroy(c2)


@pytest.mark.parametrize("nside", [24, 32])
def test_split_kernel_periodic(ctx, nside):
    """Short-range Gaussian-split kernel in the periodic unit box (perturbed
    lattice, r_s = 1.25 mesh cells, cutoff 4.5 r_s, theta = 0.5): minimum
    image offsets, cutoff masking, the trace term of the cells."""
    x, m = synth.perturbed_lattice(nside, synth.rng(4))
    rs = 1.25 / nside
    rcut = 4.5 * rs
    log("case split lattice %d^3 rs=%g rcut=%g" % (nside, rs, rcut))
    T = orc.Tree(x, m, 0.5, 64, box=1.0, rcut=rcut)
    mat = orc.materialise(T, x, m)
    # the cutoff decisions from FP64 offsets to the group centres are the
    # definition's (absolute FP64 separations) on every term of these lists
    assert orc.mask_flips(mat, x, 1.0, rcut) == 0
    upload(ctx, mat, x, split=(rs, rcut, 1.0))
    for bk, ok in ((bhq.SPLIT_QUAD, orc.SPLIT_QUAD),
                   (bhq.SPLIT_MONO, orc.SPLIT_MONO)):
        for prec in PRECS:
            a_ref, p_ref = orc.eval_lists(ok, mat, x, 0.0, box=1.0, rs=rs,
                                          rcut=rcut, mask=orc.MASK_F64_OFS)
            log("  kernel=%s precision=%s" % (bhq.KERNEL_NAMES[bk],
                                               bhq.PRECISION_NAMES[prec]))
            a, p = run(ctx, mat, len(m), bk, prec)
            err = errors(a, p, a_ref, p_ref)
            log("    %s" % err)
            assert_parity(err, prec, "split %s %s" % (bk, prec))
            # instances with capped registers (6 and 8 waves per SIMD),
            # eager and persistent: the same arithmetic, the same bits
            for w in (6, 8):
                for pers in (0, 1):
                    bhq.bhq_set_tuning(ctx, 256, 2, 0, pers, 0, 1, w)
                    aw, pw = run(ctx, mat, len(m), bk, prec)
                    bhq.bhq_set_tuning(ctx)
                    assert np.array_equal(a, aw) and np.array_equal(p, pw), (w, pers)
            # cross-block j-split: the parts' cutoff decisions (and the FP32
            # band's FP64 re-decisions) read the entries of their own part
            for js in (2, 4):
                try:
                    bhq.bhq_set_tuning(ctx, 256, 2, 0, 0, 0, js)
                    aj, pj = run(ctx, mat, len(m), bk, prec)
                    assert_parity(errors(aj, pj, a_ref, p_ref), prec,
                                  "split %s %s jsplit %d" % (bk, prec, js))
                    bhq.bhq_set_tuning(ctx, 256, 2, 2, 1, 0, js)
                    ap, pp = run(ctx, mat, len(m), bk, prec)
                finally:
                    bhq.bhq_set_tuning(ctx)
                assert np.array_equal(aj, ap) and np.array_equal(pj, pp), js


def test_split_multipass_groups(ctx):
    """Split kernels on groups larger than one pass of the block (up to 539
    i-particles: two passes at two i-particles per thread, three at one):
    the cutoff decisions and the FP32 band's FP64 re-decisions index the
    i-particles of the current pass."""
    x, m = synth.perturbed_lattice(32, synth.rng(9))
    rs = 1.25 / 32
    rcut = 4.5 * rs
    T = orc.Tree(x, m, 0.5, 600, box=1.0, rcut=rcut)
    assert np.diff(T.i_off).max() > 512
    mat = orc.materialise(T, x, m)
    assert orc.mask_flips(mat, x, 1.0, rcut) == 0
    upload(ctx, mat, x, split=(rs, rcut, 1.0))
    try:
        for bk, ok in ((bhq.SPLIT_QUAD, orc.SPLIT_QUAD), (bhq.SPLIT_MONO, orc.SPLIT_MONO)):
            a_ref, p_ref = orc.eval_lists(ok, mat, x, 0.0, box=1.0, rs=rs, rcut=rcut,
                                          mask=orc.MASK_F64_OFS)
            for prec in PRECS:
                for shape in ((256, 2, 0, 0, 0, 1), (256, 1, 0, 0, 0, 1), (256, 2, 0, 0, 0, 2)):
                    bhq.bhq_set_tuning(ctx, *shape)
                    a, p = run(ctx, mat, len(m), bk, prec)
                    err = errors(a, p, a_ref, p_ref)
                    log("case split multipass kernel=%s precision=%s shape=%s %s"
                        % (bhq.KERNEL_NAMES[bk], bhq.PRECISION_NAMES[prec], shape, err))
                    assert_parity(err, prec, "split multipass %s %s %s" % (bk, prec, shape))
    finally:
        bhq.bhq_set_tuning(ctx)


def test_count_live_and_clock(ctx):
    """bhq_count_live counts the terms the cutoff keeps exactly as the
    oracle's definition does (materialised and index lists); the clock
    window reports a shader clock in a physical range."""
    torch = pytest.importorskip("torch")
    x, m = synth.perturbed_lattice(24, synth.rng(4))
    rs = 1.25 / 24
    rcut = 4.5 * rs
    T = orc.Tree(x, m, 0.5, 64, box=1.0, rcut=rcut)
    mat = orc.materialise(T, x, m)
    want = orc.count_keep(mat, x, 1.0, rcut, mask=orc.MASK_ABS)
    assert want == orc.count_keep(mat, x, 1.0, rcut, mask=orc.MASK_F64_OFS)
    upload(ctx, mat, x, split=(rs, rcut, 1.0))
    bhq.bhq_set_kernel(ctx, bhq.SPLIT_QUAD, bhq.FP32_OFS64)
    got = bhq.bhq_count_live(ctx)
    log("  live pairs %s of %s" % (got, bhq.bhq_get_counts(ctx)))
    assert got == want
    _upload_indexed(ctx, T, mat, x, m, split=(rs, rcut, 1.0))
    assert bhq.bhq_count_live(ctx) == want
    bhq.bhq_set_kernel(ctx, bhq.QUAD, bhq.FP32_OFS64)
    with pytest.raises(bhq.BhqError) as ei:
        bhq.bhq_count_live(ctx)
    assert ei.value.code == bhq.E_STATE
    s = torch.cuda.Stream()
    bhq.bhq_clock_begin(ctx, 20.0, s)
    mhz = bhq.bhq_clock_end(ctx)
    log("  clock window: %.0f MHz" % mhz)
    assert 100.0 < mhz < 4000.0
    with pytest.raises(bhq.BhqError) as ei:
        bhq.bhq_clock_end(ctx)
    assert ei.value.code == bhq.E_STATE


def _upload_indexed(ctx, T, mat, x, m, eps2=None, split=None):
    x = np.asarray(x, np.float64).reshape(-1, 3)
    bhq.bhq_set_groups(ctx, mat["i_off"], mat["gcenter"], mat["jp_off"],
                       mat["jc_off"])
    bhq.bhq_set_i(ctx, x[mat["i_idx"]])
    if eps2 is not None:
        e2 = np.broadcast_to(np.asarray(eps2, np.float64), (x.shape[0],))
        bhq.bhq_set_eps2_i(ctx, np.ascontiguousarray(e2[mat["i_idx"]]))
    if split is not None:
        bhq.bhq_set_split(ctx, *split)
    bhq.bhq_set_pool_particles(ctx, x, m)
    bhq.bhq_set_pool_cells(ctx, T.com, T.mass, T.q, T.trace)
    bhq.bhq_set_jp_idx(ctx, 0, T.jp_idx)
    bhq.bhq_set_jc_idx(ctx, 0, T.jc_node)


def test_index_lists_equal_materialised(ctx):
    """Index-mode lists (pools + int32 indices) give bitwise the result of
    materialised lists: the same FP64 data reach the same arithmetic."""
    c = synth.config_plummer_16k()
    x, m = c["x"], c["m"]
    T = orc.Tree(x, m, 0.5, 64)
    mat = orc.materialise(T, x, m)
    e2 = c["eps"] ** 2
    ref = {}
    upload(ctx, mat, x, eps2=e2)
    for bk in (bhq.QUAD, bhq.MONO):
        for prec in PRECS:
            ref[(bk, prec)] = run(ctx, mat, len(m), bk, prec)
    log("case index lists plummer16k")
    _upload_indexed(ctx, T, mat, x, m, eps2=e2)
    for (bk, prec), (a0, p0) in ref.items():
        a1, p1 = run(ctx, mat, len(m), bk, prec)
        assert np.array_equal(a0, a1) and np.array_equal(p0, p1), (bk, prec)
    a_ref, p_ref = orc.eval_lists(orc.QUAD, mat, x, e2)
    a, p = run(ctx, mat, len(m), bhq.QUAD, bhq.FP32_OFS64)
    assert_parity(errors(a, p, a_ref, p_ref), bhq.FP32_OFS64, "indexed")


def test_split_fp32_cutoff_range(ctx):
    """FP32 split kernels take erfc and the related functions from a table
    of r / 2r_s in [0, 2.5] (plus one interval for the rounding of r at the
    cutoff): a cutoff of 5 r_s is accepted and evaluated to the FP32 bar,
    5.2 r_s, 7.5 r_s and 9 r_s are refused for FP32 and accepted for FP64.
    FP64 takes exp(-u^2) and erfc from its table up to u = 4 (8 r_s) and
    from the library beyond, so 9 r_s runs both forms side by side."""
    x, m = synth.perturbed_lattice(8, synth.rng(4))
    rs = 0.04
    for rcut in (0.3, 5.2 * rs, 9.0 * rs):
        T = orc.Tree(x, m, 0.5, 64, box=1.0, rcut=rcut)
        mat = orc.materialise(T, x, m)
        upload(ctx, mat, x, split=(rs, rcut, 1.0))
        bhq.bhq_set_kernel(ctx, bhq.SPLIT_QUAD, bhq.FP32_OFS64)
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_compute(ctx)
        assert ei.value.code == bhq.E_ARG
        a_ref, p_ref = orc.eval_lists(orc.SPLIT_QUAD, mat, x, 0.0, box=1.0, rs=rs,
                                      rcut=rcut, mask=orc.MASK_F64_OFS)
        a, p = run(ctx, mat, len(m), bhq.SPLIT_QUAD, bhq.FP64)
        assert_parity(errors(a, p, a_ref, p_ref), bhq.FP64, "split fp64 rcut %g" % rcut)
    # the accepted edge: terms out to u = 2.5, the last table interval
    # (group cells of 1/8 plus 2 rcut stay below half the box)
    x, m = synth.perturbed_lattice(24, synth.rng(5))
    rs = 1.25 / 64
    rcut = 5.0 * rs
    T = orc.Tree(x, m, 0.5, 64, box=1.0, rcut=rcut)
    mat = orc.materialise(T, x, m)
    assert orc.mask_flips(mat, x, 1.0, rcut) == 0
    upload(ctx, mat, x, split=(rs, rcut, 1.0))
    for bk, ok in ((bhq.SPLIT_QUAD, orc.SPLIT_QUAD), (bhq.SPLIT_MONO, orc.SPLIT_MONO)):
        a_ref, p_ref = orc.eval_lists(ok, mat, x, 0.0, box=1.0, rs=rs, rcut=rcut,
                                      mask=orc.MASK_F64_OFS)
        for prec in PRECS:
            a, p = run(ctx, mat, len(m), bk, prec)
            err = errors(a, p, a_ref, p_ref)
            log("  rcut = 5 rs kernel=%s precision=%s %s"
                % (bhq.KERNEL_NAMES[bk], bhq.PRECISION_NAMES[prec], err))
            assert_parity(err, prec, "split rcut = 5 rs")


def _band_pairs(rcut, deltas, seed):
    """Isolated pairs in the periodic unit box, pair k at separation
    rcut (1 + deltas[k]) along a random direction, pairs 0.2 apart."""
    g = np.random.default_rng(seed)
    n = len(deltas)
    side = int(np.ceil(n ** (1.0 / 3.0)))
    x = np.zeros((2 * n, 3))
    for k, dlt in enumerate(deltas):
        c = (np.array([k % side, (k // side) % side, k // side ** 2]) + 0.5) / side
        c = c + g.uniform(-0.02, 0.02, 3)
        u = g.normal(size=3)
        u /= np.linalg.norm(u)
        x[2 * k] = c
        x[2 * k + 1] = c + rcut * (1.0 + dlt) * u
    return np.mod(x, 1.0), np.full(2 * n, 1.0 / (2 * n))


@pytest.mark.parametrize("ncrit,nleaf", [(2, 2), (16, 8)])
def test_split_cutoff_band_pairs(ctx, ncrit, nleaf):
    """Pairs whose separation lies within FP32 rounding of the cutoff (the
    band where FP32 r^2 cannot tell the sides apart): the FP32 split kernels
    take every such decision as the FP64 definition does, so each pair's
    force is the oracle's (within the FP32 bar) or exactly zero with it.
    Groups of one pair, and of eight pairs (i-particles up to ~0.2 from the
    group centre, which widens the band)."""
    rs = 1.25 / 256
    rcut = 4.5 * rs
    mags = np.geomspace(1e-9, 1e-6, 32)
    deltas = np.concatenate([mags, -mags])
    x, m = _band_pairs(rcut, deltas, 11)
    log("case band pairs ncrit=%d nleaf=%d" % (ncrit, nleaf))
    T = orc.Tree(x, m, 0.0, ncrit, nleaf=nleaf, box=1.0, rcut=rcut)
    mat = orc.materialise(T, x, m)
    assert orc.mask_flips(mat, x, 1.0, rcut) == 0
    upload(ctx, mat, x, split=(rs, rcut, 1.0))
    a_ref, p_ref = orc.eval_lists(orc.SPLIT_MONO, mat, x, 0.0, box=1.0, rs=rs, rcut=rcut,
                                  mask=orc.MASK_F64_OFS)
    kept = np.any(a_ref != 0.0, axis=1)
    # both decisions occur, and they follow the sign of the offset from rcut
    assert np.array_equal(kept[0::2], deltas < 0) and np.array_equal(kept[1::2], deltas < 0)
    for bk in (bhq.SPLIT_MONO, bhq.SPLIT_QUAD):
        for prec in PRECS:
            a, p = run(ctx, mat, len(m), bk, prec)
            log("  band pairs kernel=%s precision=%s: %d of %d particles kept"
                % (bhq.KERNEL_NAMES[bk], bhq.PRECISION_NAMES[prec],
                   int(np.any(a != 0.0, axis=1).sum()), len(m)))
            assert np.array_equal(np.any(a != 0.0, axis=1), kept), (bk, prec)
            assert np.array_equal(p != 0.0, kept), (bk, prec)
            bhq.bhq_set_tuning(ctx, 256, 2, 0, 0, 0, 1, 6)
            aw, pw = run(ctx, mat, len(m), bk, prec)
            bhq.bhq_set_tuning(ctx)
            assert np.array_equal(a, aw) and np.array_equal(p, pw)
            ea = orc.relative_errors(a[kept], a_ref[kept])
            ep = np.abs(p[kept] - p_ref[kept]) / np.abs(p_ref[kept])
            tol = 1e-5 if prec == bhq.FP32_OFS64 else 1e-12
            assert ea.max() <= tol and ep.max() <= tol, (bk, prec, ea.max(), ep.max())
            # the same decisions with the lists cut into parts
            try:
                bhq.bhq_set_tuning(ctx, 256, 2, 0, 0, 0, 4)
                aj, pj = run(ctx, mat, len(m), bk, prec)
            finally:
                bhq.bhq_set_tuning(ctx)
            assert np.array_equal(np.any(aj != 0.0, axis=1), kept), (bk, prec, "jsplit")
            ea = orc.relative_errors(aj[kept], a_ref[kept])
            assert ea.max() <= tol, (bk, prec, "jsplit", ea.max())


def test_index_lists_split_periodic(ctx):
    x, m = synth.perturbed_lattice(24, synth.rng(4))
    rs, box = 1.25 / 24, 1.0
    rcut = 4.5 * rs
    T = orc.Tree(x, m, 0.5, 64, box=box, rcut=rcut)
    mat = orc.materialise(T, x, m)
    log("case index lists split lattice 24^3")
    _upload_indexed(ctx, T, mat, x, m, split=(rs, rcut, box))
    for prec in PRECS:
        a_ref, p_ref = orc.eval_lists(orc.SPLIT_QUAD, mat, x, 0.0, box=box,
                                      rs=rs, rcut=rcut, mask=orc.MASK_F64_OFS)
        a, p = run(ctx, mat, len(m), bhq.SPLIT_QUAD, prec)
        err = errors(a, p, a_ref, p_ref)
        log("  precision=%s %s" % (bhq.PRECISION_NAMES[prec], err))
        assert_parity(err, prec, "indexed split")
        try:
            bhq.bhq_set_tuning(ctx, 256, 2, 0, 0, 0, 4)
            a, p = run(ctx, mat, len(m), bhq.SPLIT_QUAD, prec)
        finally:
            bhq.bhq_set_tuning(ctx)
        assert_parity(errors(a, p, a_ref, p_ref), prec, "indexed split jsplit 4")


def test_index_list_errors(ctx):
    c2 = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        bhq.bhq_set_groups(c2, [0, 2], np.zeros((1, 3)), [0, 3], [0, 1])
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_set_jp_idx(c2, 0, [0, 1, 2])   # no pool yet
        assert ei.value.code == bhq.E_STATE
        bhq.bhq_set_pool_particles(c2, np.random.default_rng(0).random((3, 3)),
                                   np.ones(3))
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_set_jp_idx(c2, 0, [0, 1, 3])   # 3 is outside the pool
        assert ei.value.code == bhq.E_RANGE
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_set_jp_idx(c2, 0, [0, -1, 2])
        assert ei.value.code == bhq.E_RANGE
        bhq.bhq_set_jp_idx(c2, 0, [0, 1, 2])
        with pytest.raises(bhq.BhqError) as ei:          # mixing modes
            bhq.bhq_set_jc(c2, 0, np.zeros((1, 3)), [1.0], np.zeros((1, 6)))
        assert ei.value.code == bhq.E_STATE
        bhq.bhq_set_i(c2, np.random.default_rng(1).random((2, 3)))
        bhq.bhq_set_eps(c2, 0.1)
        with pytest.raises(bhq.BhqError) as ei:          # jc indices missing
            bhq.bhq_compute(c2)
        assert ei.value.code == bhq.E_STATE
        bhq.bhq_set_pool_cells(c2, np.zeros((1, 3)), [0.5], np.zeros((1, 6)))
        bhq.bhq_set_jc_idx(c2, 0, [0])
        bhq.bhq_compute(c2)
        a, p = bhq.bhq_get_result(c2, 2)
        assert np.all(np.isfinite(a)) and np.all(p < 0)
    finally:
        bhq.bhq_destroy(c2)


def test_product_index_lists_equal_materialised(ctx):
    x, m = synth.clustered(1 << 15, synth.rng(2))
    L = bhq.bhq_build_lists(x, m, 0.5, 128)
    try:
        bhq.bhq_set_lists(ctx, L, x, m)
        bhq.bhq_set_eps(ctx, 2e-4)
        out = []
        for mode in ("materialised", "indexed"):
            if mode == "indexed":
                bhq.bhq_set_lists_indexed(ctx, L, x, m)
                bhq.bhq_set_eps(ctx, 2e-4)
            log("case product lists %s" % mode)
            bhq.bhq_set_kernel(ctx, bhq.QUAD, bhq.FP32_OFS64)
            bhq.bhq_compute(ctx)
            out.append(bhq.bhq_get_result(ctx, len(m)))
        assert np.array_equal(out[0][0], out[1][0])
        assert np.array_equal(out[0][1], out[1][1])
    finally:
        bhq.bhq_lists_free(L)


def test_quad_soft_index_lists_and_trace_effect():
    """The complete softened quadrupole on index lists from the host
    builder (cell traces from the cell pool) against the oracle's own tree;
    with a large softening the trace term moves the result well beyond the
    FP64 bar, so the comparison shows the kernel uses it."""
    x, m = synth.plummer(12000, synth.rng(14))
    eps = 0.08
    T = orc.Tree(x, m, 0.6, 64)
    mat = orc.materialise(T, x, m)
    ref_soft = orc.eval_lists(orc.QUAD_SOFT, mat, x, eps * eps)
    ref_quad = orc.eval_lists(orc.QUAD, mat, x, eps * eps)
    diff = errors(ref_soft[0], ref_soft[1], ref_quad[0], ref_quad[1])
    log("case quad_soft: oracle soft vs traceless %s" % diff)
    assert diff["rms"] > 1e-6
    L = bhq.bhq_build_lists(x, m, 0.6, 64)
    c = bhq.bhq_create(0, bhq.QUAD_SOFT, bhq.FP32_OFS64)
    try:
        bhq.bhq_set_lists_indexed(c, L, x, m)
        idx = bhq.bhq_lists_export(L, len(m))["i_idx"]
        bhq.bhq_set_eps(c, eps)
        for prec in PRECS:
            bhq.bhq_set_kernel(c, bhq.QUAD_SOFT, prec)
            bhq.bhq_compute(c)
            a_g, p_g = bhq.bhq_get_result(c, len(m))
            a = np.zeros_like(a_g)
            p = np.zeros_like(p_g)
            a[idx] = a_g
            p[idx] = p_g
            err = errors(a, p, *ref_soft)
            log("  precision=%s %s" % (bhq.PRECISION_NAMES[prec], err))
            assert_parity(err, prec, "quad_soft index lists")
    finally:
        bhq.bhq_lists_free(L)
        bhq.bhq_destroy(c)
