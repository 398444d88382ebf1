"""GPU parity at the benchmark configurations' full sizes, in the launch
configuration bench.py times: lists from the library's host builder
uploaded as index lists, one 256-thread block per group in LPT order.
The oracle builds its own tree and lists; where it cannot evaluate every
particle in seconds it walks every k-th group and those groups' particles
are compared (the two builders' lists are identical, which the CPU tests
check on smaller inputs).

Bars: FP32 with FP64 offsets <= 2e-6 rms and <= 1e-4 max relative
acceleration error per particle; FP64 <= 1e-12 rms and <= 1e-10 max.  For
the short-range split kernel the oracle decides the cutoff from FP64
offsets to the group centres, which on the compared lists is shown to agree
with the definition's absolute FP64 separations term by term.
"""
import numpy as np
import pytest

import oracle as orc
from _parity import assert_parity, errors, log
from paper_1812_07313_amd import bhq, synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _gpu_product(x, m, theta, ncrit, kernel, eps=None, eps2=None, box=0.0,
                 rcut=0.0, rs=0.0, sys_off=None, tuning=None, replays=1):
    """Bench configuration: host builder lists, index upload, the default
    launch or the given bhq_set_tuning arguments; returns {precision:
    (a, phi)} in original particle order.  With replays > 1 every further
    compute (a graph replay when the tuning asks for one) must give the
    first one's result bit for bit."""
    if sys_off is not None:
        L = bhq.bhq_build_lists_batch(sys_off, x, m, theta, ncrit)
    else:
        L = bhq.bhq_build_lists(x, m, theta, ncrit, box=box, rcut=rcut)
    ctx = bhq.bhq_create(0, kernel, bhq.FP32_OFS64)
    out = {}
    try:
        bhq.bhq_set_lists_indexed(ctx, L, x, m)
        idx = bhq.bhq_lists_export(L, len(m))["i_idx"]
        bhq.bhq_lists_free(L)
        L = None
        if eps2 is not None:
            bhq.bhq_set_eps2_i(ctx, eps2[idx])
        elif eps is not None:
            bhq.bhq_set_eps(ctx, eps)
        if rs:
            bhq.bhq_set_split(ctx, rs, rcut, box)
        if tuning is not None:
            bhq.bhq_set_tuning(ctx, *tuning)
        for prec in (bhq.FP32_OFS64, bhq.FP64):
            bhq.bhq_set_kernel(ctx, kernel, prec)
            bhq.bhq_compute(ctx)
            a_g, p_g = bhq.bhq_get_result(ctx, len(m))
            for _ in range(replays - 1):
                bhq.bhq_compute(ctx)
                a_r, p_r = bhq.bhq_get_result(ctx, len(m))
                assert np.array_equal(a_g, a_r) and np.array_equal(p_g, p_r)
            a = np.empty_like(a_g)
            p = np.empty_like(p_g)
            a[idx] = a_g
            p[idx] = p_g
            out[prec] = (a, p)
    finally:
        if L is not None:
            bhq.bhq_lists_free(L)
        bhq.bhq_destroy(ctx)
    return out


def _check(name, gpu, ref_fn, sel):
    for prec, (a, p) in gpu.items():
        a_ref, p_ref = ref_fn(prec)
        err = errors(a[sel], p[sel], a_ref[sel], p_ref[sel])
        log("  %s precision=%s on %d particles: %s"
            % (name, bhq.PRECISION_NAMES[prec], len(sel), err))
        assert_parity(err, prec, name)


def test_uniform_cube_1m():
    """Uniform cube N = 2^20, eps = 1e-3, theta = 0.5, ncrit = 256: every
    particle, quadrupole and monopole kernels."""
    c = synth.config_uniform_cube()
    x, m, eps = c["x"], c["m"], c["eps"]
    log("case cube 2^20 (all particles)")
    T = orc.Tree(x, m, 0.5, 256)
    mat = orc.materialise(T, x, m)
    sel = np.arange(len(m))
    for bk, ok in ((bhq.QUAD, orc.QUAD), (bhq.MONO, orc.MONO)):
        gpu = _gpu_product(x, m, 0.5, 256, bk, eps=eps)
        ref = orc.eval_lists(ok, mat, x, eps * eps)
        _check("cube %s" % bhq.KERNEL_NAMES[bk], gpu, lambda prec: ref, sel)


def test_plummer_16k_bench_shapes():
    """Plummer sphere N = 16384, eps = 1/64, theta = 0.5, ncrit = 64, at
    every launch shape the bench times for it (1 or 2 i-particles per
    thread, cross-block j-split 1 to 8, registers capped for 6 or 8 waves):
    every particle against the oracle."""
    c = synth.config_plummer_16k()
    x, m, eps = c["x"], c["m"], c["eps"]
    T = orc.Tree(x, m, 0.5, 64)
    ref = orc.eval_lists(orc.QUAD, orc.materialise(T, x, m), x, eps * eps)
    shapes = [(256, ipt, 0, 0, 0, js) for ipt in (1, 2) for js in (1, 2, 4, 8)]
    shapes += [(256, 1, 0, 0, 0, js, w) for js in (2, 4) for w in (6, 8)]
    for shape in shapes:
        log("case plummer16k shape %s" % (shape,))
        gpu = _gpu_product(x, m, 0.5, 64, bhq.QUAD, eps=eps, tuning=shape)
        _check("plummer16k %s" % (shape,), gpu, lambda prec: ref, np.arange(len(m)))


def test_clustered_4m_sampled():
    """512 Plummer clusters + background, N = 2^22, eps = 2e-4,
    theta = 0.5, ncrit = 256: the particles of every 64th group."""
    c = synth.config_clustered()
    x, m, eps = c["x"], c["m"], c["eps"]
    log("case clustered 2^22 (sampled groups)")
    gpu = _gpu_product(x, m, 0.5, 256, bhq.QUAD, eps=eps)
    log("  persistent per-XCD queues (a launch the bench times)")
    gpu_p = _gpu_product(x, m, 0.5, 256, bhq.QUAD, eps=eps, tuning=(256, 2, 0, 1, 0, 1))
    for prec in gpu:
        assert np.array_equal(gpu[prec][0], gpu_p[prec][0])
        assert np.array_equal(gpu[prec][1], gpu_p[prec][1])
    T = orc.Tree(x, m, 0.5, 256, walk_stride=64)
    groups = np.arange(0, T.ngroups, 64)
    mat = T.sample_mat(x, m, groups)
    ref = orc.eval_lists(orc.QUAD, mat, x, eps * eps)
    _check("clustered", gpu, lambda prec: ref, mat["i_idx"])


def test_batched_256_systems():
    """256 Plummer systems, N log-uniform in [2^10, 2^16], own eps each,
    theta = 0.6, ncrit = 64: every particle, from one eager launch and from
    one persistent launch replayed from a HIP graph (three replays, each
    bitwise equal to the eager launch's result)."""
    systems = synth.batched_plummer(256)
    sizes = np.array([len(s[1]) for s in systems])
    off = np.concatenate([[0], np.cumsum(sizes)])
    X = np.concatenate([s[0] for s in systems])
    M = np.concatenate([s[1] for s in systems])
    E2 = np.concatenate([np.full(len(s[1]), s[2] ** 2) for s in systems])
    log("case batched 256 systems, %d particles" % len(M))
    gpu = _gpu_product(X, M, 0.6, 64, bhq.QUAD, eps2=E2, sys_off=off)
    log("  persistent launch replayed from a HIP graph")
    gpu_graph = _gpu_product(X, M, 0.6, 64, bhq.QUAD, eps2=E2, sys_off=off,
                             tuning=(256, 2, 0, 1, 1, 1), replays=3)
    for prec in gpu:
        assert np.array_equal(gpu[prec][0], gpu_graph[prec][0])
        assert np.array_equal(gpu[prec][1], gpu_graph[prec][1])
    a_ref = np.zeros((len(M), 3))
    p_ref = np.zeros(len(M))
    for s, (x, m, eps) in enumerate(systems):
        T = orc.Tree(x, m, 0.6, 64)
        a, p = orc.eval_lists(orc.QUAD, orc.materialise(T, x, m), x, eps * eps)
        a_ref[off[s]:off[s + 1]] = a
        p_ref[off[s]:off[s + 1]] = p
    _check("batched", gpu, lambda prec: (a_ref, p_ref), np.arange(len(M)))
    # ncrit 128 (the bench's choice among 64 and 128), one i-particle per
    # thread with registers capped for 6 waves, eager and from a replayed
    # persistent graph
    log("  ncrit 128, 1 i/thread, 6 waves: eager and persistent graph")
    gpu = _gpu_product(X, M, 0.6, 128, bhq.QUAD, eps2=E2, sys_off=off,
                       tuning=(256, 1, 0, 0, 0, 1, 6))
    gpu_graph = _gpu_product(X, M, 0.6, 128, bhq.QUAD, eps2=E2, sys_off=off,
                             tuning=(256, 1, 0, 1, 1, 1, 6), replays=3)
    for prec in gpu:
        assert np.array_equal(gpu[prec][0], gpu_graph[prec][0])
        assert np.array_equal(gpu[prec][1], gpu_graph[prec][1])
    for s, (x, m, eps) in enumerate(systems):
        T = orc.Tree(x, m, 0.6, 128)
        a, p = orc.eval_lists(orc.QUAD, orc.materialise(T, x, m), x, eps * eps)
        a_ref[off[s]:off[s + 1]] = a
        p_ref[off[s]:off[s + 1]] = p
    _check("batched ncrit 128", gpu, lambda prec: (a_ref, p_ref), np.arange(len(M)))


def test_periodic_lattice_16m_sampled():
    """Perturbed lattice N = 2^24 in the periodic unit box, Gaussian split
    r_s = 1.25/256, cutoff 4.5 r_s, theta = 0.5, ncrit = 64: the particles
    of every 2000th group."""
    c = synth.config_lattice()
    x, m, rs, rcut = c["x"], c["m"], c["rs"], c["rcut"]
    log("case lattice 2^24 (sampled groups)")
    gpu = _gpu_product(x, m, 0.5, 64, bhq.SPLIT_QUAD, box=1.0, rcut=rcut,
                       rs=rs)
    T = orc.Tree(x, m, 0.5, 64, box=1.0, rcut=rcut, walk_stride=2000)
    groups = np.arange(0, T.ngroups, 2000)
    mat = T.sample_mat(x, m, groups)
    flips = orc.mask_flips(mat, x, 1.0, rcut)
    log("  cutoff decisions differing from the definition's: %d" % flips)
    assert flips == 0
    ref = orc.eval_lists(orc.SPLIT_QUAD, mat, x, 0.0, box=1.0, rs=rs, rcut=rcut,
                         mask=orc.MASK_F64_OFS)
    _check("lattice", gpu, lambda prec: ref, mat["i_idx"])
    # the configuration the bench times: ncrit 128, registers capped for 6
    # waves (FP64 runs its own instance)
    log("case lattice 2^24 at ncrit 128, 6 waves (sampled groups)")
    gpu = _gpu_product(x, m, 0.5, 128, bhq.SPLIT_QUAD, box=1.0, rcut=rcut, rs=rs,
                       tuning=(256, 2, 0, 0, 0, 1, 6))
    T = orc.Tree(x, m, 0.5, 128, box=1.0, rcut=rcut, walk_stride=2000)
    mat = T.sample_mat(x, m, np.arange(0, T.ngroups, 2000))
    assert orc.mask_flips(mat, x, 1.0, rcut) == 0
    ref = orc.eval_lists(orc.SPLIT_QUAD, mat, x, 0.0, box=1.0, rs=rs, rcut=rcut,
                         mask=orc.MASK_F64_OFS)
    _check("lattice ncrit 128", gpu, lambda prec: ref, mat["i_idx"])


@pytest.mark.parametrize("which", ["cube", "clustered", "lattice", "batched"])
def test_device_lists_full_size(which):
    """Device-built lists at the benchmark sizes equal the host builder's
    entry for entry (particle order, offsets, every list entry in order)
    and the cell moments bit for bit."""
    torch = pytest.importorskip("torch")
    if which == "cube":
        c = synth.config_uniform_cube()
        box = rcut = 0.0
    elif which == "clustered":
        c = synth.config_clustered()
        box = rcut = 0.0
    elif which == "lattice":
        c = synth.config_lattice()
        box, rcut = 1.0, c["rcut"]
    else:
        systems = synth.batched_plummer(256)
        sizes = np.array([len(q[1]) for q in systems])
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        c = dict(x=np.concatenate([q[0] for q in systems]),
                 m=np.concatenate([q[1] for q in systems]), theta=0.6)
        box = rcut = 0.0
    x, m = c["x"], c["m"]
    ncrit = 64 if which in ("lattice", "batched") else 256
    log("case device lists full size %s (n=%d)" % (which, len(m)))
    if which == "batched":
        L = bhq.bhq_build_lists_batch(off, x, m, c["theta"], ncrit)
    else:
        L = bhq.bhq_build_lists(x, m, c["theta"], ncrit, box=box, rcut=rcut)
    try:
        h = bhq.bhq_lists_export(L, len(m))
        hc = bhq.bhq_lists_cells(L)
        hs = bhq.bhq_lists_sizes(L)
    finally:
        bhq.bhq_lists_free(L)
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        xt = torch.from_numpy(x).cuda()
        mt = torch.from_numpy(m).cuda()
        # the first build counts, then fills; the rebuild walks once into
        # slots sized from the first (same lists either way)
        for build in range(2):
            if which == "batched":
                bhq.bhq_build_lists_device_batch(ctx, off, xt, mt, c["theta"], ncrit)
            else:
                bhq.bhq_build_lists_device(ctx, xt, mt, c["theta"], ncrit, 8, box, rcut)
            assert bhq.bhq_get_build_info(ctx)[0] == (build == 1)
            assert bhq.bhq_get_lists_sizes(ctx) == hs
            d = bhq.bhq_get_lists(ctx, len(m))
            for k in ("i_idx", "i_off", "jp_off", "jc_off", "jc_cell", "jp_idx"):
                assert np.array_equal(h[k], d[k]), (build, k)
                del d[k]
            dc = bhq.bhq_get_cells(ctx)
            for k in ("com", "mass", "q", "trace"):
                assert np.array_equal(hc[k].view(np.int64), dc[k].view(np.int64)), (build, k)
            log("  build %d: %d groups, %d + %d entries, %d cells: identical" % ((build,) + hs))
        del xt, mt
    finally:
        bhq.bhq_destroy(ctx)


def test_pm_lattice_16m():
    """The particle-mesh long-range force on the 2^24 lattice with the
    benchmark's mesh (256^3, r_s = 1.25 mesh spacings) against the FP64 PM
    reference, every particle."""
    torch = pytest.importorskip("torch")
    from oracle import pm as opm
    c = synth.config_lattice()
    x, m, rs = c["x"], c["m"], c["rs"]
    log("case pm lattice 2^24, mesh 256")
    a_ref, p_ref = opm.pm(x, m, 1.0, 256, rs)
    pm = bhq.bhq_pm_create(256, 1.0, rs)
    try:
        xt = torch.from_numpy(x).cuda()
        mt = torch.from_numpy(m).cuda()
        a = torch.zeros((len(m), 3), dtype=torch.float64, device="cuda")
        p = torch.zeros(len(m), dtype=torch.float64, device="cuda")
        bhq.bhq_pm_compute(pm, xt, mt, a, p)
        ag, pg = a.cpu().numpy(), p.cpu().numpy()
    finally:
        bhq.bhq_pm_destroy(pm)
    sa = np.sqrt((a_ref ** 2).sum(1).mean())
    ea = np.abs(ag - a_ref).max() / sa
    ep = np.abs(pg - p_ref).max() / np.sqrt((p_ref ** 2).mean())
    log("  force %.3g, potential %.3g (max error / rms)" % (ea, ep))
    assert ea < 1e-10 and ep < 1e-10
