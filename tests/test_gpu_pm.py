"""GPU: the particle-mesh long-range force against the FP64 particle-mesh
reference (same method, different code), against the mesh-free
wave-vector sum, and the TreePM total (split-kernel tree + PM) against the
oracle's split tree plus its PM."""
import numpy as np
import pytest

import oracle as orc
from oracle import pm as opm
from _parity import log
from paper_1812_07313_amd import bhq, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


def _rel(a, ref):
    """Errors relative to the rms of the reference."""
    scale = np.sqrt((ref ** 2).sum(-1).mean()) if ref.ndim == 2 else np.sqrt((ref ** 2).mean())
    return np.abs(a - ref).max() / scale


@pytest.mark.parametrize("n,nmesh", [(3000, 32), (20000, 64)])
def test_pm_matches_reference(n, nmesh):
    g = np.random.default_rng(n)
    x = g.random((n, 3))
    m = g.uniform(0.5, 1.5, n) / n
    rs = 1.25 / nmesh
    a_ref, p_ref = opm.pm(x, m, 1.0, nmesh, rs)
    pm = bhq.bhq_pm_create(nmesh, 1.0, rs)
    try:
        xt, mt = _t(x), _t(m)
        a = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
        p = torch.zeros(n, dtype=torch.float64, device="cuda")
        bhq.bhq_pm_compute(pm, xt, mt, a, p)
        ms = bhq.bhq_pm_get_ms(pm)
        ea, ep = _rel(a.cpu().numpy(), a_ref), _rel(p.cpu().numpy(), p_ref)
        log("case pm n=%d mesh=%d: force %.3g pot %.3g (rel. to rms), %.3f ms"
            % (n, nmesh, ea, ep, ms))
        assert ea < 1e-11 and ep < 1e-11
        # bitwise reproducible; accumulate adds the same values
        a1, p1 = a.cpu().numpy(), p.cpu().numpy()
        bhq.bhq_pm_compute(pm, xt, mt, a, p)
        assert np.array_equal(a.cpu().numpy(), a1) and np.array_equal(p.cpu().numpy(), p1)
        bhq.bhq_pm_compute(pm, xt, mt, a, p, accumulate=True)
        assert np.array_equal(a.cpu().numpy(), a1 + a1)
    finally:
        bhq.bhq_pm_destroy(pm)


def test_pm_clustered_reads_memory():
    """A clump: the neighbourhood of the tiles around it holds more particles
    than the assignment keeps in LDS, so those tiles read the particles
    from memory.  The result matches the reference as elsewhere, and is
    the same bits every run."""
    n, nmesh = 6000, 32
    g = np.random.default_rng(17)
    x = (0.5 + g.normal(size=(n, 3)) * 0.6 / nmesh) % 1.0
    m = g.uniform(0.5, 1.5, n) / n
    rs = 1.25 / nmesh
    a_ref, p_ref = opm.pm(x, m, 1.0, nmesh, rs)
    pm = bhq.bhq_pm_create(nmesh, 1.0, rs)
    try:
        xt, mt = _t(x), _t(m)
        a = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
        p = torch.zeros(n, dtype=torch.float64, device="cuda")
        bhq.bhq_pm_compute(pm, xt, mt, a, p)
        ea, ep = _rel(a.cpu().numpy(), a_ref), _rel(p.cpu().numpy(), p_ref)
        log("case pm clump n=%d mesh=%d: force %.3g pot %.3g" % (n, nmesh, ea, ep))
        assert ea < 1e-11 and ep < 1e-11
        a1 = a.cpu().numpy()
        bhq.bhq_pm_compute(pm, xt, mt, a, p)
        assert np.array_equal(a.cpu().numpy(), a1)
    finally:
        bhq.bhq_pm_destroy(pm)


def test_pm_against_k_sum():
    """One unit mass: the GPU mesh force agrees with the mesh-free sum to
    the TSC accuracy at r_s = 1.25 mesh spacings."""
    nmesh, rs = 32, 1.25 / 32
    g = np.random.default_rng(5)
    xp = g.random((1, 3))
    pts = (xp + g.normal(size=(80, 3)) * 4 * rs) % 1.0
    x = np.vstack([xp, pts])
    m = np.concatenate([[1.0], np.zeros(80)])
    pm = bhq.bhq_pm_create(nmesh, 1.0, rs)
    try:
        a = torch.zeros((81, 3), dtype=torch.float64, device="cuda")
        bhq.bhq_pm_compute(pm, _t(x), _t(m), a)
        a_pm = a.cpu().numpy()[1:]
    finally:
        bhq.bhq_pm_destroy(pm)
    a_ex, _ = opm.direct_k_sum(pts, xp, [1.0], 1.0, rs)
    e = np.linalg.norm(a_pm - a_ex, axis=1) / np.linalg.norm(a_ex, axis=1)
    log("case pm vs k-sum: rms %.3g max %.3g" % (np.sqrt((e * e).mean()), e.max()))
    assert np.sqrt((e * e).mean()) < 1e-2


def test_treepm_total_matches_oracle():
    """Perturbed 16^3 lattice: device lists + FP64 split tree + PM on the
    GPU equals the oracle's split tree (its own lists) plus its PM."""
    x, m = synth.perturbed_lattice(16, synth.rng(4))
    nmesh = 16
    rs = 1.25 / nmesh
    rcut = 4.5 * rs
    T = orc.Tree(x, m, 0.5, 32, box=1.0, rcut=rcut)
    mat = orc.materialise(T, x, m)
    a_s, p_s = orc.eval_lists(orc.SPLIT_QUAD, mat, x, 0.0, box=1.0, rs=rs, rcut=rcut,
                              mask=orc.MASK_F64_OFS)
    a_l, p_l = opm.pm(x, m, 1.0, nmesh, rs)
    ctx = bhq.bhq_create(0, bhq.SPLIT_QUAD, bhq.FP64)
    pm = bhq.bhq_pm_create(nmesh, 1.0, rs)
    try:
        xt, mt = _t(x), _t(m)
        bhq.bhq_build_lists_device(ctx, xt, mt, 0.5, 32, 8, 1.0, rcut)
        bhq.bhq_set_split(ctx, rs, rcut, 1.0)
        bhq.bhq_compute(ctx)
        a = torch.zeros((len(m), 3), dtype=torch.float64, device="cuda")
        p = torch.zeros(len(m), dtype=torch.float64, device="cuda")
        bhq.bhq_get_result_device(ctx, a, p)
        bhq.bhq_pm_compute(pm, xt, mt, a, p, accumulate=True)
        ag, pg = a.cpu().numpy(), p.cpu().numpy()
    finally:
        bhq.bhq_pm_destroy(pm)
        bhq.bhq_destroy(ctx)
    e = _rel(ag, a_s + a_l)
    log("case treepm 16^3: total force vs oracle %.3g; long/short rms ratio %.3g"
        % (e, np.sqrt((a_l ** 2).sum(1).mean() / (a_s ** 2).sum(1).mean())))
    assert e < 1e-10
    assert _rel(pg, p_s + p_l) < 1e-10


def test_pm_errors():
    for args in ((3, 1.0, 0.1), (33, 1.0, 0.1), (32, 0.0, 0.1), (32, 1.0, -1.0),
                 (2048, 1.0, 0.1)):
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_pm_create(*args)
        assert ei.value.code == bhq.E_ARG
    pm = bhq.bhq_pm_create(16, 1.0, 0.1)
    try:
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_pm_get_ms(pm)
        assert ei.value.code == bhq.E_STATE
        x = np.random.default_rng(1).random((10, 3))
        a = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
        rc = bhq.lib().bhq_pm_compute(pm, 10, x.ctypes.data, _t(np.ones(10)).data_ptr(),
                                      a.data_ptr(), None, 0, None)
        assert rc == bhq.E_ARG
    finally:
        bhq.bhq_pm_destroy(pm)
