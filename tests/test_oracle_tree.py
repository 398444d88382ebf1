"""Pins for the oracle's tree, groups, lists and tree accuracy (CPU only).

Structure (Sec. 3.4): groups partition the particles and hold at most
n_crit each; every group's list covers every particle exactly once; each
accepted cell passes the opening criterion l/d < theta (Sec. 1) and its
parent does not.  Accuracy (Sec. 4): theta = 0 is direct summation;
quadrupole errors are below monopole errors at equal theta; errors at the
90th percentile scale roughly as theta^(5/2) (monopole) and theta^(7/2)
(quadrupole), as stated for Fig. 2.
"""
import json
import os

import numpy as np
import pytest

from conftest import GOLDEN
from paper_1812_07313_amd import synth


def _dist2_point_cube(p, c, s):
    v = np.maximum(np.abs(p - c) - 0.5 * s, 0.0)
    return float(np.sum(v * v))


def _check_structure(orc, x, m, theta, ncrit):
    T = orc.Tree(x, m, theta, ncrit)
    n = len(m)
    # groups partition the particles, contiguous in perm order
    assert T.i_off[0] == 0 and T.i_off[-1] == n
    assert np.all(np.diff(T.i_off) > 0)
    assert np.array_equal(np.sort(T.perm), np.arange(n))
    for g in range(T.ngroups):
        nd = T.gnode[g]
        assert T.count[nd] <= ncrit or T.leaf[nd]
        if T.parent[nd] >= 0:
            assert T.count[T.parent[nd]] > ncrit
        assert T.first[nd] == T.i_off[g]
        assert T.count[nd] == T.i_off[g + 1] - T.i_off[g]
    # each list covers each particle exactly once
    for g in range(T.ngroups):
        cover = np.zeros(n, np.int64)
        np.add.at(cover, T.jp_idx[T.jp_off[g]:T.jp_off[g + 1]], 1)
        nd_g = T.gnode[g]
        gc, gs = T.center[nd_g], T.side[nd_g]
        for c in T.jc_node[T.jc_off[g]:T.jc_off[g + 1]]:
            cover[T.perm[T.first[c]:T.first[c] + T.count[c]]] += 1
            assert T.count[c] >= 2
            d2 = _dist2_point_cube(T.com[c], gc, gs)
            assert T.side[c] ** 2 < theta ** 2 * d2
            p = T.parent[c]
            contains = (T.first[p] <= T.first[nd_g] and
                        T.first[nd_g] + T.count[nd_g] <= T.first[p] + T.count[p])
            assert contains or not (T.side[p] ** 2 <
                                    theta ** 2 * _dist2_point_cube(T.com[p], gc, gs))
        assert np.all(cover == 1), g
        # the group's own particles are always direct j-particles
        own = T.perm[T.i_off[g]:T.i_off[g + 1]]
        assert np.all(np.isin(own, T.jp_idx[T.jp_off[g]:T.jp_off[g + 1]]))
    return T


@pytest.mark.parametrize("theta,ncrit", [(0.5, 64), (0.8, 16), (0.3, 128)])
def test_structure_plummer(orc, theta, ncrit):
    x, m = synth.plummer(3000, synth.rng(0))
    _check_structure(orc, x, m, theta, ncrit)


def test_structure_uniform_and_duplicates(orc):
    x, m = synth.uniform_cube(2000, synth.rng(1))
    x[100:140] = x[7]          # 41 coincident particles: depth cap leaf
    T = _check_structure(orc, x, m, 0.6, 32)
    assert T.depth.max() == 21


def test_single_group_when_n_le_ncrit(orc):
    x, m = synth.plummer(50, synth.rng(0))
    T = orc.Tree(x, m, 0.5, 64)
    assert T.ngroups == 1 and T.n_jc == 0 and T.n_jp == 50


def test_theta_zero_is_direct_sum(orc):
    x, m = synth.plummer(2048, synth.rng(0))
    eps2 = (1 / 64) ** 2
    T = orc.Tree(x, m, 0.0, 64)
    assert T.n_jc == 0 and T.n_jp == T.ngroups * len(m)
    mat = orc.materialise(T, x, m)
    a, phi = orc.eval_lists(orc.QUAD, mat, x, eps2)
    ad, pd = orc.direct(x, m, eps2)
    np.testing.assert_allclose(a, ad, rtol=1e-12, atol=1e-13 * np.abs(ad).max())
    np.testing.assert_allclose(phi, pd, rtol=1e-13)


def test_direct_momentum_and_symmetry(orc):
    """Pairwise antisymmetry: sum_i m_i a_i = 0 for a common softening; a
    particle at the centre of a cube of equal masses feels no force."""
    x, m = synth.plummer(1500, synth.rng(0))
    a, _ = orc.direct(x, m, 0.01 ** 2)
    mom = (m[:, None] * a).sum(0)
    assert np.abs(mom).max() <= 1e-14 * (m[:, None] * np.abs(a)).sum()
    v = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1)
                  for sz in (-1, 1)], float) * 0.7
    xs = np.vstack([np.zeros((1, 3)), v])
    ms = np.array([3.0] + [1.0] * 8)
    a, phi = orc.direct(xs, ms, 0.2 ** 2)
    assert np.abs(a[0]).max() < 1e-15   # single terms are ~0.4
    assert phi[0] == pytest.approx(-8 / np.sqrt(3 * 0.49 + 0.04) - 3 / 0.2,
                                   rel=1e-14)


def _tree_errors(orc, x, m, eps2, thetas, ncrit, a_ref):
    out = {}
    for th in thetas:
        T = orc.Tree(x, m, th, ncrit)
        mat = orc.materialise(T, x, m)
        for kind, name in ((orc.MONO, "mono"), (orc.QUAD, "quad")):
            a, _ = orc.eval_lists(kind, mat, x, eps2)
            e = orc.relative_errors(a, a_ref)
            out[(name, th)] = (np.sqrt(np.mean(e ** 2)), np.percentile(e, 90))
    return out


@pytest.fixture(scope="module")
def sphere_errors(orc):
    x, m = synth.uniform_sphere(16384, synth.rng(7))
    eps2 = (1 / 64) ** 2
    ad, _ = orc.direct(x, m, eps2)
    thetas = (0.2, 0.3, 0.4, 0.5, 0.6, 0.7)
    return thetas, _tree_errors(orc, x, m, eps2, thetas, 64, ad)


def test_quad_beats_mono_at_equal_theta(sphere_errors):
    thetas, err = sphere_errors
    for th in (0.3, 0.5, 0.7):
        assert err[("quad", th)][0] < err[("mono", th)][0]
        assert err[("quad", th)][1] < err[("mono", th)][1]


def test_error_converges_as_theta_shrinks(sphere_errors):
    thetas, err = sphere_errors
    for name in ("mono", "quad"):
        e90 = [err[(name, th)][1] for th in thetas]
        assert all(e90[k] < e90[k + 1] for k in range(len(e90) - 1)), e90


def test_error_scaling_with_theta(sphere_errors):
    """Fig. 2 text: 90% errors ~ theta^(5/2) (mono) and theta^(7/2) (quad)."""
    with open(os.path.join(GOLDEN, "paper_claims.json")) as f:
        claims = json.load(f)["error_scaling"]
    thetas, err = sphere_errors
    lt = np.log(np.array(thetas))
    for name in ("mono", "quad"):
        le = np.log([err[(name, th)][1] for th in thetas])
        slope = np.polyfit(lt, le, 1)[0]
        assert abs(slope - claims[name]) <= claims["tolerance"], (name, slope)


def test_split_tree_theta_zero_is_short_range_direct(orc):
    """Periodic short-range kernel: with theta = 0 the tree lists (pruned at
    the cutoff, minimum image) reproduce the direct short-range sum."""
    x, m = synth.perturbed_lattice(16, synth.rng(4))
    rs = 1.25 / 16
    rcut = 4.5 * rs
    T = orc.Tree(x, m, 0.0, 32, box=1.0, rcut=rcut)
    mat = orc.materialise(T, x, m)
    a, p = orc.eval_lists(orc.SPLIT_QUAD, mat, x, 0.0, box=1.0, rs=rs, rcut=rcut)
    ad, pd = orc.direct(x, m, 0.0, split=True, box=1.0, rs=rs, rcut=rcut)
    np.testing.assert_allclose(a, ad, rtol=1e-12, atol=1e-13 * np.abs(ad).max())
    np.testing.assert_allclose(p, pd, rtol=1e-12)
    # pruning really happened: lists are shorter than N
    assert T.n_jp < T.ngroups * len(m)


def test_split_tree_quad_beats_mono(orc):
    x, m = synth.perturbed_lattice(16, synth.rng(4))
    rs = 1.25 / 16
    rcut = 4.5 * rs
    ad, _ = orc.direct(x, m, 0.0, split=True, box=1.0, rs=rs, rcut=rcut)
    T = orc.Tree(x, m, 0.5, 32, box=1.0, rcut=rcut)
    mat = orc.materialise(T, x, m)
    eq = orc.relative_errors(orc.eval_lists(orc.SPLIT_QUAD, mat, x, 0.0, box=1.0,
                                            rs=rs, rcut=rcut)[0], ad)
    em = orc.relative_errors(orc.eval_lists(orc.SPLIT_MONO, mat, x, 0.0, box=1.0,
                                            rs=rs, rcut=rcut)[0], ad)
    assert np.sqrt(np.mean(eq ** 2)) < 0.5 * np.sqrt(np.mean(em ** 2))


def test_split_tree_cutoff_pruning_is_exact(orc):
    """The cutoff only removes entries whose every pair is beyond rcut:
    lists built without it (the whole box walked, every accepted cell kept)
    give the same short-range forces as the pruned lists, bit for bit, and
    the pruned lists are much shorter.  This pins both the skip of cells
    whose cube is beyond rcut and the drop of accepted cells whose centre
    of mass is at least rcut from the group cube."""
    x, m = synth.perturbed_lattice(16, synth.rng(4))
    rs = 1.25 / 16
    rcut = 4.5 * rs
    kw = dict(box=1.0, rs=rs, rcut=rcut)
    full = orc.Tree(x, m, 0.5, 32, box=1.0, rcut=0.0)
    pruned = orc.Tree(x, m, 0.5, 32, box=1.0, rcut=rcut)
    for kind in (orc.SPLIT_QUAD, orc.SPLIT_MONO):
        a0, p0 = orc.eval_lists(kind, orc.materialise(full, x, m), x, 0.0, **kw)
        a1, p1 = orc.eval_lists(kind, orc.materialise(pruned, x, m), x, 0.0, **kw)
        assert np.array_equal(a0, a1) and np.array_equal(p0, p1)
    assert pruned.n_jc < 0.5 * full.n_jc
    # every kept cell has its centre of mass within rcut (1 + 2^-16) of the
    # group cube, and the full lists hold cells that the cube test alone
    # would keep but the centre-of-mass test drops
    def dist(T, com, g):
        d = np.abs(com - T.center[T.gnode[g]])
        d = np.minimum(d, 1.0 - d) - 0.5 * T.side[T.gnode[g]]
        return np.sqrt((np.maximum(d, 0) ** 2).sum(-1))

    def cube_dist(T, nodes, g):
        d = np.abs(T.center[nodes] - T.center[T.gnode[g]])
        d = np.minimum(d, 1.0 - d) - 0.5 * (T.side[nodes][:, None] + T.side[T.gnode[g]])
        return np.sqrt((np.maximum(d, 0) ** 2).sum(-1))

    rdrop = rcut * (1 + 2.0 ** -16)
    dropped = 0
    for g in range(0, pruned.ngroups, 5):
        kept = pruned.jc_node[pruned.jc_off[g]:pruned.jc_off[g + 1]]
        assert np.all(dist(pruned, pruned.com[kept], g) < rdrop)
        allc = full.jc_node[full.jc_off[g]:full.jc_off[g + 1]]
        dropped += np.sum((cube_dist(full, allc, g) <= rcut)
                          & (dist(full, full.com[allc], g) >= rdrop))
    assert dropped > 0
