"""The product host list builder (libbhq, bhq_build_lists) against the
oracle's tree walk: same groups, same i-particle order, same j-particle
lists and the same j-cells (identified by their particle ranges), with
moments equal to rounding.  Two independent implementations of Sec. 1 and
Sec. 3.4.  (The two could in principle disagree on a cell whose opening
test l^2 < theta^2 d^2 is within rounding of equality, since their moments
are summed in different orders; none of these inputs has such a cell.)"""
import numpy as np
import pytest

from paper_1812_07313_amd import bhq, synth


def _compare(orc, x, m, theta, ncrit, box=0.0, rcut=0.0):
    T = orc.Tree(x, m, theta, ncrit, box=box, rcut=rcut)
    L = bhq.bhq_build_lists(x, m, theta, ncrit, box=box, rcut=rcut)
    try:
        P = bhq.bhq_lists_export(L, len(m))
        C = bhq.bhq_lists_cells(L)
    finally:
        bhq.bhq_lists_free(L)
    assert np.array_equal(P["i_idx"], T.perm)
    assert np.array_equal(P["i_off"], T.i_off)
    np.testing.assert_array_equal(P["center"], T.center[T.gnode])
    np.testing.assert_array_equal(P["side"], T.side[T.gnode])
    assert np.array_equal(P["jp_off"], T.jp_off)
    assert np.array_equal(P["jc_off"], T.jc_off)
    assert np.array_equal(P["jp_idx"], T.jp_idx)
    # j-cells: same cells in the same order (cell ids differ: the product
    # numbers cells breadth-first, the oracle depth-first), identified by
    # mass and centre of mass; moments agree to rounding (direct sums in
    # the oracle, parallel-axis shifts in the product)
    cp, co = P["jc_cell"], T.jc_node
    np.testing.assert_allclose(C["mass"][cp], T.mass[co], rtol=1e-13)
    np.testing.assert_allclose(C["com"][cp], T.com[co], rtol=1e-12, atol=1e-14)
    qs = np.abs(T.q[co]).max(axis=1, keepdims=True) + 1e-300
    np.testing.assert_allclose(C["q"][cp] / qs, T.q[co] / qs, rtol=0, atol=1e-10)
    np.testing.assert_allclose(C["trace"][cp], T.trace[co], rtol=1e-10)
    return T


def test_lists_match_oracle_plummer_16k(orc):
    c = synth.config_plummer_16k()
    _compare(orc, c["x"], c["m"], c["theta"], c["ncrit"])


@pytest.mark.parametrize("theta", [0.3, 0.7])
def test_lists_match_oracle_uniform_64k(orc, theta):
    x, m = synth.uniform_cube(1 << 16, synth.rng(1))
    _compare(orc, x, m, theta, 256)


def test_lists_match_oracle_clustered(orc):
    x, m = synth.clustered(1 << 15, synth.rng(2))
    _compare(orc, x, m, 0.5, 64)


def test_lists_match_oracle_periodic_cutoff(orc):
    x, m = synth.perturbed_lattice(24, synth.rng(4))
    rs = 1.25 / 24
    _compare(orc, x, m, 0.5, 32, box=1.0, rcut=4.5 * rs)


def test_batch_builder_matches_per_system_oracle(orc):
    """bhq_build_lists_batch: each system's groups and lists are the
    oracle's lists of that system alone, shifted to the concatenated
    indexing."""
    systems = synth.batched_plummer(7, lo=8.0, hi=11.0)
    sizes = [len(s[1]) for s in systems]
    off = np.concatenate([[0], np.cumsum(sizes)])
    X = np.concatenate([s[0] for s in systems])
    M = np.concatenate([s[1] for s in systems])
    L = bhq.bhq_build_lists_batch(off, X, M, 0.6, 64)
    try:
        P = bhq.bhq_lists_export(L, len(M))
        C = bhq.bhq_lists_cells(L)
    finally:
        bhq.bhq_lists_free(L)
    g0 = 0
    for s, (x, m, _) in enumerate(systems):
        T = orc.Tree(x, m, 0.6, 64)
        a = off[s]
        ng = T.ngroups
        assert np.array_equal(P["i_idx"][a:off[s + 1]], T.perm + a)
        assert np.array_equal(P["i_off"][g0:g0 + ng + 1] - a, T.i_off)
        jp0, jc0 = P["jp_off"][g0], P["jc_off"][g0]
        assert np.array_equal(P["jp_off"][g0:g0 + ng + 1] - jp0, T.jp_off)
        assert np.array_equal(P["jc_off"][g0:g0 + ng + 1] - jc0, T.jc_off)
        assert np.array_equal(P["jp_idx"][jp0:jp0 + T.n_jp] - a, T.jp_idx)
        cp = P["jc_cell"][jc0:jc0 + T.n_jc]
        np.testing.assert_allclose(C["mass"][cp], T.mass[T.jc_node], rtol=1e-13)
        np.testing.assert_allclose(C["com"][cp], T.com[T.jc_node], rtol=1e-12,
                                   atol=1e-14)
        g0 += ng
    assert g0 == len(P["i_off"]) - 1
