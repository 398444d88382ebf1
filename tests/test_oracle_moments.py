"""Pins for the oracle's cell moments (Sec. 3 eqs. 2-3), CPU only:
tracelessness, the parallel-axis theorem, rotation covariance, and the
one-particle special case."""
import numpy as np

from paper_1812_07313_amd import synth


def _Q(q):
    return np.array([[q[0], q[1], q[2]], [q[1], q[3], q[4]], [q[2], q[4], q[5]]])


def test_traceless_and_symmetric_storage(orc):
    g = np.random.default_rng(1)
    for k in (2, 7, 100, 1000):
        x = g.normal(size=(k, 3)) * g.uniform(0.1, 10.0)
        m = g.uniform(0.1, 2.0, k)
        M, com, q, T = orc.moments(x, m)
        # eq. (3): q22 = -(q00 + q11); the oracle computes q22 directly
        assert abs(q[0] + q[3] + q[5]) <= 1e-13 * T
        np.testing.assert_allclose(M, m.sum(), rtol=1e-14)
        np.testing.assert_allclose(com, (m[:, None] * x).sum(0) / m.sum(),
                                   rtol=1e-12, atol=1e-14 * np.abs(x).max())


def test_single_particle_has_no_quadrupole(orc):
    M, com, q, T = orc.moments(np.array([[0.3, -2.0, 5.0]]), [1.7])
    assert M == 1.7
    np.testing.assert_array_equal(com, [0.3, -2.0, 5.0])
    assert np.all(q == 0.0) and T == 0.0


def test_parallel_axis_theorem(orc):
    """Q of a union = sum over parts of [Q_c + M_c (3 D D^T - |D|^2 1)],
    D = com_c - com_union (a textbook identity, not the oracle's formula)."""
    g = np.random.default_rng(2)
    parts = [(g.normal(size=(k, 3)) * s + c, g.uniform(0.5, 1.5, k))
             for k, s, c in ((13, 0.3, (1, 0, 0)), (29, 0.1, (0, 2, -1)),
                             (5, 0.7, (-1, -1, 3)))]
    x = np.concatenate([p[0] for p in parts])
    m = np.concatenate([p[1] for p in parts])
    M, com, q, T = orc.moments(x, m)
    Qsum = np.zeros((3, 3))
    Tsum = 0.0
    for xp, mp in parts:
        Mc, cc, qc, Tc = orc.moments(xp, mp)
        D = cc - com
        Qsum += _Q(qc) + Mc * (3 * np.outer(D, D) - D.dot(D) * np.eye(3))
        Tsum += Tc + Mc * D.dot(D)
    np.testing.assert_allclose(_Q(q), Qsum, rtol=1e-12, atol=1e-12 * T)
    assert T == np.float64(Tsum) or abs(T - Tsum) <= 1e-12 * T


def test_rotation_covariance(orc):
    g = np.random.default_rng(3)
    x = g.normal(size=(50, 3)) * np.array([2.0, 1.0, 0.3])
    m = g.uniform(0.5, 1.5, 50)
    A = g.normal(size=(3, 3))
    R, _ = np.linalg.qr(A)
    _, _, q, T = orc.moments(x, m)
    _, _, qr, Tr = orc.moments(x @ R.T, m)
    np.testing.assert_allclose(_Q(qr), R @ _Q(q) @ R.T, atol=1e-12 * T)
    assert Tr == np.float64(Tr) and abs(Tr - T) <= 1e-12 * T


def test_plummer_sphere_is_nearly_isotropic(orc):
    """A large isotropic sample has |Q| << T (sampling noise only)."""
    x, m = synth.plummer(20000, synth.rng(0))
    _, _, q, T = orc.moments(x, m)
    assert np.abs(_Q(q)).max() < 0.1 * T
