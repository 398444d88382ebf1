"""Pins for the oracle's leapfrog (CPU only): time reversibility (a wrong
kick/drift order or sign breaks it), second-order convergence on a
two-body circular orbit whose period is known in closed form, and bounded
energy error."""
import math

import numpy as np


def _plummer_small(n, seed):
    g = np.random.default_rng(seed)
    r = 1.0 / np.sqrt(g.uniform(0.05, 0.95, n) ** (-2.0 / 3.0) - 1.0)
    u = g.normal(size=(n, 3))
    x = r[:, None] * u / np.linalg.norm(u, axis=1)[:, None]
    v = g.normal(size=(n, 3)) * 0.3
    return x, v, np.full(n, 1.0 / n)


def test_time_reversible(orc):
    x0, v0, m = _plummer_small(200, 41)
    x1, v1, _, _ = orc.leapfrog(x0, v0, m, 0.05, 0.01, 20, 0.5, 16)
    x2, v2, _, _ = orc.leapfrog(x1, -v1, m, 0.05, 0.01, 20, 0.5, 16)
    assert np.abs(x1 - x0).max() > 1e-3             # it moved
    np.testing.assert_allclose(x2, x0, rtol=0, atol=1e-11)
    np.testing.assert_allclose(-v2, v0, rtol=0, atol=1e-11)


def test_two_body_period_second_order(orc):
    """Equal masses 1/2 at +-1/2 on a circle: separation 1, total mass 1,
    so the period is 2 pi (Kepler) and each moves at speed 1/2.  After one
    period the error falls by 4 when dt halves."""
    x0 = np.array([[0.5, 0.0, 0.0], [-0.5, 0.0, 0.0]])
    v0 = np.array([[0.0, 0.5, 0.0], [0.0, -0.5, 0.0]])
    m = np.array([0.5, 0.5])
    errs = []
    for nstep in (200, 400, 800):
        dt = 2.0 * math.pi / nstep
        x, v, _, _ = orc.leapfrog(x0, v0, m, 1e-5, dt, nstep, 0.0, 8)
        errs.append(np.abs(x - x0).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert errs[0] < 1e-2
    assert np.all((ratios > 3.6) & (ratios < 4.4)), ratios


def test_energy_bounded(orc):
    x, v, m = _plummer_small(300, 42)
    eps = 0.05
    xs, vs, _, phi0 = orc.leapfrog(x, v, m, eps, 0.005, 0, 0.5, 16)

    def energy(xx, vv, phi):
        return 0.5 * np.sum(m * (vv ** 2).sum(1)) + 0.5 * np.sum(m * (phi + m / eps))

    e0 = energy(xs, vs, phi0)
    x1, v1, _, phi1 = orc.leapfrog(x, v, m, eps, 0.005, 100, 0.5, 16)
    assert abs(energy(x1, v1, phi1) - e0) < 2e-3 * abs(e0)


def test_periodic_wrap_and_split_reversible(orc):
    """Periodic TreePM leapfrog (split tree + PM): reversible, and positions
    stay in [0, box)."""
    g = np.random.default_rng(43)
    x = g.random((300, 3))
    v = g.normal(size=(300, 3)) * 0.3
    m = np.full(300, 1.0 / 300)
    rs = 1.25 / 16
    kw = dict(box=1.0, rs=rs, rcut=4.5 * rs, pm_mesh=16, kind=orc.SPLIT_QUAD)
    x1, v1, _, _ = orc.leapfrog(x, v, m, 0.0, 0.01, 10, 0.5, 16, **kw)
    assert np.all((x1 >= 0) & (x1 < 1))
    x2, v2, _, _ = orc.leapfrog(x1, -v1, m, 0.0, 0.01, 10, 0.5, 16, **kw)
    d = np.abs(x2 - x)
    d = np.minimum(d, 1.0 - d)
    assert d.max() < 1e-11 and np.abs(-v2 - v).max() < 1e-11
