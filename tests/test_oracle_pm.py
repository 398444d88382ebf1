"""Pins for the particle-mesh long-range reference (CPU only).

The wave-vector sum that defines the periodic long-range force is tied to
the isolated long-range kernel -erf(r / 2 r_s) / r near a point mass (plus
the uniform background that the k = 0 mode removes, whose field is
+4 pi m r / (3 L^3); the images' tidal field vanishes by cubic symmetry),
and the particle-mesh evaluation is tied to that sum: its error is at the
level expected of TSC at r_s = 1.25 mesh spacings and falls as the mesh is
refined at fixed r_s; the mesh evaluation is linear in the masses."""
import math

import numpy as np
import pytest
from scipy import special

from oracle import pm


def _isolated(r_vec, m, rs, L):
    r = np.linalg.norm(r_vec, axis=1)
    f = m * (np.exp(-r * r / (4 * rs * rs)) / (rs * math.sqrt(math.pi) * r)
             - special.erf(r / (2 * rs)) / r ** 2)
    a = f[:, None] * r_vec / r[:, None]
    a += 4.0 * math.pi * m / (3.0 * L ** 3) * r_vec
    return a, -m * special.erf(r / (2 * rs)) / r


def test_k_sum_near_a_point_mass():
    L, rs, m = 1.0, 0.02, 0.8
    xp = np.array([[0.5, 0.5, 0.5]])
    g = np.random.default_rng(4)
    u = g.normal(size=(40, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    r_vec = u * g.uniform(0.01, 0.08, 40)[:, None]
    a, phi = pm.direct_k_sum(xp + r_vec, xp, [m], L, rs)
    a_iso, phi_iso = _isolated(r_vec, m, rs, L)
    err = np.linalg.norm(a - a_iso, axis=1) / np.linalg.norm(a_iso, axis=1)
    assert err.max() < 2e-4, err.max()
    # potentials agree up to one constant (images and background)
    dphi = (phi - phi_iso) - (phi - phi_iso).mean()
    assert np.abs(dphi).max() < 1e-3 * np.abs(phi_iso).max()


def _pm_error(n, rs, seed=1, deconvolve=True):
    L = 1.0
    g = np.random.default_rng(seed)
    xp = g.random((1, 3))
    pts = (xp + g.normal(size=(60, 3)) * 4 * rs) % 1.0
    a_pm, _ = pm.pm(np.vstack([xp, pts]), np.concatenate([[1.0], np.zeros(60)]), L, n, rs,
                    deconvolve=deconvolve)
    a_ex, _ = pm.direct_k_sum(pts, xp, [1.0], L, rs)
    e = np.linalg.norm(a_pm[1:] - a_ex, axis=1) / np.linalg.norm(a_ex, axis=1)
    return math.sqrt((e * e).mean())


def test_pm_against_k_sum_and_refinement():
    rs = 1.25 / 32
    e32 = _pm_error(32, rs)
    e64 = _pm_error(64, rs)
    assert e32 < 1e-2, e32
    assert e64 < e32 / 4, (e32, e64)
    assert _pm_error(32, rs, deconvolve=False) > e32


def test_pm_linear_in_mass():
    g = np.random.default_rng(7)
    x = g.random((30, 3))
    m1 = g.random(30)
    m2 = g.random(30)
    a1, p1 = pm.pm(x, m1, 1.0, 16, 0.08)
    a2, p2 = pm.pm(x, m2, 1.0, 16, 0.08)
    a3, p3 = pm.pm(x, m1 + 2.0 * m2, 1.0, 16, 0.08)
    np.testing.assert_allclose(a3, a1 + 2.0 * a2, rtol=1e-10, atol=1e-12 * np.abs(a3).max())
    np.testing.assert_allclose(p3, p1 + 2.0 * p2, rtol=1e-10, atol=1e-12 * np.abs(p3).max())


def test_tsc_weights_partition_of_unity():
    x = np.random.default_rng(2).random((1000, 3))
    i0, w = pm.tsc_weights(x, 1.0 / 16, 16)
    np.testing.assert_allclose(w.sum(0), 1.0, rtol=1e-15)
    assert np.all(w >= 0) and np.all((i0 >= 0) & (i0 < 16))
    # first moment: sum_o w_o (i0 + o) h = x (TSC reproduces linear functions)
    h = 1.0 / 16
    pos = sum(w[o] * ((np.floor(x / h + 0.5) + o - 1) * h) for o in range(3))
    np.testing.assert_allclose(pos, x, atol=1e-15)
