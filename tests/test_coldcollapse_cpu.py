"""Host logic of the cold-collapse runs (CPU only): the initial state, the
density profile and centre, and the run comparison."""
import numpy as np
import pytest

from paper_1812_07313_amd import coldcollapse as cc
from paper_1812_07313_amd import synth


def test_cold_sphere_initial_state():
    x, v, m = synth.cold_sphere(20000, synth.rng(5))
    r = np.sqrt((x * x).sum(1))
    assert r.max() <= 1.0 and m.sum() == pytest.approx(1.0)
    np.testing.assert_allclose(v.mean(0), 0.0, atol=1e-15)
    K = 0.5 * np.sum(m * (v * v).sum(1))
    assert 2 * K / 0.6 == pytest.approx(0.1, rel=1e-12)
    # uniform in the ball: the enclosed mass grows as r^3
    assert np.mean(r < 0.5) == pytest.approx(0.125, abs=0.01)


def test_density_profile_and_centre():
    g = np.random.default_rng(3)
    x, m = synth.uniform_sphere(200000, g)
    shift = np.array([0.3, -0.2, 0.1])
    c = cc.density_centre(x + shift, m)
    np.testing.assert_allclose(c, shift, atol=0.05)
    p = cc.density_profile(x, m, np.zeros(3), rmin=0.1, rmax=2.0, nbins=10)
    rho = np.array(p["rho"])
    # shells inside the sphere holding enough particles for a 5 % check
    inside = (np.array(p["r"]) < 0.9) & (np.array(p["count"]) >= 4000)
    assert inside.sum() >= 4
    np.testing.assert_allclose(rho[inside], 3.0 / (4.0 * np.pi), rtol=0.05)
    assert np.all(rho[np.array(p["r"]) > 1.05] == 0.0)
    r = np.sqrt((x * x).sum(1))
    assert sum(p["count"]) == np.sum((r >= 0.1) & (r < 2.0))


def test_compare_runs():
    prof = dict(r=[0.1, 1.0], rho=[10.0, 1.0], count=[500, 50])
    prof2 = dict(r=[0.1, 1.0], rho=[20.0, 5.0], count=[500, 500])
    res = {"A": dict(profile=prof), "B": dict(profile=prof2)}
    out = cc.compare(res)
    assert out["A"]["max_abs_log10_ratio"] == 0.0
    assert out["B"]["max_abs_log10_ratio"] == pytest.approx(np.log10(2.0))
    assert out["B"]["shells"] == 1
