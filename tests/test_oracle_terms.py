"""Pins for the oracle's single-interaction terms (CPU only).

Each check ties the oracle to something other than itself: hand-derived
closed forms (tests/golden/closed_forms.json), a = -grad phi by central
differences (Sec. 3 eq. 6), the order of accuracy of a second-order
multipole expansion, and library special functions (scipy) for the split
kernel.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import special

from conftest import GOLDEN


def _fixture():
    with open(os.path.join(GOLDEN, "closed_forms.json")) as f:
        return json.load(f)


def test_two_body_closed_form(orc):
    fx = _fixture()["two_body"]
    x = np.array(fx["x"])
    m = np.array(fx["m"])
    a, phi = orc.direct(x, m, fx["eps"] ** 2)
    np.testing.assert_allclose(a, np.array(fx["a"]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(phi, np.array(fx["phi"]), rtol=1e-15)


def test_axis_pair_moments_and_expansion(orc):
    fx = _fixture()["axis_pair"]
    s, mm, D = fx["s"], fx["m"], fx["D"]
    x = np.array([[0.0, 0.0, s], [0.0, 0.0, -s]])
    M, com, q, T = orc.moments(x, [mm, mm])
    assert M == 2 * mm
    np.testing.assert_allclose(com, 0.0, atol=1e-17)
    np.testing.assert_allclose(q, fx["Q"], rtol=1e-14, atol=1e-17)
    assert T == pytest.approx(fx["T"], rel=1e-14)
    # on the axis: field point (0, 0, D), d = com - r_i
    a, phi = orc.pc_quad(np.array([0.0, 0.0, -D]), M, q, 0.0)
    assert phi == pytest.approx(fx["axis_phi"], rel=1e-14)
    np.testing.assert_allclose(a, fx["axis_a"], rtol=1e-14, atol=1e-16)
    # the residual against the exact two-body potential is the hexadecapole
    exact = fx["axis_exact_phi"]
    assert (exact - phi) == pytest.approx(fx["axis_residual_leading"], rel=0.05)
    # in the plane: field point (D, 0, 0)
    a, phi = orc.pc_quad(np.array([-D, 0.0, 0.0]), M, q, 0.0)
    assert phi == pytest.approx(fx["plane_phi"], rel=1e-14)
    np.testing.assert_allclose(a, fx["plane_a"], rtol=1e-14, atol=1e-16)
    assert abs(fx["plane_exact_phi"] - phi) < 5e-6


def test_monopole_cell_is_point_mass(orc):
    d = np.array([0.3, -1.2, 0.7])
    a1, p1 = orc.pc_mono(d, 2.5, 0.01)
    a2, p2 = orc.pp_plummer(d, 2.5, 0.01)
    assert np.array_equal(a1, a2) and p1 == p2
    # a zero quadrupole reduces the quad term to the monopole term
    a3, p3 = orc.pc_quad(d, 2.5, np.zeros(6), 0.01)
    np.testing.assert_allclose(a3, a1, rtol=1e-15)
    assert p3 == pytest.approx(p1, rel=1e-15)


def _num_grad(f, x0, h):
    g = np.zeros(3)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        g[k] = (f(x0 + e) - f(x0 - e)) / (2 * h)
    return g


@pytest.mark.parametrize("eps2", [0.0, 0.04])
def test_quad_force_is_minus_gradient(orc, eps2):
    """a = -grad_i phi (eq. 6); the field point moves, d = com - x_i."""
    g = np.random.default_rng(5)
    for _ in range(20):
        q = g.normal(size=6)
        q[5] = -(q[0] + q[3])
        com = g.normal(size=3) * 2.0
        xi = g.normal(size=3) * 0.3
        M = g.uniform(0.5, 2.0)

        def phi_at(xp):
            return orc.pc_quad(com - xp, M, q, eps2)[1]

        a, _ = orc.pc_quad(com - xi, M, q, eps2)
        np.testing.assert_allclose(a, -_num_grad(phi_at, xi, 1e-5),
                                   rtol=1e-7, atol=1e-9 * np.abs(a).max())


def _cluster(g, k, scale):
    x = g.normal(size=(k, 3)) * scale * np.array([1.0, 0.6, 0.35])
    m = g.uniform(0.5, 1.5, k)
    return x, m


def test_expansion_order(orc):
    """Error of a second-order (quadrupole) cell expansion falls as (l/D)^3,
    of a monopole as (l/D)^2, against summing the cell's particles
    (direct pair terms, themselves pinned by the closed forms)."""
    g = np.random.default_rng(11)
    xc, mc = _cluster(g, 40, 1.0)
    xi = np.array([7.0, 3.0, -5.0])
    err_q, err_m = [], []
    for scale in (0.4, 0.2, 0.1, 0.05):
        x = xc * scale
        M, com, q, _ = orc.moments(x, mc)
        a_ex = np.zeros(3)
        for p in range(len(mc)):
            a_ex += orc.pp_plummer(x[p] - xi, mc[p], 0.0)[0]
        aq, _ = orc.pc_quad(com - xi, M, q, 0.0)
        am, _ = orc.pc_mono(com - xi, M, 0.0)
        err_q.append(np.linalg.norm(aq - a_ex) / np.linalg.norm(a_ex))
        err_m.append(np.linalg.norm(am - a_ex) / np.linalg.norm(a_ex))
    rq = np.array(err_q[:-1]) / np.array(err_q[1:])
    rm = np.array(err_m[:-1]) / np.array(err_m[1:])
    assert np.all((rq > 6.5) & (rq < 10.0)), rq
    assert np.all((rm > 3.3) & (rm < 4.8)), rm
    assert np.all(np.array(err_q) < np.array(err_m))


def test_split_kernel_library_values(orc):
    """Phi(r) = -erfc(r/2rs)/r (scipy's erfc), and the radial derivative
    functions against numerical derivatives of Phi."""
    rs = 0.01
    for r in (0.002, 0.01, 0.02, 0.04):
        Phi, D1, D2, D3 = orc.split_derivs(r, rs)
        assert Phi == pytest.approx(-special.erfc(r / (2 * rs)) / r, rel=1e-14)
        h = r * 1e-4

        def fPhi(t):
            return orc.split_derivs(t, rs)[0]

        def fD1(t):
            return orc.split_derivs(t, rs)[1]

        def fD2(t):
            return orc.split_derivs(t, rs)[2]

        assert D1 == pytest.approx((fPhi(r + h) - fPhi(r - h)) / (2 * h) / r,
                                   rel=1e-6)
        assert D2 == pytest.approx((fD1(r + h) - fD1(r - h)) / (2 * h) / r,
                                   rel=1e-6)
        assert D3 == pytest.approx((fD2(r + h) - fD2(r - h)) / (2 * h) / r,
                                   rel=1e-6)


def test_split_kernel_newtonian_limit(orc):
    """rs -> infinity: Phi = -1/r, D1 = r^-3, D2 = -3 r^-5, D3 = 15 r^-7."""
    r = 0.37
    Phi, D1, D2, D3 = orc.split_derivs(r, 1e9)
    assert Phi == pytest.approx(-1 / r, rel=1e-8)
    assert D1 == pytest.approx(r ** -3, rel=1e-8)
    assert D2 == pytest.approx(-3 * r ** -5, rel=1e-8)
    assert D3 == pytest.approx(15 * r ** -7, rel=1e-8)
    # g(0) = 1: the split pair force tends to the Newtonian one as r -> 0
    r = 1e-6
    _, D1, _, _ = orc.split_derivs(r, 1.0)
    assert D1 * r ** 3 == pytest.approx(1.0, rel=1e-9)


def test_split_cell_order_and_gradient(orc):
    """Split cell term (with the trace T): force = -grad phi, third-order
    accuracy against summing the cell's particles with the split pair
    kernel, cutoff masking."""
    g = np.random.default_rng(3)
    rs, rcut = 0.02, 0.09
    xc, mc = _cluster(g, 30, 1.0)
    xi = np.array([0.05, -0.02, 0.03])
    errs = []
    for scale in (0.004, 0.002, 0.001):
        x = xc * scale
        M, com, q, T = orc.moments(x, mc)
        a_ex = np.zeros(3)
        for p in range(len(mc)):
            a_ex += orc.pp_split(x[p] - xi, mc[p], rs, rcut)[0]
        a, _ = orc.pc_split(com - xi, M, q, T, rs, rcut, True)
        errs.append(np.linalg.norm(a - a_ex) / np.linalg.norm(a_ex))

        def phi_at(xp):
            return orc.pc_split(com - xp, M, q, T, rs, rcut, True)[1]

        np.testing.assert_allclose(a, -_num_grad(phi_at, xi, 1e-6), rtol=1e-6)
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 6.5), ratios
    # beyond the cutoff, nothing
    a, phi = orc.pc_split(np.array([rcut * 1.01, 0, 0]), 1.0, np.zeros(6), 0.0,
                          rs, rcut, True)
    assert phi == 0.0 and np.all(a == 0.0)
    a, phi = orc.pp_split(np.zeros(3), 1.0, rs, rcut)
    assert phi == 0.0 and np.all(a == 0.0)


def test_split_pair_gradient(orc):
    rs, rcut = 0.01, 0.045
    d = np.array([0.011, -0.004, 0.006])
    a, _ = orc.pp_split(d, 1.3, rs, rcut)

    def phi_at(xp):
        return orc.pp_split(d - xp, 1.3, rs, rcut)[1]

    np.testing.assert_allclose(a, -_num_grad(phi_at, np.zeros(3), 1e-7),
                               rtol=1e-6)
    assert math.isfinite(a[0])


def test_split_cutoff_decision_modes(orc):
    """The cutoff decision taken from FP64 offsets to a group centre agrees
    with the definition (FP64, absolute separations) everywhere except
    within rounding of r = rcut; the self pair is always excluded."""
    g = np.random.default_rng(21)
    rcut, box = 0.02, 1.0
    c = np.array([0.51, 0.49, 0.502])
    agree = 0
    for _ in range(4000):
        xi = c + g.uniform(-0.01, 0.01, 3)
        xj = xi + g.normal(size=3) * 0.015
        xj = np.mod(xj, 1.0)
        d = xj - xi
        d -= np.rint(d)
        r = np.linalg.norm(d)
        modes = [orc.split_keep(mm, xj, xi, c, box, rcut)
                 for mm in (orc.MASK_ABS, orc.MASK_F64_OFS)]
        assert modes[0] == (r < rcut)
        if abs(r - rcut) > 1e-12 * rcut:
            assert modes[0] == modes[1]
            agree += 1
    assert agree > 3990
    for mm in (orc.MASK_ABS, orc.MASK_F64_OFS):
        assert not orc.split_keep(mm, c, c, c, box, rcut)
    # just inside / outside the cutoff along an axis, far from rounding
    xi = c.copy()
    for frac, keep in ((0.999, True), (1.001, False)):
        xj = xi + np.array([rcut * frac, 0, 0])
        for mm in (orc.MASK_ABS, orc.MASK_F64_OFS):
            assert orc.split_keep(mm, xj, xi, c, box, rcut) == keep
    # minimum image across the periodic boundary
    xi = np.array([0.999, 0.5, 0.5])
    xj = np.array([0.004, 0.5, 0.5])
    for mm in (orc.MASK_ABS, orc.MASK_F64_OFS):
        assert orc.split_keep(mm, xj, xi, np.array([0.995, 0.5, 0.5]), box, rcut)


def test_mask_flips_counts_disagreements(orc):
    """mask_flips counts exactly the terms on which the two decisions
    differ: a pair placed within an ulp of the cutoff, where they can
    disagree, is found by search and counted once (in both directions of
    the pair list); lists far from the cutoff give zero."""
    g = np.random.default_rng(5)
    rcut, box = 0.0215, 1.0
    found = None
    for _ in range(20000):
        xi = g.uniform(0.3, 0.7, 3)
        u = g.normal(size=3)
        u /= np.linalg.norm(u)
        xj = xi + rcut * u * (1.0 + g.uniform(-4e-16, 4e-16))
        c = xi + g.uniform(-0.01, 0.01, 3)
        if orc.split_keep(orc.MASK_ABS, xj, xi, c, box, rcut) != \
                orc.split_keep(orc.MASK_F64_OFS, xj, xi, c, box, rcut):
            found = (xi, xj, c)
            break
    assert found is not None
    xi, xj, c = found
    x = np.array([xi, xj])
    mat = dict(i_idx=np.array([0], np.int64), i_off=np.array([0, 1], np.int64),
               jp_off=np.array([0, 2], np.int64), jp_x=x.copy(),
               jc_off=np.array([0, 0], np.int64), jc_x=np.zeros((0, 3)),
               gcenter=c.reshape(1, 3))
    assert orc.mask_flips(mat, x, box, rcut) == 1
    mat["jp_x"] = np.array([xi, xi + np.array([0.5 * rcut, 0, 0])])
    assert orc.mask_flips(mat, x, box, rcut) == 0


def test_count_keep_brute_force(orc):
    """count_keep equals a numpy count of 0 < |d| < rcut over every (i, entry)
    pair of small lists (minimum image in the unit box)."""
    g = np.random.default_rng(8)
    x = g.uniform(0, 1, (3000, 3))
    m = np.full(3000, 1.0 / 3000)
    rcut = 0.2
    T = orc.Tree(x, m, 0.8, 16, box=1.0, rcut=rcut)
    mat = orc.materialise(T, x, m)
    want = [0, 0]
    for gi in range(len(mat["i_off"]) - 1):
        xi = x[mat["i_idx"][mat["i_off"][gi]:mat["i_off"][gi + 1]]]
        for k, key in ((0, "jp"), (1, "jc")):
            xj = mat[key + "_x"][mat[key + "_off"][gi]:mat[key + "_off"][gi + 1]]
            d = xj[None, :, :] - xi[:, None, :]
            d -= np.rint(d)
            r = np.sqrt((d * d).sum(2))
            want[k] += int(((r > 0) & (r < rcut)).sum())
    assert orc.count_keep(mat, x, 1.0, rcut) == tuple(want)
    assert want[0] > 0 and want[1] > 0


# --- the complete softened quadrupole (with the trace term) ---------------------

def test_soft_quad_limits(orc):
    """T = 0 gives eq. (1) exactly (orc_pc_quad); eps = 0 makes the trace
    term vanish for any T (the unsoftened potential is harmonic)."""
    g = np.random.default_rng(31)
    for _ in range(20):
        d = g.normal(size=3)
        q = g.normal(size=6)
        q[5] = -(q[0] + q[3])
        M, T, e2 = g.uniform(0.5, 2), g.uniform(0.1, 1), g.uniform(0.01, 0.5)
        a1, p1 = orc.pc_quad_soft(d, M, q, 0.0, e2)
        a2, p2 = orc.pc_quad(d, M, q, e2)
        np.testing.assert_allclose(a1, a2, rtol=1e-14, atol=1e-16)
        assert p1 == pytest.approx(p2, rel=1e-14)
        a1, p1 = orc.pc_quad_soft(d, M, q, T, 0.0)
        a2, p2 = orc.pc_quad(d, M, q, 0.0)
        np.testing.assert_allclose(a1, a2, rtol=1e-12, atol=1e-14)
        assert p1 == pytest.approx(p2, rel=1e-12)


def test_soft_quad_minus_gradient(orc):
    g = np.random.default_rng(32)
    for _ in range(20):
        q = g.normal(size=6)
        q[5] = -(q[0] + q[3])
        com = g.normal(size=3) * 2.0
        xi = g.normal(size=3) * 0.3
        M, T, e2 = g.uniform(0.5, 2.0), g.uniform(0.1, 1.0), g.uniform(0.05, 1.0)

        def phi_at(xp):
            return orc.pc_quad_soft(com - xp, M, q, T, e2)[1]

        a, _ = orc.pc_quad_soft(com - xi, M, q, T, e2)
        np.testing.assert_allclose(a, -_num_grad(phi_at, xi, 1e-5), rtol=1e-7,
                                   atol=1e-9 * np.abs(a).max())


@pytest.mark.parametrize("where", ["plane", "axis"])
def test_soft_quad_axis_pair_closed_form(orc, where):
    """Two masses m at +-s on the z axis, softening eps, field point at
    distance D in the plane or on the axis.  The exact softened two-body
    potential expands as -2m/rhat + m s^2 (eps^2 - 2 D^2)/rhat^5 on the axis
    and -2m/rhat + m s^2/rhat^3 in the plane (hand Taylor expansion in s,
    rhat^2 = D^2 + eps^2), so the complete expansion leaves an O(s^4)
    residual, while the traceless one misses m s^2 eps^2 / rhat^5."""
    m, D, eps = 0.7, 1.0, 0.5
    rhat = math.sqrt(D * D + eps * eps)
    res_soft, res_tl = [], []
    for s in (0.1, 0.05, 0.025):
        x = np.array([[0.0, 0.0, s], [0.0, 0.0, -s]])
        M, com, q, T = orc.moments(x, [m, m])
        if where == "plane":
            xi = np.array([D, 0.0, 0.0])
            closed = -2 * m / rhat + m * s * s / rhat ** 3
        else:
            xi = np.array([0.0, 0.0, D])
            closed = -2 * m / rhat + m * s * s * (eps * eps - 2 * D * D) / rhat ** 5
        exact = -m / np.linalg.norm(np.append(x[0] - xi, eps)) \
            - m / np.linalg.norm(np.append(x[1] - xi, eps))
        _, p_soft = orc.pc_quad_soft(com - xi, M, q, T, eps * eps)
        _, p_tl = orc.pc_quad(com - xi, M, q, eps * eps)
        assert p_soft == pytest.approx(closed, rel=1e-13)
        assert (p_soft - p_tl) == pytest.approx(m * s * s * eps * eps / rhat ** 5, rel=1e-9)
        res_soft.append(abs(exact - p_soft))
        res_tl.append(abs(exact - p_tl))
    r_soft = np.array(res_soft[:-1]) / np.array(res_soft[1:])
    r_tl = np.array(res_tl[:-1]) / np.array(res_tl[1:])
    assert np.all((r_soft > 14) & (r_soft < 18)), r_soft      # O(s^4)
    assert np.all((r_tl > 3.5) & (r_tl < 4.5)), r_tl          # O(s^2)


def test_soft_quad_expansion_order(orc):
    """Against summing a cluster's particles with the softened pair kernel
    at eps comparable to the distance: the complete expansion's error falls
    as (l/D)^3, the traceless one's as (l/D)^2."""
    g = np.random.default_rng(33)
    xc, mc = _cluster(g, 40, 1.0)
    xi = np.array([2.0, 1.0, -1.5])
    eps2 = 1.5
    err_s, err_t = [], []
    for scale in (0.2, 0.1, 0.05, 0.025):
        x = xc * scale
        M, com, q, T = orc.moments(x, mc)
        a_ex = np.zeros(3)
        for p in range(len(mc)):
            a_ex += orc.pp_plummer(x[p] - xi, mc[p], eps2)[0]
        a_s, _ = orc.pc_quad_soft(com - xi, M, q, T, eps2)
        a_t, _ = orc.pc_quad(com - xi, M, q, eps2)
        err_s.append(np.linalg.norm(a_s - a_ex) / np.linalg.norm(a_ex))
        err_t.append(np.linalg.norm(a_t - a_ex) / np.linalg.norm(a_ex))
    rs = np.array(err_s[:-1]) / np.array(err_s[1:])
    rt = np.array(err_t[:-1]) / np.array(err_t[1:])
    assert np.all((rs > 6.5) & (rs < 10.0)), rs
    assert np.all((rt > 3.3) & (rt < 4.8)), rt
    assert np.all(np.array(err_s) < np.array(err_t))
