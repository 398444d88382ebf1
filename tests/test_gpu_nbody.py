"""GPU: leapfrog time integration (device lists + forces + kick/drift every
step) against the oracle's leapfrog over its own tree forces, and the
time-step helpers of the C ABI against plain arithmetic on the host."""
import ctypes

import numpy as np
import pytest

import oracle as orc
from _parity import log
from paper_1812_07313_amd import bhq, synth
from paper_1812_07313_amd.nbody import NBody

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ic(n, seed):
    return synth.cold_sphere(n, synth.rng(5, seed))


@pytest.mark.parametrize("kernel,okind", [(bhq.QUAD, orc.QUAD), (bhq.MONO, orc.MONO),
                                          (bhq.QUAD_SOFT, orc.QUAD_SOFT)])
def test_leapfrog_fp64_matches_oracle(kernel, okind):
    """FP64 path, 8 steps of dt = 2^-8 on a cold sphere of 3000 particles:
    positions and velocities agree with the oracle's leapfrog to the
    summation-order level (the lists are identical at every step)."""
    x, v, m = _ic(3000, 1)
    eps, theta, ncrit, dt, steps = 2.0 ** -6, 0.5, 64, 2.0 ** -8, 8
    log("case leapfrog fp64 %s" % bhq.KERNEL_NAMES[kernel])
    xr, vr, ar, pr = orc.leapfrog(x, v, m, eps, dt, steps, theta, ncrit, kind=okind)
    with NBody(x, v, m, eps, theta, ncrit, kernel=kernel, precision=bhq.FP64) as sim:
        sim.step(dt, steps)
        xg, vg = sim.state()
        ag = sim.a.cpu().numpy()
        pg = sim.pot.cpu().numpy()
    dx = np.abs(xg - xr).max()
    dv = np.abs(vg - vr).max()
    log("  max |dx| %.3g  max |dv| %.3g" % (dx, dv))
    assert dx < 1e-12 and dv < 1e-12
    err = orc.relative_errors(ag, ar)
    assert err.max() < 1e-10
    np.testing.assert_allclose(pg, pr, rtol=1e-10)


def test_leapfrog_fp32_close_to_oracle():
    """FP32 path: after 8 steps the trajectories stay within the FP32
    force error times the elapsed time squared."""
    x, v, m = _ic(3000, 2)
    eps, theta, ncrit, dt, steps = 2.0 ** -6, 0.5, 64, 2.0 ** -8, 8
    xr, vr, _, _ = orc.leapfrog(x, v, m, eps, dt, steps, theta, ncrit)
    with NBody(x, v, m, eps, theta, ncrit) as sim:
        sim.step(dt, steps)
        xg, vg = sim.state()
    dx = np.abs(xg - xr).max()
    dv = np.abs(vg - vr).max()
    log("case leapfrog fp32: max |dx| %.3g  max |dv| %.3g" % (dx, dv))
    assert dx < 1e-7 and dv < 1e-5


def test_step_helpers_match_host_arithmetic():
    """get_result_device = get_result scattered to input order (bitwise);
    kick_drift = v + dtk a, x + dtd v in plain FP64 (bitwise); energies =
    the host sums to rounding."""
    x, v, m = _ic(5000, 3)
    eps = 2.0 ** -6
    with NBody(x, v, m, eps, 0.6, 64) as sim:
        sim.forces()
        a_tree, p_tree = bhq.bhq_get_result(sim.ctx, len(m))
        idx = bhq.bhq_get_lists(sim.ctx, len(m))["i_idx"]
        a_in = np.zeros_like(a_tree)
        p_in = np.zeros_like(p_tree)
        a_in[idx] = a_tree
        p_in[idx] = p_tree
        torch.cuda.synchronize()
        assert np.array_equal(sim.a.cpu().numpy(), a_in)
        assert np.array_equal(sim.pot.cpu().numpy(), p_in)
        K, W = sim.energies()
        Kh = 0.5 * np.sum(m * (v * v).sum(1))
        Wh = 0.5 * np.sum(m * (p_in + m / eps))
        assert K == pytest.approx(Kh, rel=1e-13)
        assert W == pytest.approx(Wh, rel=1e-13)
        # initial virial ratio of the cold sphere, |W| near 3/5
        log("case cold sphere: 2K/|W| = %.4f, W = %.4f" % (2 * K / abs(W), W))
        assert 0.09 < 2 * K / abs(W) < 0.11
        x0, v0 = sim.state()
        a0 = sim.a.cpu().numpy()
        bhq.bhq_kick_drift(sim.ctx, sim.x, sim.v, sim.a, 0.3, 0.7)
        x1, v1 = sim.state()
        vv = v0 + 0.3 * a0
        assert np.array_equal(v1, vv)
        assert np.array_equal(x1, x0 + 0.7 * vv)
        bhq.bhq_kick_drift(sim.ctx, None, sim.v, sim.a, -0.3, 0.0)
        x2, v2 = sim.state()
        assert np.array_equal(x2, x1) and np.array_equal(v2, vv + (-0.3) * a0)


def test_energy_conservation_short_run():
    """Cold sphere, 2^14 particles, 128 steps of 2^-8 (half a free-fall
    time): the FP32 path conserves energy to a few 1e-4."""
    x, v, m = _ic(1 << 14, 4)
    eps = 2.0 ** -7
    with NBody(x, v, m, eps, 0.5, 64) as sim:
        K0, W0 = sim.energies()
        sim.step(2.0 ** -8, 128)
        K1, W1 = sim.energies()
    e0, e1 = K0 + W0, K1 + W1
    log("case energy: E0 %.6f E1 %.6f rel %.3g (K %.4f -> %.4f)"
        % (e0, e1, abs(e1 - e0) / abs(e0), K0, K1))
    assert K1 > 2 * K0                       # it is collapsing
    assert abs(e1 - e0) < 5e-4 * abs(e0)


def test_step_helper_errors():
    x, v, m = _ic(100, 5)
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        a = torch.zeros((100, 3), dtype=torch.float64, device="cuda")
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_get_result_device(ctx, a)
        assert ei.value.code == bhq.E_STATE
        vt = torch.zeros((100, 3), dtype=torch.float64, device="cuda")
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_kick_drift(ctx, None, vt, a, 0.1, float("nan"))
        assert ei.value.code == bhq.E_NONFINITE
        rc = bhq.lib().bhq_kick_drift(ctx, 100, None, vt.data_ptr(), v.ctypes.data, 0.1,
                                      0.0, None)
        assert rc == bhq.E_ARG
    finally:
        bhq.bhq_destroy(ctx)


@pytest.mark.slow
def test_cold_collapse_small():
    """The cold-collapse driver on 2^14 particles through the collapse
    (t = 0 .. 2, 512 steps): energy is conserved to 1 % and a dense core
    forms (central density far above the initial 3/(4 pi))."""
    from paper_1812_07313_amd import coldcollapse as cc
    r = cc.run("C", n=1 << 14, t_end=2.0, eps=2.0 ** -6, ncrit=64)
    log("case cold collapse small: %.2f ms/step, dE/E %.3g"
        % (1e3 * r["s_per_step"], r["rel_energy_change"]))
    assert abs(r["rel_energy_change"]) < 1e-2
    p = r["profile"]
    core = [rho for rr, rho, c in zip(p["r"], p["rho"], p["count"]) if rr < 0.1 and c >= 50]
    assert core and max(core) > 20 * 3.0 / (4.0 * np.pi)


@pytest.mark.parametrize("sort_every", [0, 2])
def test_treepm_leapfrog_fp64_matches_oracle(sort_every):
    """Periodic TreePM, FP64: 4 steps on a perturbed 16^3 lattice with a
    velocity field that carries particles across the box faces; positions
    and velocities agree with the oracle's TreePM leapfrog (split tree on
    its own lists + its PM + the same wrap) to the summation-order level."""
    x, m = synth.perturbed_lattice(16, synth.rng(4))
    v = synth.rng(6).normal(size=x.shape) * 0.2
    nmesh = 16
    rs = 1.25 / nmesh
    rcut = 4.5 * rs
    theta, ncrit, dt, steps = 0.5, 32, 2.0 ** -6, 4
    log("case treepm leapfrog fp64 16^3")
    xr, vr, ar, pr = orc.leapfrog(x, v, m, 0.0, dt, steps, theta, ncrit,
                                  kind=orc.SPLIT_QUAD, box=1.0, rs=rs, rcut=rcut,
                                  pm_mesh=nmesh)
    with NBody(x, v, m, 0.0, theta, ncrit, kernel=bhq.SPLIT_QUAD, precision=bhq.FP64,
               box=1.0, rs=rs, rcut=rcut, pm_mesh=nmesh, sort_every=sort_every) as sim:
        sim.step(dt, steps)
        xg, vg = sim.state()
        ag, pg = sim.accelerations()
    assert np.all((xg >= 0) & (xg < 1))
    d = np.abs(xg - xr)
    d = np.minimum(d, 1.0 - d)
    dv = np.abs(vg - vr).max()
    crossed = np.sum(np.any(np.abs(xr - (x + steps * dt * v)) > 0.5, axis=1))
    log("  max |dx| %.3g  max |dv| %.3g  (%d particles wrapped)" % (d.max(), dv, crossed))
    assert crossed > 0
    assert d.max() < 1e-12 and dv < 1e-11
    assert orc.relative_errors(ag, ar).max() < 1e-9
    np.testing.assert_allclose(pg, pr, rtol=1e-9, atol=1e-12)


def test_wrap_periodic_bitwise():
    """bhq_wrap_periodic = x - box floor(x / box), one box off at box, in
    plain FP64 (bitwise), for points inside, outside and on the faces."""
    g = np.random.default_rng(8)
    box = 0.75
    x = np.concatenate([g.uniform(-3, 4, (997, 3)),
                        np.array([[0.0, box, -box], [-1e-300, 2 * box, -0.0],
                                  [box * (1 - 2 ** -53), -box * 2 ** -60, 3 * box]])])
    ctx = bhq.bhq_create(0, bhq.SPLIT_QUAD, bhq.FP64)
    try:
        xt = torch.from_numpy(x.copy()).cuda()
        bhq.bhq_wrap_periodic(ctx, xt, box)
        xg = xt.cpu().numpy()
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_wrap_periodic(ctx, xt, 0.0)
        assert ei.value.code == bhq.E_ARG
    finally:
        bhq.bhq_destroy(ctx)
    y = x - box * np.floor(x / box)
    y = np.where(y >= box, y - box, y)
    assert np.array_equal(xg, y)
    assert np.all((xg >= 0) & (xg < box))


def test_sort_to_tree_order():
    """bhq_sort_to_tree_order: the arrays come back permuted into tree order
    (row k = input row order[k]), bhq_get_lists then reports the identity,
    and the results of the same evaluation come back in the new order."""
    x, v, m = _ic(5000, 7)
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        xt, vt, mt = (torch.from_numpy(a.copy()).cuda() for a in (x, v, m))
        ids = torch.arange(len(m), dtype=torch.int64, device="cuda")
        bhq.bhq_build_lists_device(ctx, xt, mt, 0.6, 64)
        bhq.bhq_set_eps(ctx, 2.0 ** -6)
        bhq.bhq_compute(ctx)
        a0 = torch.zeros((len(m), 3), dtype=torch.float64, device="cuda")
        bhq.bhq_get_result_device(ctx, a0)
        order = bhq.bhq_get_lists(ctx, len(m))["i_idx"]
        assert not np.array_equal(order, np.arange(len(m)))
        bhq.bhq_sort_to_tree_order(ctx, [xt, vt, mt, ids])
        assert np.array_equal(xt.cpu().numpy(), x[order])
        assert np.array_equal(vt.cpu().numpy(), v[order])
        assert np.array_equal(mt.cpu().numpy(), m[order])
        assert np.array_equal(ids.cpu().numpy(), order)
        assert np.array_equal(bhq.bhq_get_lists(ctx, len(m))["i_idx"], np.arange(len(m)))
        a1 = torch.zeros_like(a0)
        bhq.bhq_get_result_device(ctx, a1)
        assert np.array_equal(a1.cpu().numpy(), a0.cpu().numpy()[order])
        # errors: wrong count, row size not a multiple of 8
        f = (ctypes.c_void_p * 1)(xt.data_ptr())
        for n, rb in ((len(m) - 1, 24), (len(m), 12), (len(m), 72)):
            r = (ctypes.c_int * 1)(rb)
            assert bhq.lib().bhq_sort_to_tree_order(ctx, n, 1, f, r, None) == bhq.E_ARG
    finally:
        bhq.bhq_destroy(ctx)
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        with pytest.raises(bhq.BhqError) as ei:
            bhq.bhq_sort_to_tree_order(ctx, [torch.zeros(10, dtype=torch.float64,
                                                         device="cuda")])
        assert ei.value.code == bhq.E_STATE
    finally:
        bhq.bhq_destroy(ctx)


@pytest.mark.parametrize("kernel", [bhq.QUAD, bhq.MONO])
def test_sorted_state_same_trajectory(kernel):
    """NBody keeping its state in tree order (sorted at every build, or every
    third) follows the same FP64 trajectory as the unsorted run: only the
    order of the particles inside a leaf changes, and with it the summation
    order."""
    x, v, m = _ic(3000, 8)
    eps, theta, ncrit, dt, steps = 2.0 ** -6, 0.5, 64, 2.0 ** -8, 8
    out = []
    for every in (0, 1, 3):
        with NBody(x, v, m, eps, theta, ncrit, kernel=kernel, precision=bhq.FP64,
                   sort_every=every) as sim:
            sim.step(dt, steps)
            out.append(sim.state() + sim.accelerations() + sim.energies())
    for o in out[1:]:
        for a, b in zip(out[0][:4], o[:4]):
            np.testing.assert_allclose(a, b, rtol=0, atol=1e-11 * np.abs(a).max())
        assert o[4] == pytest.approx(out[0][4], rel=1e-13)
        assert o[5] == pytest.approx(out[0][5], rel=1e-13)
