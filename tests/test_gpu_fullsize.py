"""GPU parity at the benchmark's full size: uniform cube, N = 2^20,
theta = 0.5, ncrit = 256, eps = 1e-3, in the launch configuration the
benchmark times (one block per group, LPT order, default stream).  The
oracle evaluates every particle's list, so all 2^20 outputs are compared."""
import numpy as np
import pytest

import oracle as orc
from _parity import assert_parity, errors, log, run, upload
from paper_1812_07313_amd import bhq, synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def test_uniform_cube_1m_full_size():
    c = synth.config_uniform_cube()
    x, m, eps = c["x"], c["m"], c["eps"]
    log("case cube 2^20 theta=0.5: building oracle lists")
    T = orc.Tree(x, m, c["theta"], c["ncrit"])
    mat = orc.materialise(T, x, m)
    log("  groups %d, n_pp %d, n_pc %d" % ((T.ngroups,) + T.interaction_counts()))
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        upload(ctx, mat, x, eps2=eps * eps)
        for bk, ok in ((bhq.QUAD, orc.QUAD), (bhq.MONO, orc.MONO)):
            a_ref, p_ref = orc.eval_lists(ok, mat, x, eps * eps)
            for prec in (bhq.FP32_OFS64, bhq.FP64):
                log("  kernel=%s precision=%s" % (bhq.KERNEL_NAMES[bk],
                                                   bhq.PRECISION_NAMES[prec]))
                a, p = run(ctx, mat, len(m), bk, prec)
                err = errors(a, p, a_ref, p_ref)
                log("    %s" % err)
                assert_parity(err, prec, "cube 2^20")
    finally:
        bhq.bhq_destroy(ctx)
