"""Helpers shared by the GPU parity tests: feed oracle-built interaction
lists to libbhq through the C ABI and compare with the oracle's evaluation
of the same lists."""
import sys

import numpy as np

import oracle as orc
from paper_1812_07313_amd import bhq

# Parity bars.  FP32 bulk arithmetic with FP64 group offsets: per-particle
# relative acceleration error <= 2e-6 rms and <= 1e-4 max.  FP64: the two
# sides differ in summation order, the kernels' rsqrt (a hardware estimate
# and one series step) and, in the split kernels, exp(-u^2) and erfc from
# tables (within 5e-16 relative), all far below 1e-12.
TOL = {
    bhq.FP32_OFS64: dict(rms=2e-6, max=1e-4, pot_rms=2e-6, pot_max=1e-4),
    bhq.FP64: dict(rms=1e-12, max=1e-10, pot_rms=1e-12, pot_max=1e-10),
}


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def upload(ctx, mat, x, eps2=None, split=None):
    """Materialised oracle lists -> context (group order)."""
    x = np.asarray(x, np.float64).reshape(-1, 3)
    i_idx = mat["i_idx"]
    bhq.bhq_set_groups(ctx, mat["i_off"], mat["gcenter"], mat["jp_off"],
                       mat["jc_off"])
    bhq.bhq_set_i(ctx, x[i_idx])
    if eps2 is not None:
        e2 = np.broadcast_to(np.asarray(eps2, np.float64), (x.shape[0],))
        bhq.bhq_set_eps2_i(ctx, np.ascontiguousarray(e2[i_idx]))
    if split is not None:
        bhq.bhq_set_split(ctx, *split)
    if len(mat["jp_m"]):
        bhq.bhq_set_jp(ctx, 0, mat["jp_x"], mat["jp_m"])
    else:
        bhq.bhq_set_jp(ctx, 0, np.zeros((0, 3)), np.zeros(0))
    bhq.bhq_set_jc(ctx, 0, mat["jc_x"], mat["jc_m"], mat["jc_q"], mat["jc_t"])


def run(ctx, mat, n, kernel, precision, stream=None):
    """Compute with (kernel, precision); results in original order."""
    bhq.bhq_set_kernel(ctx, kernel, precision)
    bhq.bhq_compute(ctx, stream)
    a_g, p_g = bhq.bhq_get_result(ctx, n)
    a = np.zeros((n, 3))
    p = np.zeros(n)
    a[mat["i_idx"]] = a_g
    p[mat["i_idx"]] = p_g
    return a, p


def errors(a, p, a_ref, p_ref):
    """Per-particle relative errors; where the reference acceleration is
    exactly zero (a lone particle) the result must be exactly zero too."""
    a = np.asarray(a).reshape(-1, 3)
    a_ref = np.asarray(a_ref).reshape(-1, 3)
    zero = np.all(a_ref == 0.0, axis=1)
    assert np.all(a[zero] == 0.0), "non-zero force where the oracle has none"
    ea = np.zeros(len(a))
    if np.any(~zero):
        ea[~zero] = orc.relative_errors(a[~zero], a_ref[~zero])
    ep = np.abs(p - p_ref) / np.abs(p_ref)
    return dict(rms=float(np.sqrt(np.mean(ea ** 2))), max=float(ea.max()),
                pot_rms=float(np.sqrt(np.mean(ep ** 2))), pot_max=float(ep.max()))


def assert_parity(err, precision, what=""):
    tol = TOL[precision]
    bad = {k: (err[k], tol[k]) for k in tol if not err[k] <= tol[k]}
    assert not bad, "%s parity failed: %s (all: %s)" % (what, bad, err)
