"""Benchmark: Barnes-Hut tree force evaluation (monopole + traceless
quadrupole cells, Plummer-softened particle terms) over per-group
interaction lists on one MI355X.

Workload (one "step" = one force evaluation of every particle):
uniform random cube [0,1)^3, N = 2^20 equal-mass particles drawn in FP32,
eps = 1e-3, theta = 0.5, ncrit = 256; quadrupole kernel, FP32 arithmetic
with FP64 group-relative offsets.  Lists are built on the host by the
library's builder and resident in HBM before the timed region.

Prints ONE JSON line: throughput in Ginteractions/s (particle-particle plus
particle-cell interactions per second), the FP32 VALU roofline of the force
kernel, the other variants (monopole, FP64) on the same workload, and the
FP64 oracle timed on the host's cores.

    python bench.py [--steps K] [--warmup W] [--theta T] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1812_07313_amd import bhq, synth  # noqa: E402

# Hardware flops per interaction (FMA = 2, rsqrt = 1, others 1) of the
# kernels' arithmetic: particle term 14 VALU ops / 20 flops, quadrupole
# cell term 34 ops / 53 flops, monopole cell = particle term.
FLOPS_PP = 20
FLOPS_PC = {bhq.QUAD: 53, bhq.MONO: 20}
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (packed FP32)
PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector peak
METRIC = ("Ginteractions/s + s/force-eval at fixed rms error; quad vs mono, "
          "FP32 vs FP64")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_variant(torch, ctx, kernel, precision, steps, warmup, stream):
    bhq.bhq_set_kernel(ctx, kernel, precision)
    for _ in range(warmup):
        bhq.bhq_compute(ctx, stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        bhq.bhq_compute(ctx, stream)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    return wall / steps * 1e3, float(np.mean(kern_ms)), float(np.median(kern_ms))


def cpu_baseline(x, m, eps, theta, ncrit):
    """The FP64 oracle (test infrastructure) timed on this host's cores,
    evaluating the whole workload's lists once."""
    import oracle as orc
    T = orc.Tree(x, m, theta, ncrit)
    mat = orc.materialise(T, x, m)
    n_pp, n_pc = T.interaction_counts()
    t0 = time.perf_counter()
    orc.eval_lists(orc.QUAD, mat, x, eps * eps)
    dt = time.perf_counter() - t0
    return {"value": (n_pp + n_pc) / dt / 1e9, "unit": "Ginteractions/s",
            "cores": orc.num_threads(), "kind": "oracle",
            "sample": "one full FP64 evaluation of all %d particles' lists "
                      "(%.3g interactions, %.2f s)" % (len(m), n_pp + n_pc, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before timing, copy a buffer of this many MiB "
                         "device-to-device once (a plain copy kernel of known "
                         "size, to calibrate HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build evaluates the force "
              "path on a single MI355X (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    if args.copy_calibration_mib > 0:
        nel = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d MiB read + %d MiB written"
            % (args.copy_calibration_mib, args.copy_calibration_mib))
        del src, dst

    c = synth.config_uniform_cube(n=args.n, theta=args.theta)
    x, m, eps, theta, ncrit = c["x"], c["m"], c["eps"], c["theta"], c["ncrit"]
    t0 = time.perf_counter()
    L = bhq.bhq_build_lists(x, m, theta, ncrit)
    t_build = time.perf_counter() - t0
    ng, njp, njc, _ = bhq.bhq_lists_sizes(L)
    log("lists: %d groups, %d j-particles, %d j-cells, built in %.2f s"
        % (ng, njp, njc, t_build))

    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        t0 = time.perf_counter()
        bhq.bhq_set_lists(ctx, L, x, m)
        bhq.bhq_set_eps(ctx, eps)
        t_upload = time.perf_counter() - t0
        bhq.bhq_lists_free(L)
        n_pp, n_pc = bhq.bhq_get_counts(ctx)
        n_int = n_pp + n_pc
        stream = torch.cuda.current_stream()

        ms_step, ms_kern, ms_kern_med = time_variant(
            torch, ctx, bhq.QUAD, bhq.FP32_OFS64, args.steps, args.warmup,
            stream)
        log("quad fp32: %.3f ms/step (kernel %.3f ms)" % (ms_step, ms_kern))
        bhq.bhq_compute(ctx, stream)
        a32, p32 = bhq.bhq_get_result(ctx, len(m))

        variants = {}
        if not args.no_variants:
            for kern, prec in ((bhq.MONO, bhq.FP32_OFS64), (bhq.QUAD, bhq.FP64),
                               (bhq.MONO, bhq.FP64)):
                vs, vk, _ = time_variant(torch, ctx, kern, prec,
                                         max(3, args.steps // 4), 1, stream)
                flops = FLOPS_PP * n_pp + FLOPS_PC[kern] * n_pc
                peak = PEAK_FP64_TFLOPS if prec == bhq.FP64 else PEAK_FP32_TFLOPS
                variants["%s_%s" % (bhq.KERNEL_NAMES[kern],
                                    bhq.PRECISION_NAMES[prec])] = {
                    "ms_per_eval": round(vs, 4), "kernel_ms": round(vk, 4),
                    "Ginteractions_per_s": round(n_int / vk / 1e6, 2),
                    "tflops": round(flops / vk / 1e9, 2),
                    "frac_of_peak": round(flops / vk / 1e9 / peak, 4)}
                log("%s_%s: kernel %.3f ms" % (bhq.KERNEL_NAMES[kern],
                                                bhq.PRECISION_NAMES[prec], vk))
            bhq.bhq_set_kernel(ctx, bhq.QUAD, bhq.FP64)
            bhq.bhq_compute(ctx, stream)
            a64, _ = bhq.bhq_get_result(ctx, len(m))
            e = np.linalg.norm(a32 - a64, axis=1) / np.linalg.norm(a64, axis=1)
            variants["quad_fp32_vs_fp64_rel_err"] = {
                "rms": float(np.sqrt(np.mean(e ** 2))), "max": float(e.max())}
    finally:
        bhq.bhq_destroy(ctx)

    flops = FLOPS_PP * n_pp + FLOPS_PC[bhq.QUAD] * n_pc
    achieved = flops / (ms_kern * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host ...")
        cpu = cpu_baseline(x, m, eps, theta, ncrit)

    out = {
        "metric": METRIC,
        "value": round(n_int / (ms_step * 1e-3) / 1e9, 3),
        "unit": "Ginteractions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "uniform cube [0,1)^3, N=%d (FP32 draws), "
                               "eps=1e-3, theta=%g, ncrit=%d; quadrupole, FP32 "
                               "with FP64 group offsets" % (len(m), theta, ncrit),
                   "n": len(m), "theta": theta, "ncrit": ncrit, "eps": eps,
                   "groups": ng, "n_pp": n_pp, "n_pc": n_pc},
        "s_per_force_eval": round(ms_step * 1e-3, 6),
        "kernel_ms": round(ms_kern, 4), "kernel_ms_median": round(ms_kern_med, 4),
        "pc_Ginteractions_per_s": round(n_pc / (ms_kern * 1e-3) / 1e9, 3),
        "host_list_build_s": round(t_build, 3), "upload_s": round(t_upload, 3),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
