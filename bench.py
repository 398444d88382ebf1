"""Benchmark: Barnes-Hut tree force evaluation (monopole + traceless
quadrupole cells, Plummer-softened particle terms) over per-group
interaction lists on one MI355X.

Default workload (one "step" = one force evaluation of every particle):
uniform random cube [0,1)^3, N = 2^20 equal-mass particles drawn in FP32,
eps = 1e-3, theta = 0.5, ncrit = 256; quadrupole kernel, FP32 arithmetic
with FP64 group-relative offsets.  Lists are built on the host by the
library's builder and are resident in HBM before the timed region.

Prints ONE JSON line (logs go to stderr): throughput in Ginteractions/s
(particle-particle plus particle-cell interactions per second), the FP32
VALU roofline of the force kernel with the shader clock measured beside as
many launches right after the timed ones, the paper-convention GFLOP/s, the other variants on the
same lists (monopole, FP64, complete softened quadrupole), the
quadrupole-versus-monopole comparison at equal rms force error (the paper's
Table 2 question), the FP64 oracle timed on the host's cores (all of them
and one), and compact records of the other four configurations (Plummer
16k, clustered 2^22, 256 batched systems, periodic lattice 2^24 with the
split kernel priced on its pairs inside the cutoff), each on device-built
lists with the oracle on sampled groups beside it.

    python bench.py [--steps K] [--warmup W] [--workload NAME]
        [--no-cpu-baseline] [--no-fixed-error] [--no-variants] [--no-configs]

Other workloads (--workload): sphere and plummer4m (the paper's homogeneous
sphere and Plummer model, N = 4,194,304), plummer16k, clustered, batched,
lattice.
"""
import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1812_07313_amd import bhq, synth  # noqa: E402

# Algorithmic flops per interaction (FMA = 2, rsqrt = 1, other operations
# 1) of the kernels' arithmetic: particle term 14 VALU operations and 20
# flops; quadrupole cell term 34 operations and 53 flops; a monopole cell is
# a particle term; the complete softened quadrupole adds one FMA to the
# cell term (35 operations, 55 flops).  The split kernels add their
# radial-function evaluation; their counts follow.
FLOPS_PP = 20
FLOPS_PC = {bhq.QUAD: 53, bhq.MONO: 20, bhq.QUAD_SOFT: 55}
# FP32 split kernels, per term inside the cutoff (FMA = 2, rsqrt and fract 1,
# the table index conversion 0): particle term 36 (separation 8, rsqrt 1,
# r 1, table variable and fraction 2, erfc and g by Horner 12, the rest 12);
# quadrupole cell term 97 (the same start, four Horner functions 24, D1..D3,
# Q d and d.Q.d, the trace terms and the accumulation); monopole cell 37.
# Masked terms (beyond the cutoff) do no work of the method and are not
# counted: the split roofline is priced on the pairs bhq_count_live finds.
FLOPS_SPLIT_PP = 36
FLOPS_SPLIT_PC = {bhq.SPLIT_QUAD: 97, bhq.SPLIT_MONO: 37}
# FP64 split kernels: the same terms with the radial functions from degree-9
# (exp(-u^2)) and degree-7 (erfcx) polynomials instead of cubics.  Particle
# term 62 (u, table variable and fraction 3, Horner 18 + 14, erfc, the
# e^{-u^2}/sqrt(pi) factor and g 5, the rest as in FP32); quadrupole cell
# term 123 (the particle term's radial part plus u^2, h, k, G2 and G3 12,
# and the FP32 cell term's other 71); monopole cell 63.
FLOPS_SPLIT64_PP = 62
FLOPS_SPLIT64_PC = {bhq.SPLIT_QUAD: 123, bhq.SPLIT_MONO: 63}
# the paper's convention for one particle-cell quadrupole interaction
# (rsqrt counted as 20 flops, Sec. 3.3 and Sec. 5.2)
PAPER_FLOPS_PC = 71
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak
PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector peak
METRIC = ("Ginteractions/s + s/force-eval at fixed rms error; quad vs mono, "
          "FP32 vs FP64")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_digest():
    """sha256 over the force kernels' source: bhq_kernels.hip followed by the
    interaction terms it includes (bhq_terms.h)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("bhq_kernels.hip", "bhq_terms.h"):
        with open(os.path.join(ROOT, "paper_1812_07313_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_traffic(profile="force_kernel_quad_fp32_cube1m.md"):
    """HBM bytes per launch of the quadrupole FP32 kernel on the default
    workload, from the committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE, calibrated against a plain copy).  None when the kernel
    source has changed since those counters were taken."""
    try:
        digest = kernel_source_digest()
        with open(os.path.join(ROOT, "profiles", profile)) as f:
            text = f.read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines()
                  if line.startswith(("kernel_source_sha256:",
                                      "traffic_bytes_per_launch:")))
    if fields.get("kernel_source_sha256", "").strip() != digest:
        return None
    return int(fields["traffic_bytes_per_launch"].strip())


# --- workloads ----------------------------------------------------------------

def workload(name, n=None):
    """Particles and parameters of a named configuration."""
    if name == "cube":
        c = synth.config_uniform_cube(n=n or (1 << 20))
        return dict(name="uniform cube [0,1)^3, N=%d (FP32 draws), eps=1e-3, "
                         "theta=0.5" % len(c["m"]),
                    x=c["x"], m=c["m"], eps=c["eps"], theta=0.5, ncrit=256,
                    kernel=bhq.QUAD)
    if name == "sphere":
        # the paper's homogeneous sphere at its Table 2 size
        nn = n or 4194304
        x, m = synth.uniform_sphere(nn, synth.rng(5))
        return dict(name="homogeneous sphere (radius 1) N=%d, eps=2^-8, "
                         "theta=0.5" % nn,
                    x=x, m=m, eps=2.0 ** -8, theta=0.5, ncrit=256,
                    kernel=bhq.QUAD)
    if name == "plummer4m":
        # the paper's Plummer model at its Table 2 size (softening as for the
        # homogeneous sphere: the paper gives none for these runs)
        nn = n or 4194304
        x, m = synth.plummer(nn, synth.rng(6))
        return dict(name="Plummer sphere (scale radius 1) N=%d, eps=2^-8, theta=0.5" % nn,
                    x=x, m=m, eps=2.0 ** -8, theta=0.5, ncrit=256, kernel=bhq.QUAD)
    if name == "plummer16k":
        c = synth.config_plummer_16k()
        return dict(name="Plummer sphere N=16384, eps=1/64, theta=0.5",
                    x=c["x"], m=c["m"], eps=c["eps"], theta=0.5, ncrit=64,
                    kernel=bhq.QUAD)
    if name == "clustered":
        c = synth.config_clustered(n=n or (1 << 22))
        return dict(name="512 Plummer clusters + 10%% background, N=%d, "
                         "eps=2e-4, theta=0.5" % len(c["m"]),
                    x=c["x"], m=c["m"], eps=c["eps"], theta=0.5, ncrit=256,
                    kernel=bhq.QUAD)
    if name == "batched":
        systems = synth.batched_plummer(256)
        sizes = np.array([len(s[1]) for s in systems])
        off = np.concatenate([[0], np.cumsum(sizes)])
        return dict(name="256 Plummer systems, N log-uniform in [2^10, 2^16] "
                         "(total %d), eps=1/(4 N^(1/3)), theta=0.6" % off[-1],
                    x=np.concatenate([s[0] for s in systems]),
                    m=np.concatenate([s[1] for s in systems]),
                    eps2=np.concatenate([np.full(len(s[1]), s[2] ** 2)
                                         for s in systems]),
                    sys_off=off, theta=0.6, ncrit=64, kernel=bhq.QUAD,
                    tune_ncrits=(64, 128, 256))
    if name == "lattice":
        c = synth.config_lattice(nside=int(round((n or (1 << 24)) ** (1 / 3))))
        return dict(name="perturbed lattice N=%d in the periodic unit box, "
                         "Gaussian split r_s=1.25/256, cutoff 4.5 r_s, "
                         "theta=0.5" % len(c["m"]),
                    x=c["x"], m=c["m"], theta=0.5, ncrit=128, box=1.0,
                    rs=c["rs"], rcut=c["rcut"], kernel=bhq.SPLIT_QUAD,
                    tune_ncrits=(64, 128, 256), waves_per_eu=6)
    raise SystemExit("unknown workload %r" % name)


def build_lists(W, theta, ncrit):
    t0 = time.perf_counter()
    if W.get("sys_off") is not None:
        L = bhq.bhq_build_lists_batch(W["sys_off"], W["x"], W["m"], theta, ncrit,
                                      nleaf=min(8, ncrit))
    else:
        L = bhq.bhq_build_lists(W["x"], W["m"], theta, ncrit,
                                nleaf=min(8, ncrit), box=W.get("box", 0.0),
                                rcut=W.get("rcut", 0.0))
    return L, time.perf_counter() - t0


def device_list_build(torch, W, theta, ncrit, sizes, repeats=3):
    """Time bhq_build_lists_device on the workload (particles already in
    device memory; the call returns when the lists are complete) and check
    that it gives the host builder's list sizes."""
    xt = torch.from_numpy(np.ascontiguousarray(W["x"])).cuda()
    mt = torch.from_numpy(np.ascontiguousarray(W["m"])).cuda()
    e2t = (torch.from_numpy(np.ascontiguousarray(W["eps2"])).cuda()
           if W.get("eps2") is not None else None)
    ctx = bhq.bhq_create(0, W["kernel"], bhq.FP32_OFS64)
    try:
        ts = []
        for _ in range(repeats + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if W.get("sys_off") is not None:
                bhq.bhq_build_lists_device_batch(ctx, W["sys_off"], xt, mt, theta, ncrit,
                                                 min(8, ncrit), eps2=e2t)
            else:
                bhq.bhq_build_lists_device(ctx, xt, mt, theta, ncrit, min(8, ncrit),
                                           W.get("box", 0.0), W.get("rcut", 0.0))
            ts.append(time.perf_counter() - t0)
        same = bhq.bhq_get_lists_sizes(ctx) == tuple(sizes)
        one_walk = bhq.bhq_get_build_info(ctx)[0]
    finally:
        bhq.bhq_destroy(ctx)
    # the first call counts, then fills; the rebuilds walk once into slots
    return {"ms": round(float(np.median(ts[1:])) * 1e3, 3),
            "first_call_ms": round(ts[0] * 1e3, 3), "rebuild_one_walk": bool(one_walk),
            "sizes_equal_host": bool(same)}


def pm_long_range(torch, W, short_ms, repeats):
    """Time the particle-mesh long-range part that completes the split
    kernel into a TreePM force: a mesh of spacing r_s / 1.25 (256^3 for the
    2^24 lattice), particles already in device memory."""
    nmesh = int(round(1.25 * W["box"] / W["rs"]))
    nmesh += nmesh & 1
    xt = torch.from_numpy(np.ascontiguousarray(W["x"])).cuda()
    mt = torch.from_numpy(np.ascontiguousarray(W["m"])).cuda()
    a = torch.zeros((len(W["m"]), 3), dtype=torch.float64, device="cuda")
    p = torch.zeros(len(W["m"]), dtype=torch.float64, device="cuda")
    pm = bhq.bhq_pm_create(nmesh, W["box"], W["rs"])
    try:
        ms = []
        for _ in range(repeats + 1):
            bhq.bhq_pm_compute(pm, xt, mt, a, p)
            ms.append(bhq.bhq_pm_get_ms(pm))
    finally:
        bhq.bhq_pm_destroy(pm)
    pm_ms = float(np.median(ms[1:]))
    del xt, mt, a, p
    return {"nmesh": nmesh, "pm_ms": round(pm_ms, 3),
            "short_range_kernel_ms": round(short_ms, 3),
            "treepm_force_ms": round(pm_ms + short_ms, 3),
            "treepm_step_ms": round(treepm_step(torch, W, nmesh), 3)}


def treepm_step(torch, W, nmesh, steps=3):
    """Wall time of one periodic TreePM leapfrog step on the workload (kick,
    drift, wrap, device list rebuild, split kernel, PM, kick), particles and
    velocities in device memory (put into tree order every 8 builds), after
    one step that includes the first (counting) list build."""
    from paper_1812_07313_amd.nbody import NBody
    v = np.zeros_like(W["x"])
    with NBody(W["x"], v, W["m"], 0.0, W["theta"], W["ncrit"], min(8, W["ncrit"]),
               kernel=W["kernel"], box=W["box"], rs=W["rs"], rcut=W["rcut"],
               pm_mesh=nmesh, sort_every=8) as sim:
        sim.step(1e-3, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(1e-3, steps)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3


def upload(ctx, W, L, indexed=False):
    t0 = time.perf_counter()
    if indexed:
        bhq.bhq_set_lists_indexed(ctx, L, W["x"], W["m"])
    else:
        bhq.bhq_set_lists(ctx, L, W["x"], W["m"])
    P = bhq.bhq_lists_export(L, len(W["m"]))
    if W.get("eps2") is not None:
        bhq.bhq_set_eps2_i(ctx, W["eps2"][P["i_idx"]])
    elif W.get("eps") is not None:
        bhq.bhq_set_eps(ctx, W["eps"])
    if W.get("rs"):
        bhq.bhq_set_split(ctx, W["rs"], W["rcut"], W.get("box", 0.0))
    return P, time.perf_counter() - t0


def time_variant(torch, ctx, kernel, precision, steps, warmup, stream, clock=False,
                 warm_ms=30.0):
    """Wall time per step over `steps` back-to-back launches, and the mean
    and median kernel duration from events recorded on the launch stream.
    Untimed launches first: `warmup` of them, and more until `warm_ms` of
    wall time has passed (the shader clock drops while the GPU idles, for
    instance while the host rebuilds lists, and takes tens of ms of work to
    come back: launches timed right after such a gap ran up to 15 % slow).
    clock: also the mean shader clock (MHz) of one CU over `steps` more
    launches right after the timed ones (bhq_clock_begin on a stream of its
    own, over their first 80 %), else None.  The clock reader runs beside
    untimed launches because beside the timed ones it slowed them by 3 %."""
    bhq.bhq_set_kernel(ctx, kernel, precision)
    t_w = time.perf_counter()
    k = 0
    while k < warmup or (time.perf_counter() - t_w) * 1e3 < warm_ms:
        bhq.bhq_compute(ctx, stream)
        k += 1
        if k >= warmup:
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
    mhz = None
    if clock and steps > 0:
        side = torch.cuda.Stream()
        bhq.bhq_clock_begin(ctx, min(0.8 * steps * float(np.mean(kern_ms)), 10000.0), side)
        for _ in range(steps):
            bhq.bhq_compute(ctx, stream)
        torch.cuda.synchronize()
        mhz = bhq.bhq_clock_end(ctx)
    return wall / steps * 1e3, float(np.mean(kern_ms)), float(np.median(kern_ms)), mhz


def result_orig(ctx, P, n):
    a_g, p_g = bhq.bhq_get_result(ctx, n)
    a = np.zeros_like(a_g)
    p = np.zeros_like(p_g)
    a[P["i_idx"]] = a_g
    p[P["i_idx"]] = p_g
    return a, p


# --- tree error against direct summation ---------------------------------------

def direct_reference(W, P, nsample=4096, seed=7):
    """FP64 direct-summation accelerations (Sec. 4, eq. 8 reference) for a
    sample of whole groups, computed by the library's FP64 kernel with each
    sampled group's list set to every particle of its system."""
    n = len(W["m"])
    ng = len(P["i_off"]) - 1
    rng = np.random.default_rng(seed)
    sel, tot = [], 0
    for g in rng.permutation(ng):
        sel.append(g)
        tot += P["i_off"][g + 1] - P["i_off"][g]
        if tot >= nsample:
            break
    sel = np.sort(np.array(sel))
    sys_off = W.get("sys_off")
    if sys_off is None:
        sys_off = np.array([0, n])
    x, m = W["x"], W["m"]
    i_off, jp_off, centers, i_idx, jp_x, jp_m = [0], [0], [], [], [], []
    for g in sel:
        members = P["i_idx"][P["i_off"][g]:P["i_off"][g + 1]]
        s = np.searchsorted(sys_off, members[0], side="right") - 1
        a, b = sys_off[s], sys_off[s + 1]
        xs, ms = x[a:b], m[a:b]
        if W.get("rcut"):
            # short-range kernel: only particles within the cutoff of the
            # group's cell can contribute (minimum image in the box)
            d = xs - P["center"][g]
            box = W.get("box", 0.0)
            if box > 0:
                d -= box * np.rint(d / box)
            v = np.maximum(np.abs(d) - 0.5 * P["side"][g], 0.0)
            keep = np.einsum("ij,ij->i", v, v) <= W["rcut"] ** 2
            xs, ms = xs[keep], ms[keep]
        i_idx.append(members)
        i_off.append(i_off[-1] + len(members))
        jp_x.append(xs)
        jp_m.append(ms)
        jp_off.append(jp_off[-1] + len(ms))
        centers.append(P["center"][g])
    i_idx = np.concatenate(i_idx)
    ctx = bhq.bhq_create(0, W["kernel"], bhq.FP64)
    try:
        bhq.bhq_set_groups(ctx, i_off, np.array(centers), jp_off,
                           np.zeros(len(i_off), np.int64))
        bhq.bhq_set_i(ctx, x[i_idx])
        if W.get("eps2") is not None:
            bhq.bhq_set_eps2_i(ctx, W["eps2"][i_idx])
        elif W.get("eps") is not None:
            bhq.bhq_set_eps(ctx, W["eps"])
        if W.get("rs"):
            bhq.bhq_set_split(ctx, W["rs"], W["rcut"], W.get("box", 0.0))
        bhq.bhq_set_jp(ctx, 0, np.concatenate(jp_x), np.concatenate(jp_m))
        bhq.bhq_set_jc(ctx, 0, np.zeros((0, 3)), np.zeros(0), np.zeros((0, 6)))
        bhq.bhq_compute(ctx)
        a, _ = bhq.bhq_get_result(ctx, len(i_idx))
    finally:
        bhq.bhq_destroy(ctx)
    return i_idx, a


def lane_slot_fraction(i_off, jp_off, jc_off, block, ipt, ops_pp=14, ops_pc=34):
    """Fraction of the lane-slots the force kernel's term loops issue that
    hold a real (i-particle, list entry) pair, from the group sizes and the
    kernel's slicing: a pass over nic <= block * ipt i-particles of a group
    gives each slice P = ceil(nic / ipt) threads and runs S = floor(block / P)
    slices; every wave holding an active thread issues (ipt slots per lane);
    a tile of T = S floor(block / S) list entries takes ceil(cnt / S) steps.
    Particle and cell terms are weighted by their VALU operation counts."""
    ni = np.diff(np.asarray(i_off, np.int64))
    lists = ((np.diff(np.asarray(jp_off, np.int64)), ops_pp),
             (np.diff(np.asarray(jc_off, np.int64)), ops_pc))
    issued = useful = 0.0
    for ib in range(0, int(ni.max()) if len(ni) else 0, block * ipt):
        nic = np.clip(ni - ib, 0, block * ipt)
        on = nic > 0
        nic = nic[on]
        P = -(-nic // ipt)
        S = block // P
        waves = -(-(S * P) // 64)
        T = S * (block // S)
        for n, ops in lists:
            n = n[on]
            steps = (n // T) * (T // S) + -(-(n % T) // S)
            issued += float(np.sum(waves * 64 * ipt * steps)) * ops
            useful += float(np.sum(nic * n)) * ops
    return useful / issued if issued else 1.0


def tree_error(a_tree, ref):
    idx, a_dir = ref
    e = (np.linalg.norm(a_tree[idx] - a_dir, axis=1) /
         np.linalg.norm(a_dir, axis=1))
    return dict(rms=float(np.sqrt(np.mean(e ** 2))),
                p90=float(np.percentile(e, 90)), max=float(e.max()))


def fixed_error_study(torch, ctx, W, ref, stream, steps):
    """Quadrupole versus monopole at equal rms force error: for monopole
    theta0 in {0.3, 0.5, 0.7} find the quadrupole theta with the same rms
    tree error (log-log interpolation over a theta grid), rebuild the
    lists there and time both kernels, in FP32 and FP64, and the device
    rebuild of the tree and lists at that theta: the total (build + FP32
    force) is the GPU's counterpart of the paper's T_total."""
    xt = torch.from_numpy(np.ascontiguousarray(W["x"])).cuda()
    mt = torch.from_numpy(np.ascontiguousarray(W["m"])).cuda()
    e2t = (torch.from_numpy(np.ascontiguousarray(W["eps2"])).cuda()
           if W.get("eps2") is not None else None)
    bctx = bhq.bhq_create(0, W["kernel"], bhq.FP32_OFS64)

    def build_ms(theta):
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if W.get("sys_off") is not None:
                bhq.bhq_build_lists_device_batch(bctx, W["sys_off"], xt, mt, theta, W["ncrit"],
                                                 min(8, W["ncrit"]), eps2=e2t)
            else:
                bhq.bhq_build_lists_device(bctx, xt, mt, theta, W["ncrit"],
                                           min(8, W["ncrit"]), W.get("box", 0.0),
                                           W.get("rcut", 0.0))
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts[1:])) * 1e3   # rebuilds

    def measure(kernel, theta, timing):
        L, _ = build_lists(W, theta, W["ncrit"])
        try:
            P, _ = upload(ctx, W, L, indexed=W.get("indexed", False))
        finally:
            bhq.bhq_lists_free(L)
        bhq.bhq_set_kernel(ctx, kernel, bhq.FP32_OFS64)
        bhq.bhq_compute(ctx, stream)
        a, _ = result_orig(ctx, P, len(W["m"]))
        out = dict(theta=round(theta, 4), err=tree_error(a, ref))
        if timing:
            pp, pc = bhq.bhq_get_counts(ctx)
            for prec in (bhq.FP32_OFS64, bhq.FP64):
                _, km, _, _ = time_variant(torch, ctx, kernel, prec, steps, 1,
                                           stream)
                out["ms_" + bhq.PRECISION_NAMES[prec]] = round(km, 4)
            out["n_pp"], out["n_pc"] = pp, pc
            out["build_ms"] = round(build_ms(theta), 4)
        return out

    try:
        return _fixed_error_rows(measure)
    finally:
        bhq.bhq_destroy(bctx)


def _fixed_error_rows(measure):
    quad_grid = [measure(bhq.QUAD, th, False)
                 for th in (0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0)]
    lt = np.log([q["theta"] for q in quad_grid])
    le = np.log([q["err"]["rms"] for q in quad_grid])
    rows = []
    for th0 in (0.3, 0.5, 0.7):
        mono = measure(bhq.MONO, th0, True)
        target = np.log(mono["err"]["rms"])
        if target <= le[0]:
            thq = float(np.exp(lt[0]))
        elif target >= le[-1]:
            thq = float(np.exp(lt[-1]))
        else:
            thq = float(np.exp(np.interp(target, le, lt)))
        quad = measure(bhq.QUAD, thq, True)
        rows.append(dict(mono=mono, quad=quad,
                         quad_speedup_fp32=round(mono["ms_fp32_ofs64"] /
                                                 quad["ms_fp32_ofs64"], 3),
                         quad_speedup_fp64=round(mono["ms_fp64"] /
                                                 quad["ms_fp64"], 3),
                         quad_speedup_total_fp32=round(
                             (mono["build_ms"] + mono["ms_fp32_ofs64"]) /
                             (quad["build_ms"] + quad["ms_fp32_ofs64"]), 3)))
        log("fixed error %.3g: mono theta %.2f %.3f ms | quad theta %.3f "
            "(err %.3g) %.3f ms" % (mono["err"]["rms"], th0,
                                    mono["ms_fp32_ofs64"], thq,
                                    quad["err"]["rms"], quad["ms_fp32_ofs64"]))
    return dict(rows=rows, quad_theta_grid=[dict(theta=q["theta"],
                                                 rms=q["err"]["rms"])
                                            for q in quad_grid])


# --- CPU baseline -----------------------------------------------------------------

def host_info():
    """The host CPU: model, sockets x cores (lscpu), logical CPUs, and the
    CPUs this process may run on."""
    info = {"model": None, "physical_cores": None, "threads_per_core": None,
            "logical_cpus": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0))}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        kv = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        info["model"] = kv.get("Model name")
        sockets = int(kv.get("Socket(s)", "0") or 0)
        per = int(kv.get("Core(s) per socket", "0") or 0)
        info["physical_cores"] = sockets * per or None
        info["threads_per_core"] = int(kv.get("Thread(s) per core", "0") or 0) or None
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return info


def _sample_interactions(mat):
    ni = np.diff(mat["i_off"])
    return int(np.sum(ni * (np.diff(mat["jp_off"]) + np.diff(mat["jc_off"]))))


def cpu_baseline(W, a_gpu, host):
    """The FP64 oracle (test infrastructure) timed on this host's cores: its
    own tree, groups and lists (built separately, timed), one evaluation of
    every particle's lists with all its threads, and one thread on every
    16th group (the paper's single-core setting).  Its result also gives the
    GPU FP32 path's error against the oracle."""
    import oracle as orc
    nt = orc.num_threads()
    t0 = time.perf_counter()
    T = orc.Tree(W["x"], W["m"], W["theta"], W["ncrit"])
    t_tree = time.perf_counter() - t0
    mat = orc.materialise(T, W["x"], W["m"])
    n_pp, n_pc = T.interaction_counts()
    t0 = time.perf_counter()
    a_o, _ = orc.eval_lists(orc.QUAD, mat, W["x"], W["eps"] ** 2)
    dt = time.perf_counter() - t0
    e = orc.relative_errors(a_gpu, a_o)
    smat = T.sample_mat(W["x"], W["m"], np.arange(0, T.ngroups, 16))
    n1 = _sample_interactions(smat)
    orc.set_threads(1)
    try:
        t0 = time.perf_counter()
        orc.eval_lists(orc.QUAD, smat, W["x"], W["eps"] ** 2)
        dt1 = time.perf_counter() - t0
    finally:
        orc.set_threads(nt)
    return {"value": round((n_pp + n_pc) / dt / 1e9, 4),
            "unit": "Ginteractions/s", "cores": nt,
            "kind": "oracle",
            "sample": "one full FP64 evaluation of all %d particles' lists "
                      "(%.3g interactions, %.2f s, %d threads)" % (len(W["m"]), n_pp + n_pc,
                                                                  dt, nt),
            "one_thread": {"value": round(n1 / dt1 / 1e9, 4), "unit": "Ginteractions/s",
                           "sample": "every 16th group (%.3g interactions, %.2f s)" % (n1, dt1)},
            "tree_and_lists_s": round(t_tree, 3),
            "host": host,
            "gpu_fp32_vs_oracle": {"rms": float(np.sqrt(np.mean(e ** 2))),
                                   "max": float(e.max())}}


def direct_check(W, ref):
    """The sampled direct-sum reference of the tree-error study (the
    library's FP64 kernel over every particle) against the oracle's direct
    summation of the same targets: the largest relative difference."""
    import oracle as orc
    idx, a_lib = ref
    t0 = time.perf_counter()
    e2 = W["eps2"] if W.get("eps2") is not None else W["eps"] ** 2
    a_o, _ = orc.direct(W["x"], W["m"], e2, targets=idx)
    dt = time.perf_counter() - t0
    e = orc.relative_errors(a_lib, a_o)
    return {"targets": int(len(idx)), "max_rel_diff": float(e.max()),
            "rms_rel_diff": float(np.sqrt(np.mean(e ** 2))), "oracle_s": round(dt, 2)}


# --- the other configurations (compact records) ----------------------------------

def _dev_ctx(torch, W, ncrit, kernel):
    """A context holding device-built lists of the workload."""
    xt = torch.from_numpy(np.ascontiguousarray(W["x"])).cuda()
    mt = torch.from_numpy(np.ascontiguousarray(W["m"])).cuda()
    ctx = bhq.bhq_create(0, kernel, bhq.FP32_OFS64)
    try:
        if W.get("sys_off") is not None:
            e2t = torch.from_numpy(np.ascontiguousarray(W["eps2"])).cuda()
            bhq.bhq_build_lists_device_batch(ctx, W["sys_off"], xt, mt, W["theta"], ncrit,
                                             min(8, ncrit), eps2=e2t)
        else:
            bhq.bhq_build_lists_device(ctx, xt, mt, W["theta"], ncrit, min(8, ncrit),
                                       W.get("box", 0.0), W.get("rcut", 0.0))
            if W.get("eps") is not None:
                bhq.bhq_set_eps(ctx, W["eps"])
        if W.get("rs"):
            bhq.bhq_set_split(ctx, W["rs"], W["rcut"], W.get("box", 0.0))
    except Exception:
        bhq.bhq_destroy(ctx)
        raise
    return ctx


def _result_input_order(torch, ctx, n, stream):
    a = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    p = torch.empty(n, dtype=torch.float64, device="cuda")
    bhq.bhq_compute(ctx, stream)
    bhq.bhq_get_result_device(ctx, a, p, stream)
    torch.cuda.synchronize()
    return a.cpu().numpy(), p.cpu().numpy()


def _priced(kernel, n_pp, n_pc, ms, peak, fp64=False):
    if kernel in FLOPS_PC:
        flops = FLOPS_PP * n_pp + FLOPS_PC[kernel] * n_pc
    elif fp64:
        flops = FLOPS_SPLIT64_PP * n_pp + FLOPS_SPLIT64_PC[kernel] * n_pc
    else:
        flops = FLOPS_SPLIT_PP * n_pp + FLOPS_SPLIT_PC[kernel] * n_pc
    tf = flops / (ms * 1e-3) / 1e12
    return {"tflops": round(tf, 3), "frac": round(tf / peak, 4)}


def config_record(torch, stream, W, kernel, ncrit, shapes, steps, fp64=True, live=False):
    """One configuration on device-built lists: the FP32 kernel time for each
    launch shape (bhq_set_tuning arguments) and the fastest, the FP64 time at
    that shape, throughput and the FP32 roofline fraction; for the split
    kernels the pairs inside the cutoff and the roofline priced on them.
    Returns (record, FP32 accelerations, FP32 potentials), in input order."""
    ctx = _dev_ctx(torch, W, ncrit, kernel)
    n = len(W["m"])
    try:
        n_pp, n_pc = bhq.bhq_get_counts(ctx)
        ng = bhq.bhq_get_lists_sizes(ctx)[0]
        rows = []
        for shape in shapes:
            bhq.bhq_set_tuning(ctx, *shape)
            _, km, kmed, _ = time_variant(torch, ctx, kernel, bhq.FP32_OFS64, steps, 2, stream)
            rows.append(dict(shape=list(shape), kernel_ms=round(km, 4),
                             kernel_ms_median=round(kmed, 4)))
        best = min(rows, key=lambda r: r["kernel_ms"])
        bhq.bhq_set_tuning(ctx, *best["shape"])
        km = best["kernel_ms"]
        rec = {"workload": W["name"] + ", ncrit=%d" % ncrit, "n": n, "groups": ng,
               "n_pp": n_pp, "n_pc": n_pc, "kernel": bhq.KERNEL_NAMES[kernel],
               "launch": dict(zip(("block", "i_per_thread", "blocks_per_cu", "persistent",
                                   "graph", "jsplit", "waves_per_eu"), best["shape"])),
               "shapes": rows, "kernel_ms_fp32": km,
               "Ginteractions_per_s": round((n_pp + n_pc) / km / 1e6, 2),
               "s_per_force_eval": round(km * 1e-3, 7)}
        if live:
            lp, lc = bhq.bhq_count_live(ctx)
            rec["live_pp"], rec["live_pc"] = lp, lc
            rec["live_fraction"] = {"pp": round(lp / max(n_pp, 1), 4),
                                    "pc": round(lc / max(n_pc, 1), 4)}
            rec["live_Ginteractions_per_s"] = round((lp + lc) / km / 1e6, 2)
            rec["roofline_fp32"] = dict(_priced(kernel, lp, lc, km, PEAK_FP32_TFLOPS),
                                        priced_on="pairs inside the cutoff")
        else:
            rec["roofline_fp32"] = _priced(kernel, n_pp, n_pc, km, PEAK_FP32_TFLOPS)
        a32, p32 = _result_input_order(torch, ctx, n, stream)
        if fp64:
            _, k64, _, _ = time_variant(torch, ctx, kernel, bhq.FP64, max(5, steps // 2), 1,
                                        stream)
            rec["kernel_ms_fp64"] = round(k64, 4)
            if live:
                rec["roofline_fp64"] = dict(_priced(kernel, lp, lc, k64, PEAK_FP64_TFLOPS,
                                                    fp64=True),
                                            priced_on="pairs inside the cutoff")
            else:
                rec["roofline_fp64"] = _priced(kernel, n_pp, n_pc, k64, PEAK_FP64_TFLOPS)
            a64, _ = _result_input_order(torch, ctx, n, stream)
            e = np.linalg.norm(a32 - a64, axis=1) / np.linalg.norm(a64, axis=1)
            rec["fp32_vs_fp64_rel_err"] = {"rms": float(np.sqrt(np.mean(e ** 2))),
                                           "max": float(e.max())}
    finally:
        bhq.bhq_destroy(ctx)
    return rec, a32, p32


def oracle_leg(W, kernel, ncrit, a_gpu, stride):
    """The oracle on every stride-th group of its own tree (the same lists as
    the GPU's): its FP64 rate, its tree and list build time, and the GPU
    FP32 result's error against it on those groups' particles."""
    import oracle as orc
    okind = {bhq.QUAD: orc.QUAD, bhq.SPLIT_QUAD: orc.SPLIT_QUAD}[kernel]
    t0 = time.perf_counter()
    T = orc.Tree(W["x"], W["m"], W["theta"], ncrit, nleaf=min(8, ncrit),
                 box=W.get("box", 0.0), rcut=W.get("rcut", 0.0), walk_stride=stride)
    t_tree = time.perf_counter() - t0
    mat = T.sample_mat(W["x"], W["m"], np.arange(0, T.ngroups, stride))
    nint = _sample_interactions(mat)
    t0 = time.perf_counter()
    if kernel == bhq.SPLIT_QUAD:
        a_o, _ = orc.eval_lists(okind, mat, W["x"], 0.0, box=W["box"], rs=W["rs"],
                                rcut=W["rcut"], mask=orc.MASK_F64_OFS)
    else:
        a_o, _ = orc.eval_lists(okind, mat, W["x"], W["eps"] ** 2)
    dt = time.perf_counter() - t0
    sel = mat["i_idx"]
    e = orc.relative_errors(a_gpu[sel], a_o[sel])
    return {"value": round(nint / dt / 1e9, 4), "unit": "Ginteractions/s",
            "cores": orc.num_threads(), "kind": "oracle",
            "sample": "every %d-th group: %d groups, %d particles, %.3g interactions, %.2f s"
                      % (stride, len(mat["i_off"]) - 1, len(sel), nint, dt),
            "tree_and_lists_s": round(t_tree, 3),
            "gpu_fp32_vs_oracle": {"rms": float(np.sqrt(np.mean(e ** 2))),
                                   "max": float(e.max()), "particles": int(len(sel))}}


def other_configs(torch, stream, steps, cpu=True):
    """Compact records of the small, clustered, batched and periodic
    configurations, each on device-built lists, with the oracle on sampled
    groups beside it."""
    import oracle as orc
    recs = {}
    eager = [(256, 2, 0, 0, 0, 1), (256, 1, 0, 0, 0, 1), (256, 2, 0, 0, 0, 1, 6)]

    W = workload("plummer16k")
    shapes = [(256, ipt, 0, 0, 0, js) for ipt in (1, 2) for js in (1, 2, 4, 8)]
    shapes += [(256, 1, 0, 0, 0, js, w) for js in (2, 4) for w in (6, 8)]
    rec, a32, _ = config_record(torch, stream, W, bhq.QUAD, 64, shapes, steps)
    if cpu:
        rec["cpu_baseline"] = oracle_leg(W, bhq.QUAD, 64, a32, 1)
        t0 = time.perf_counter()
        a_d, _ = orc.direct(W["x"], W["m"], W["eps"] ** 2)
        e = orc.relative_errors(a32, a_d)
        rec["tree_error_vs_direct"] = {"rms": float(np.sqrt(np.mean(e ** 2))),
                                       "p90": float(np.percentile(e, 90)),
                                       "max": float(e.max()),
                                       "direct_s": round(time.perf_counter() - t0, 2)}
    recs["plummer16k"] = rec
    log("plummer16k: %.4f ms (%s)" % (rec["kernel_ms_fp32"], rec["launch"]))

    W = workload("clustered")
    rec, a32, _ = config_record(torch, stream, W, bhq.QUAD, 256,
                                eager + [(256, 2, 0, 1, 0, 1)], steps)
    if cpu:
        rec["cpu_baseline"] = oracle_leg(W, bhq.QUAD, 256, a32, 64)
    recs["clustered"] = rec
    log("clustered: %.3f ms" % rec["kernel_ms_fp32"])
    del W

    W = workload("batched")
    best = None
    for ncrit in (64, 128):
        rec, a32, _ = config_record(
            torch, stream, W, bhq.QUAD, ncrit,
            eager + [(256, 1, 0, 0, 0, 1, 6), (256, 2, 0, 1, 1, 1), (256, 1, 0, 1, 1, 1),
                     (256, 1, 0, 1, 1, 1, 6)], steps)
        if best is None or rec["kernel_ms_fp32"] < best[0]["kernel_ms_fp32"]:
            best = (rec, a32, ncrit)
    rec, a32, ncrit = best
    graph = [r for r in rec["shapes"] if r["shape"][3] == 1 and r["shape"][4] == 1]
    rec["persistent_graph_kernel_ms"] = min(r["kernel_ms"] for r in graph)
    rec["eager_kernel_ms"] = min(r["kernel_ms"] for r in rec["shapes"] if r["shape"][3] == 0)
    if cpu:
        t_all, n_all, errs, t_tree = 0.0, 0, [], 0.0
        off = W["sys_off"]
        for sidx in range(0, len(off) - 1, 8):
            x, m = W["x"][off[sidx]:off[sidx + 1]], W["m"][off[sidx]:off[sidx + 1]]
            t0 = time.perf_counter()
            T = orc.Tree(x, m, W["theta"], ncrit, nleaf=min(8, ncrit))
            t_tree += time.perf_counter() - t0
            mat = orc.materialise(T, x, m)
            t0 = time.perf_counter()
            a_o, _ = orc.eval_lists(orc.QUAD, mat, x, W["eps2"][off[sidx]:off[sidx + 1]])
            t_all += time.perf_counter() - t0
            n_all += _sample_interactions(mat)
            errs.append(orc.relative_errors(a32[off[sidx]:off[sidx + 1]], a_o))
        e = np.concatenate(errs)
        rec["cpu_baseline"] = {
            "value": round(n_all / t_all / 1e9, 4), "unit": "Ginteractions/s",
            "cores": orc.num_threads(), "kind": "oracle",
            "sample": "every 8th system (32 of 256, %d particles, %.3g interactions, %.2f s)"
                      % (len(e), n_all, t_all),
            "tree_and_lists_s": round(t_tree, 3),
            "gpu_fp32_vs_oracle": {"rms": float(np.sqrt(np.mean(e ** 2))),
                                   "max": float(e.max()), "particles": int(len(e))}}
    recs["batched"] = rec
    log("batched: ncrit %d, eager %.3f ms, persistent+graph %.3f ms"
        % (ncrit, rec["eager_kernel_ms"], rec["persistent_graph_kernel_ms"]))
    del W

    W = workload("lattice")
    rec, a32, _ = config_record(torch, stream, W, bhq.SPLIT_QUAD, 128,
                                [(256, 2, 0, 0, 0, 1, 0), (256, 2, 0, 0, 0, 1, 6),
                                 (256, 2, 0, 1, 0, 1, 6), (256, 1, 0, 0, 0, 1, 0)],
                                max(5, steps // 2), live=True)
    if cpu:
        rec["cpu_baseline"] = oracle_leg(W, bhq.SPLIT_QUAD, 128, a32, 2000)
    recs["lattice"] = rec
    log("lattice: %.3f ms, live pairs %s" % (rec["kernel_ms_fp32"], rec["live_fraction"]))
    return recs


ORDERS = {"xcd": bhq.ORDER_XCD, "cost": bhq.ORDER_COST}


# --- main -------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cube",
                    choices=["cube", "sphere", "plummer4m", "plummer16k", "clustered",
                             "batched", "lattice"])
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--ncrit", type=int, default=None,
                    help="group size bound (default: the workload's)")
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--ipt", type=int, default=2,
                    help="i-particles per thread (1 or 2)")
    ap.add_argument("--persistent", type=int, default=0)
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--waves-per-eu", type=int, default=None,
                    help="register cap for 6 or 8 waves per SIMD (0: compiler's choice; "
                         "default: 6 for the lattice, where the autotuner picks it, else 0)")
    ap.add_argument("--jsplit", type=int, default=1,
                    help="parts each group's lists are cut into (1, 2, 4, 8)")
    ap.add_argument("--order", default="xcd", choices=["xcd", "cost"],
                    help="group dispatch order: contiguous pieces of equal "
                         "cost per XCD (windows sorted longest first), or "
                         "every group longest first")
    ap.add_argument("--order-window", type=int, default=bhq.ORDER_WINDOW,
                    help="window of the xcd order")
    ap.add_argument("--order-tail", type=int, default=bhq.ORDER_TAIL,
                    help="groups at the end of each XCD's piece sorted as one "
                         "window")
    ap.add_argument("--lists", default="indexed",
                    choices=["materialised", "indexed"],
                    help="list upload mode: index lists into shared particle "
                         "and cell pools, or materialised copies")
    ap.add_argument("--autotune", type=int, default=None,
                    help="1: choose ncrit and the launch shape with the "
                         "autotuner before timing (default: on for the "
                         "batched workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-fixed-error", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the records of the other four configurations")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="before timing, copy a buffer of this many MiB "
                         "device-to-device once (a plain copy kernel of known "
                         "size, to calibrate HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library evaluates the force "
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

    W = workload(args.workload, args.n)
    if args.ncrit is not None:
        W["ncrit"] = args.ncrit
    kernel = W["kernel"]
    n = len(W["m"])
    if args.waves_per_eu is None:
        args.waves_per_eu = W.get("waves_per_eu", 0)
    tuned = None
    if args.autotune is None:
        args.autotune = 1 if args.workload == "batched" else 0
    if args.autotune:
        from paper_1812_07313_amd import tune
        # the configurations that name a group size keep it; the others
        # search ncrit too
        log("autotuning %s and launch shape ..." % ("ncrit" if "tune_ncrits" in W else
                                                    "ncrit=%d fixed:" % W["ncrit"]))
        tctx = bhq.bhq_create(0, kernel, bhq.FP32_OFS64)
        try:
            r = tune.autotune(tctx, W["x"], W["m"], W["theta"], args.workload,
                              kernel=kernel, eps=W.get("eps"),
                              eps2_per_particle=W.get("eps2"),
                              sys_off=W.get("sys_off"), box=W.get("box", 0.0),
                              rcut=W.get("rcut", 0.0), rs=W.get("rs", 0.0),
                              ncrits=W.get("tune_ncrits", (W["ncrit"],)), force=True)
        finally:
            bhq.bhq_destroy(tctx)
        tuned = r["best"]
        W["ncrit"] = tuned["ncrit"]
        args.block, args.persistent = tuned["block"], tuned["persistent"]
        args.ipt = tuned["i_per_thread"]
        args.graph, args.jsplit = tuned["use_graph"], tuned["jsplit"]
        args.waves_per_eu = tuned["waves_per_eu"]
        args.order = {v: k for k, v in ORDERS.items()}[tuned["order"]]
        log("autotuned: %s" % tuned)
    L, t_build = build_lists(W, W["theta"], W["ncrit"])
    ng, njp, njc, ncell = bhq.bhq_lists_sizes(L)
    log("%s: %d groups, %d j-particles, %d j-cells, lists built in %.2f s"
        % (W["name"], ng, njp, njc, t_build))

    stream = torch.cuda.current_stream()
    ctx = bhq.bhq_create(0, kernel, bhq.FP32_OFS64)
    out_extra = {}
    try:
        P, t_upload = upload(ctx, W, L, indexed=(args.lists == "indexed"))
        bhq.bhq_lists_free(L)
        bhq.bhq_set_tuning(ctx, args.block, args.ipt,
                           tuned["blocks_per_cu"] if tuned else 0,
                           args.persistent, args.graph, args.jsplit, args.waves_per_eu)
        bhq.bhq_set_group_order(ctx, ORDERS[args.order], args.order_window,
                                args.order_tail)
        n_pp, n_pc = bhq.bhq_get_counts(ctx)
        n_int = n_pp + n_pc
        live = bhq.bhq_count_live(ctx) if kernel not in FLOPS_PC else None
        # the term loops' lane-slots that hold a pair (all list pairs, as
        # the non-split kernels evaluate them)
        lane_slots = lane_slot_fraction(P["i_off"], P["jp_off"], P["jc_off"], args.block,
                                        args.ipt)

        # The variants are timed first, and the headline launches after them.
        # From an idle GPU the shader clock ramps up over the first tens of
        # milliseconds of work; the variants' launches (reported below) take
        # the GPU there, so the W warm-up and K timed launches measure the
        # kernel at the clock it holds under sustained load.
        variants = {}
        if not args.no_variants:
            others = [(kernel, bhq.FP64)]
            if kernel == bhq.QUAD:
                others = [(bhq.MONO, bhq.FP32_OFS64), (bhq.QUAD, bhq.FP64),
                          (bhq.MONO, bhq.FP64), (bhq.QUAD_SOFT, bhq.FP32_OFS64)]
            elif kernel == bhq.SPLIT_QUAD:
                others = [(bhq.SPLIT_MONO, bhq.FP32_OFS64),
                          (bhq.SPLIT_QUAD, bhq.FP64)]
            for kern, prec in others:
                vs, vk, _, _ = time_variant(torch, ctx, kern, prec,
                                            max(5, args.steps // 2), 1, stream)
                v = {"ms_per_eval": round(vs, 4), "kernel_ms": round(vk, 4),
                     "Ginteractions_per_s": round(n_int / vk / 1e6, 2)}
                peak = (PEAK_FP64_TFLOPS if prec == bhq.FP64
                        else PEAK_FP32_TFLOPS)
                if kern in FLOPS_PC:
                    flops = FLOPS_PP * n_pp + FLOPS_PC[kern] * n_pc
                    v["tflops"] = round(flops / vk / 1e9, 2)
                    v["frac_of_peak"] = round(flops / vk / 1e9 / peak, 4)
                elif live is not None:
                    # the split variants decide the cutoff as the headline
                    # kernel does, so the same pairs are live
                    pr = _priced(kern, live[0], live[1], vk, peak, fp64=prec == bhq.FP64)
                    v["tflops"], v["frac_of_peak"] = pr["tflops"], pr["frac"]
                    v["priced_on"] = "pairs inside the cutoff"
                variants["%s_%s" % (bhq.KERNEL_NAMES[kern],
                                    bhq.PRECISION_NAMES[prec])] = v
                log("%s_%s: kernel %.3f ms" % (bhq.KERNEL_NAMES[kern],
                                                bhq.PRECISION_NAMES[prec], vk))

        # exactly args.warmup untimed launches: the variants just ran, so the
        # GPU is busy up to here
        ms_step, ms_kern, ms_kern_med, sclk = time_variant(
            torch, ctx, kernel, bhq.FP32_OFS64, args.steps, args.warmup, stream, clock=True,
            warm_ms=0.0)
        log("%s fp32: %.3f ms/step (kernel %.3f ms)"
            % (bhq.KERNEL_NAMES[kernel], ms_step, ms_kern))
        bhq.bhq_compute(ctx, stream)
        a32, _ = result_orig(ctx, P, n)

        if not args.no_variants:
            bhq.bhq_set_kernel(ctx, kernel, bhq.FP64)
            bhq.bhq_compute(ctx, stream)
            a64, _ = result_orig(ctx, P, n)
            e = np.linalg.norm(a32 - a64, axis=1) / np.linalg.norm(a64, axis=1)
            variants["fp32_vs_fp64_rel_err"] = {
                "rms": float(np.sqrt(np.mean(e ** 2))), "max": float(e.max())}

        ref = direct_reference(W, P, nsample=4096 if n <= (1 << 20) else 1024)
        out_extra["tree_error_vs_direct"] = dict(
            sample=len(ref[0]), fp32=tree_error(a32, ref))
        if not args.no_cpu_baseline and not W.get("rs"):
            log("checking the direct-sum reference with the oracle ...")
            out_extra["tree_error_vs_direct"]["reference_vs_oracle_direct"] = direct_check(W, ref)
        if kernel == bhq.QUAD and not args.no_variants:
            # the complete softened quadrupole (with the cells' trace term)
            bhq.bhq_set_kernel(ctx, bhq.QUAD_SOFT, bhq.FP32_OFS64)
            bhq.bhq_compute(ctx, stream)
            a_soft, _ = result_orig(ctx, P, n)
            out_extra["tree_error_vs_direct"]["fp32_quad_soft"] = tree_error(a_soft, ref)
            bhq.bhq_set_kernel(ctx, kernel, bhq.FP32_OFS64)
        if not args.no_fixed_error and args.workload in ("cube", "sphere", "plummer4m"):
            W["indexed"] = args.lists == "indexed"
            log("fixed-error study ...")
            out_extra["fixed_error"] = fixed_error_study(
                torch, ctx, W, ref, stream, max(5, args.steps // 4))
    finally:
        bhq.bhq_destroy(ctx)

    treepm = None
    if W.get("rs") and W.get("box"):
        treepm = pm_long_range(torch, W, ms_kern, max(3, args.steps // 4))
        log("PM long range (mesh %d): %.3f ms" % (treepm["nmesh"], treepm["pm_ms"]))
    dev_build = device_list_build(torch, W, W["theta"], W["ncrit"],
                                  (ng, njp, njc, ncell))
    if dev_build:
        log("device list build: %.2f ms (host %.3f s)" % (dev_build["ms"], t_build))

    roofline = None
    if kernel in FLOPS_PC:
        flops = FLOPS_PP * n_pp + FLOPS_PC[kernel] * n_pc
    else:
        flops = FLOPS_SPLIT_PP * live[0] + FLOPS_SPLIT_PC[kernel] * live[1]
    achieved = flops / (ms_kern * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": (profiled_traffic() if args.workload == "cube"
                            and kernel == bhq.QUAD else None)}
    if kernel not in FLOPS_PC:
        roofline["priced_on"] = "pairs inside the cutoff (bhq_count_live)"

    cpu = None
    if not args.no_cpu_baseline and args.workload == "cube":
        log("timing the oracle on the host ...")
        cpu = cpu_baseline(W, a32, host_info())

    configs = None
    if not args.no_configs and args.workload == "cube":
        log("other configurations ...")
        configs = other_configs(torch, stream, args.steps, cpu=not args.no_cpu_baseline)

    out = {
        "metric": METRIC,
        "value": round(n_int / (ms_step * 1e-3) / 1e9, 3),
        "unit": "Ginteractions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": W["name"] + ", ncrit=%d; %s kernel, FP32 with "
                   "FP64 group offsets" % (W["ncrit"], bhq.KERNEL_NAMES[kernel]),
                   "n": n, "theta": W["theta"], "ncrit": W["ncrit"],
                   "groups": ng, "n_pp": n_pp, "n_pc": n_pc,
                   "lists": args.lists, "autotuned": tuned,
                   "launch": {"block": args.block, "i_per_thread": args.ipt,
                              "persistent": args.persistent,
                              "graph": args.graph, "jsplit": args.jsplit,
                              "waves_per_eu": args.waves_per_eu,
                              "order": args.order,
                              "order_window": args.order_window,
                              "order_tail": args.order_tail}},
        "s_per_force_eval": round(ms_step * 1e-3, 6),
        "kernel_ms": round(ms_kern, 4), "kernel_ms_median": round(ms_kern_med, 4),
        "pc_Ginteractions_per_s": round(n_pc / (ms_kern * 1e-3) / 1e9, 3),
        "paper_convention_gflops": (round(PAPER_FLOPS_PC * n_pc / (ms_kern * 1e-3) / 1e9, 1)
                                    if kernel == bhq.QUAD else None),
        "sclk_mhz": round(sclk, 1) if sclk else None,
        "live_pairs": ({"pp": live[0], "pc": live[1],
                        "Ginteractions_per_s": round(sum(live) / (ms_kern * 1e-3) / 1e9, 3)}
                       if live else None),
        "lane_slot_fraction": round(lane_slots, 4),
        "host_list_build_s": round(t_build, 3), "upload_s": round(t_upload, 3),
        "device_list_build": dev_build,
        "treepm": treepm,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
        "configs": configs,
    }
    out.update(out_extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
