"""Autotuner for the force evaluation: chooses the group size bound ncrit
(which changes the interaction lists; the paper's n_crit, Sec. 3.4), the
launch shape (block size = LDS tile depth, i-particles per thread, persistent
queue and its grid size = resident blocks per CU, HIP graph replay, the
cross-block j-split for inputs with too few groups to fill the GPU, and the
occupancy: kernel instances whose registers are capped for 6 or 8 waves per
SIMD) and the group dispatch order that minimise the time of one force
evaluation.
Interactions per second alone would reward larger ncrit (more, cheaper
interactions), so the objective is seconds per evaluation.

Results are cached in a JSON file keyed by device architecture, a caller
supplied workload key, kernel, precision and theta, so that a repeated
call returns the stored choice without measuring again.
"""
import json
import os
import time

import numpy as np

from . import bhq

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "bhq",
                             "tune.json")

NCRITS = (64, 128, 256)
# launch shapes: (block, i_per_thread, blocks_per_cu, persistent, use_graph)
SHAPES = ((256, 1, 0, 0, 0), (256, 2, 0, 0, 0), (128, 1, 0, 0, 0), (128, 2, 0, 0, 0),
          (256, 1, 0, 1, 0), (256, 2, 0, 1, 0), (128, 2, 4, 1, 0),
          (256, 1, 0, 1, 1), (256, 2, 0, 1, 1), (256, 2, 0, 0, 1))
# waves per SIMD the registers must allow (0: the compiler's choice); the
# capped instances exist for block 256
WAVES = (0, 6, 8)
JSPLITS = (1,)
SMALL_JSPLITS = (1, 2, 4, 8)   # for inputs of a few hundred groups
ORDERS = (bhq.ORDER_XCD, bhq.ORDER_COST)
KNOBS = ("block", "i_per_thread", "blocks_per_cu", "persistent", "use_graph")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, db):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cache_key(arch, workload, kernel, precision, theta):
    return "%s|%s|%s|%s|theta=%.4g" % (arch, workload,
                                        bhq.KERNEL_NAMES[kernel],
                                        bhq.PRECISION_NAMES[precision], theta)


def search(measure, ncrits=NCRITS, shapes=SHAPES, orders=ORDERS, jsplits=JSPLITS,
           waves=WAVES):
    """Exhaustive search.  measure(ncrit, cfg) with cfg a dict of the launch
    knobs (block, i_per_thread, blocks_per_cu, persistent, use_graph, jsplit,
    waves_per_eu, order) returns seconds per evaluation; waves_per_eu other
    than 0 is tried for block 256 only.  Returns (best, table)."""
    table = []
    for nc in ncrits:
        for shape in shapes:
            for w in (waves if shape[0] == 256 else (0,)):
                for js in jsplits:
                    for order in orders:
                        cfg = dict(zip(KNOBS, shape), jsplit=js, waves_per_eu=w, order=order)
                        t = measure(nc, cfg)
                        table.append(dict(cfg, ncrit=nc, seconds=t))
    best = min(table, key=lambda r: r["seconds"])
    return dict(best), table


def apply(ctx, cfg):
    """Set a configuration's launch knobs and order on ctx."""
    bhq.bhq_set_tuning(ctx, cfg["block"], cfg["i_per_thread"], cfg["blocks_per_cu"],
                       cfg["persistent"], cfg.get("use_graph", 0), cfg.get("jsplit", 1),
                       cfg.get("waves_per_eu", 0))
    bhq.bhq_set_group_order(ctx, cfg["order"])


def gpu_measure(ctx, x, m, theta, kernel=bhq.QUAD, precision=bhq.FP32_OFS64,
                eps=None, eps2_per_particle=None, sys_off=None, box=0.0,
                rcut=0.0, rs=0.0, repeats=5, stream=None, indexed=True):
    """A measure() for search(): builds the lists for each ncrit once (host
    builder), uploads them to ctx and times bhq_compute with HIP events
    (median of `repeats` launches after one warm-up)."""
    state = {"ncrit": None}

    def measure(ncrit, cfg):
        if state["ncrit"] != ncrit:
            if sys_off is not None:
                L = bhq.bhq_build_lists_batch(sys_off, x, m, theta, ncrit,
                                              nleaf=min(8, ncrit))
            else:
                L = bhq.bhq_build_lists(x, m, theta, ncrit,
                                        nleaf=min(8, ncrit), box=box, rcut=rcut)
            try:
                if indexed:
                    bhq.bhq_set_lists_indexed(ctx, L, x, m)
                else:
                    bhq.bhq_set_lists(ctx, L, x, m)
                idx = bhq.bhq_lists_export(L, len(m))["i_idx"]
            finally:
                bhq.bhq_lists_free(L)
            if eps2_per_particle is not None:
                bhq.bhq_set_eps2_i(ctx, np.asarray(eps2_per_particle)[idx])
            elif eps is not None:
                bhq.bhq_set_eps(ctx, eps)
            if rs:
                bhq.bhq_set_split(ctx, rs, rcut, box)
            state["ncrit"] = ncrit
        bhq.bhq_set_kernel(ctx, kernel, precision)
        apply(ctx, cfg)
        bhq.bhq_compute(ctx, stream)
        bhq.bhq_get_kernel_ms(ctx)
        ts = []
        for _ in range(repeats):
            bhq.bhq_compute(ctx, stream)
            ts.append(bhq.bhq_get_kernel_ms(ctx))
        return float(np.median(ts)) * 1e-3

    return measure


def autotune(ctx, x, m, theta, workload, arch="gfx950", kernel=bhq.QUAD,
             precision=bhq.FP32_OFS64, cache=DEFAULT_CACHE, ncrits=NCRITS,
             shapes=SHAPES, orders=ORDERS, jsplits=JSPLITS, waves=WAVES, force=False,
             **kw):
    """Tune (or read from the cache) and leave ctx holding the best lists
    and launch shape.  Returns dict(best=..., table=..., cached=bool)."""
    key = cache_key(arch, workload, kernel, precision, theta)
    db = _load(cache)
    measure = gpu_measure(ctx, x, m, theta, kernel=kernel, precision=precision,
                          **kw)
    if not force and key in db and "waves_per_eu" in db[key]["best"]:
        best = db[key]["best"]
        measure(best["ncrit"], best)
        return dict(best=best, table=db[key]["table"], cached=True)
    t0 = time.perf_counter()
    best, table = search(measure, ncrits, shapes, orders, jsplits, waves)
    db = _load(cache)
    db[key] = dict(best=best, table=table, seconds_spent=time.perf_counter() - t0)
    _store(cache, db)
    measure(best["ncrit"], best)
    return dict(best=best, table=table, cached=False)
