"""Autotuner: the search picks the fastest measured configuration and the
cache returns it again (CPU, with a stand-in timing function); on the GPU
the tuned configuration still matches the oracle."""
import numpy as np
import pytest

import oracle as orc
from _parity import assert_parity, errors, log
from paper_1812_07313_amd import bhq, synth, tune


def test_search_picks_minimum_and_cache_roundtrip(tmp_path):
    cost = {64: 3.0, 128: 2.0, 256: 2.5}

    def measure(nc, c):
        return (cost[nc] + (0.1 if c["block"] == 128 else 0.0) - 0.05 * c["persistent"]
                - 0.01 * c["i_per_thread"] - 0.001 * (c["order"] == bhq.ORDER_COST)
                - 0.002 * c["use_graph"] + 0.0001 * c["jsplit"]
                - 0.0003 * (c["waves_per_eu"] == 6))

    best, table = tune.search(measure, jsplits=tune.SMALL_JSPLITS)
    n256 = sum(1 for s in tune.SHAPES if s[0] == 256)
    assert len(table) == (len(tune.NCRITS) * (n256 * len(tune.WAVES) + len(tune.SHAPES) - n256)
                          * len(tune.ORDERS) * len(tune.SMALL_JSPLITS))
    assert all(r["waves_per_eu"] == 0 for r in table if r["block"] == 128)
    assert best["ncrit"] == 128 and best["block"] == 256 and best["persistent"] == 1
    assert best["i_per_thread"] == 2 and best["order"] == bhq.ORDER_COST
    assert best["use_graph"] == 1 and best["jsplit"] == 1 and best["waves_per_eu"] == 6
    assert best["seconds"] == min(r["seconds"] for r in table)
    path = str(tmp_path / "tune.json")
    key = tune.cache_key("gfx950", "w", bhq.QUAD, bhq.FP32_OFS64, 0.6)
    tune._store(path, {key: {"best": best, "table": table}})
    assert tune._load(path)[key]["best"] == best
    assert tune._load(str(tmp_path / "missing.json")) == {}


@pytest.mark.gpu
def test_autotune_batched_systems_parity(tmp_path):
    systems = synth.batched_plummer(16, lo=10.0, hi=12.0)
    sizes = np.array([len(s[1]) for s in systems])
    off = np.concatenate([[0], np.cumsum(sizes)])
    X = np.concatenate([s[0] for s in systems])
    M = np.concatenate([s[1] for s in systems])
    E2 = np.concatenate([np.full(len(s[1]), s[2] ** 2) for s in systems])
    ctx = bhq.bhq_create(0, bhq.QUAD, bhq.FP32_OFS64)
    try:
        path = str(tmp_path / "tune.json")
        log("case autotune batched %d particles" % len(M))
        r = tune.autotune(ctx, X, M, 0.6, "test-batched", cache=path,
                          ncrits=(64, 128), eps2_per_particle=E2, sys_off=off,
                          jsplits=(1, 2), repeats=2)
        assert not r["cached"]
        best = r["best"]
        log("  best %s" % best)
        # the context now holds the best lists and shape: check them
        a_ref = np.zeros((len(M), 3))
        p_ref = np.zeros(len(M))
        for s, (x, m, eps) in enumerate(systems):
            T = orc.Tree(x, m, 0.6, best["ncrit"])
            mat = orc.materialise(T, x, m)
            a, p = orc.eval_lists(orc.QUAD, mat, x, eps * eps)
            a_ref[off[s]:off[s + 1]] = a
            p_ref[off[s]:off[s + 1]] = p
        L = bhq.bhq_build_lists_batch(off, X, M, 0.6, best["ncrit"])
        idx = bhq.bhq_lists_export(L, len(M))["i_idx"]
        bhq.bhq_lists_free(L)
        bhq.bhq_compute(ctx)
        a_g, p_g = bhq.bhq_get_result(ctx, len(M))
        a = np.zeros_like(a_g)
        p = np.zeros_like(p_g)
        a[idx] = a_g
        p[idx] = p_g
        assert_parity(errors(a, p, a_ref, p_ref), bhq.FP32_OFS64, "autotuned")
        r2 = tune.autotune(ctx, X, M, 0.6, "test-batched", cache=path,
                           ncrits=(64, 128), eps2_per_particle=E2, sys_off=off,
                           jsplits=(1, 2))
        assert r2["cached"] and r2["best"] == best
    finally:
        bhq.bhq_destroy(ctx)
