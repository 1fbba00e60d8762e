"""Parity of the HIP path (through the C ABI) with the CPU oracle: bit-exact
for every integer output (CSR arrays, kept edge sets, counts, splits, q_l) and
bitwise-equal doubles for the rescaled estimates (same IEEE operations)."""
import math
import sys

import numpy as np
import pytest

import light_schedule
import oracle
import synth
from synth import special

pytestmark = pytest.mark.gpu

SPLITS = [(1, 1), (1, 2), (2, 1), (0, 1), (1000, 1)]


def _log(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def _build(tc, graph, host=False):
    n, s, d = graph
    if host:
        return tc.tc_build_csr(n, s, d)
    return tc.tc_build_csr(n, _dev(s), _dev(d))


def _csr_equal(tc, g, og):
    rp, col, deg = tc.tc_graph_read(g)
    n, orp, ocol = og
    assert np.array_equal(rp.astype(np.int64), orp)
    assert np.array_equal(col, ocol)
    assert np.array_equal(deg.astype(np.int64), np.diff(orp))


def _graphs():
    return {
        "cl16k": synth.workload("cl16k"),
        "multi_loops": synth.uniform_pairs(300, 5000, 3),
        "k5": special.complete(5),
        "k65": special.complete(65),
        "wheel12": special.wheel(12),
        "petersen": special.petersen(),
        "friend9": special.friendship(9),
        "isolated": (50, np.array([3, 3, 7], np.int32), np.array([9, 3, 40], np.int32)),
        "empty": (10, np.zeros(0, np.int32), np.zeros(0, np.int32)),
        "one_vertex": (1, np.zeros(0, np.int32), np.zeros(0, np.int32)),
        "cl_dense": synth.chung_lu(3000, 120.0, 2.1, seed=5),
    }


GRAPHS = _graphs()


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_csr_build_matches_oracle(gpu, name):
    _log("csr %s" % name)
    g = _build(gpu, GRAPHS[name])
    _csr_equal(gpu, g, oracle.normalise(*GRAPHS[name]))


def test_csr_build_from_host_pointers(gpu):
    g = _build(gpu, GRAPHS["cl16k"], host=True)
    _csr_equal(gpu, g, oracle.normalise(*GRAPHS["cl16k"]))


def test_csr_rejects_out_of_range_ids(gpu):
    with pytest.raises(gpu.TcError) as e:
        gpu.tc_build_csr(5, _dev([0, 1, 5]), _dev([1, 2, 3]))
    assert e.value.status == 1
    with pytest.raises(gpu.TcError):
        gpu.tc_build_csr(5, _dev([0, -1]), _dev([1, 2]))


@pytest.mark.parametrize("p,seed", [(0.25, 0), (0.5, 1), (0.1, 2), (1.0, 3), (0.05, 4)])
def test_sample_matches_oracle(gpu, p, seed):
    _log("sample p=%g seed=%d" % (p, seed))
    G = GRAPHS["cl16k"]
    g = _build(gpu, G)
    og = oracle.normalise(*G)
    gs = gpu.tc_sample(g, p, seed)
    _csr_equal(gpu, gs, oracle.sample(og, p, seed))


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_exact_count_and_split_match_oracle(gpu, name):
    G = GRAPHS[name]
    g = _build(gpu, G)
    og = oracle.normalise(*G)
    for a, b in SPLITS:
        _log("count %s split %d/%d" % (name, a, b))
        got = gpu.tc_count_exact(g, heavy=(a, b))
        want = oracle.count_split(og, a, b)
        for k in ("triangles", "light", "heavy", "n_heavy", "m"):
            assert got[k] == want[k], (name, a, b, k, got, want)


@pytest.mark.parametrize("n", [3, 4, 31, 32, 33, 64, 100, 300])
def test_complete_graphs_all_heavy_and_all_light(gpu, n):
    G = special.complete(n)
    g = _build(gpu, G)
    for a, b in [(0, 1), (1000, 1), (1, 1)]:
        _log("K_%d split %d/%d" % (n, a, b))
        r = gpu.tc_count_exact(g, heavy=(a, b))
        assert r["triangles"] == math.comb(n, 3)
        if a == 0:
            assert r["heavy"] == math.comb(n, 3) and r["n_heavy"] == n
        if a == 1000:
            assert r["heavy"] == 0


@pytest.mark.parametrize("p", [0.25, 0.5, 0.1])
def test_estimate_matches_oracle(gpu, p):
    G = GRAPHS["cl16k"]
    g = _build(gpu, G)
    og = oracle.normalise(*G)
    seeds = list(range(8))
    _log("estimate p=%g" % p)
    per, ests, mom = gpu.tc_estimate(g, p, seeds, num_groups=4)
    counts = []
    for s, c, e in zip(seeds, per, ests):
        w = oracle.count_split(oracle.sample(og, p, s))
        for k in ("triangles", "light", "heavy", "n_heavy", "m"):
            assert c[k] == w[k], (s, k)
        assert e == oracle.estimate(w["triangles"], p)
        counts.append(w["triangles"])
    assert mom == oracle.median_of_means(counts, 4, p)


def test_estimate_p1_is_exact_count(gpu):
    G = GRAPHS["cl_dense"]
    g = _build(gpu, G)
    per, ests, mom = gpu.tc_estimate(g, 1.0, [0, 1])
    exact = gpu.tc_count_exact(g)
    assert per[0]["triangles"] == exact["triangles"] == per[1]["triangles"]
    assert ests[0] == float(exact["triangles"])


def test_rp_matches_oracle(gpu):
    G = synth.chung_lu(2000, 14.0, 2.4, seed=3)
    g = _build(gpu, G)
    og = oracle.normalise(*G)
    for k, seed in [(64, 0), (130, 5)]:
        _log("rp k=%d seed=%d" % (k, seed))
        q, est = gpu.tc_rp_trace(g, k, seed)
        oq, oest = oracle.rp_trace(og, k, seed)
        assert np.array_equal(q, oq)
        assert est == oest


@pytest.mark.parametrize("name", ["empty", "one_vertex", "isolated", "k65", "star4096", "star4097"])
@pytest.mark.parametrize("k", [1, 3, 64])
def test_rp_edge_cases(gpu, name, k):
    # K_65 has 4160 CSR entries: its rows of 64 end exactly at the 4096-entry
    # sweep-range boundary; the centre row of star4096 fills one whole range,
    # that of star4097 spills one entry into the next
    if name.startswith("star"):
        N = int(name[4:])
        G = (N + 1, np.zeros(N, np.int32), np.arange(1, N + 1, dtype=np.int32))
    else:
        G = GRAPHS[name]
    _log("rp edge case %s k=%d" % (name, k))
    g = _build(gpu, G)
    q, est = gpu.tc_rp_trace(g, k, 11)
    oq, oest = oracle.rp_trace(oracle.normalise(*G), k, 11)
    assert np.array_equal(q, oq)
    assert est == oest


def test_rp_star_bound_and_overflow(gpu):
    # star K_{1,N}: sum over CSR entries of deg_i deg_j = 2 N^2; k * 2^33 >= 2^62
    # must be refused before any q is returned, a small k must match the oracle
    # (the row of the centre spans many 4096-entry sweep ranges)
    N = 65536
    src = np.zeros(N, np.int32)
    dst = np.arange(1, N + 1, dtype=np.int32)
    g = _build(gpu, (N + 1, src, dst))
    with pytest.raises(gpu.TcError) as e:
        gpu.tc_rp_trace(g, 1 << 30, 0)
    assert "overflow" in str(e.value).lower() or "2^62" in str(e.value)
    og = oracle.normalise(N + 1, src, dst)
    q, est = gpu.tc_rp_trace(g, 70, 9)
    oq, oest = oracle.rp_trace(og, 70, 9)
    assert np.array_equal(q, oq)
    assert est == oest


def test_invalid_p_and_groups(gpu):
    g = _build(gpu, special.complete(5))
    for p in (0.0, -0.1, 1.5, float("nan"), float("inf")):
        with pytest.raises(gpu.TcError):
            gpu.tc_estimate(g, p, [0])
        with pytest.raises(gpu.TcError):
            gpu.tc_sample(g, p, 0)
    with pytest.raises(gpu.TcError):
        gpu.tc_estimate(g, 0.5, [0, 1, 2], num_groups=2)


TUNINGS = [dict(vmajor_cap=0, small_dmax=128), dict(vmajor_cap=1024, small_dmax=128),
           dict(vmajor_cap=4, small_dmax=32), dict(vmajor_cap=1 << 30, small_dmax=128),
           dict(vmajor_cap=1 << 30, small_dmax=1), dict(vmajor_cap=0, small_dmax=1)]


@pytest.mark.parametrize("name", ["cl16k", "cl_dense", "k65", "multi_loops", "wheel12"])
def test_counts_invariant_under_launch_tunings(gpu, name):
    G = GRAPHS[name]
    g = _build(gpu, G)
    og = oracle.normalise(*G)
    want = oracle.count_split(og, 1, 1)
    for p in (1.0, 0.5):
        wp = want if p == 1.0 else oracle.count_split(oracle.sample(og, p, 3), 1, 1)
        for t in TUNINGS:
            _log("tuning %s p=%g %r" % (name, p, t))
            gpu.tc_tune_set(g, p, heavy=(1, 1), blocks_per_cu=2, **t)
            if p == 1.0:
                got = gpu.tc_count_exact(g, tuned=True)
            else:
                got = gpu.tc_estimate(g, p, [3], tuned=True)[0][0]
            for k in ("triangles", "light", "heavy", "n_heavy", "m"):
                assert got[k] == wp[k], (name, p, t, k, got[k], wp[k])
            sched = light_schedule.light_work(og if p == 1.0 else oracle.sample(og, p, 3), 1, 1, t["vmajor_cap"])
            assert (got["probes"], got["gather"]) == (sched["probes"], sched["gather"]), (name, p, t, sched)


@pytest.mark.parametrize("vcap", [0, 1024, 1 << 30])
def test_long_out_lists_sorted_and_unsorted(gpu, vcap):
    # K_1100, all light: out-lists of every length up to 1099, so lists of the
    # register sort (<= 64), of the LDS sort (65..1024) and unsorted ones
    # (> 1024) all occur; exact count and the schedule's work statistics
    n = 1100
    G = special.complete(n)
    g = _build(gpu, G)
    og = oracle.normalise(*G)
    gpu.tc_tune_set(g, 1.0, heavy=(1000, 1), vmajor_cap=vcap, small_dmax=128, blocks_per_cu=2)
    _log("K_1100 vcap=%d" % vcap)
    got = gpu.tc_count_exact(g, tuned=True)
    assert got["triangles"] == got["light"] == math.comb(n, 3) and got["n_heavy"] == 0
    sched = light_schedule.light_work(og, 1000, 1, vcap)
    assert (got["probes"], got["gather"]) == (sched["probes"], sched["gather"]), sched
    for p, seed in ((0.5, 7), (0.9, 8)):
        gpu.tc_tune_set(g, p, heavy=(1000, 1), vmajor_cap=vcap, small_dmax=128, blocks_per_cu=2)
        gs = oracle.sample(og, p, seed)
        r = gpu.tc_estimate(g, p, [seed], tuned=True)[0][0]
        assert r["triangles"] == oracle.count(gs)
        s2 = light_schedule.light_work(gs, 1000, 1, vcap)
        assert (r["probes"], r["gather"]) == (s2["probes"], s2["gather"]), (p, s2)


def test_autotune_keeps_the_count(gpu):
    G = GRAPHS["cl_dense"]
    g = _build(gpu, G)
    og = oracle.normalise(*G)
    best = gpu.tc_autotune(g, 0.5, seed=1, search_heavy=True)
    assert best == gpu.tc_tune_get(g, 0.5)
    got = gpu.tc_estimate(g, 0.5, [1], tuned=True)[0][0]
    assert got["triangles"] == oracle.count(oracle.sample(og, 0.5, 1))
    a, b = best["heavy_num"], best["heavy_den"]
    assert (a, b) in {(1, 4), (1, 2), (1, 1), (2, 1)}
    assert got["heavy"] == oracle.count_split(oracle.sample(og, 0.5, 1), a, b)["heavy"]
