"""The test-side model of the light phase's schedule (light_schedule.py),
which the GPU tests hold the work statistics to, against the rule written out
with plain loops on small graphs, and the bound that makes the rank-ordered
suffix worthwhile: summed over the pairs, the shorter streamed list never
exceeds the wedge count."""
import itertools

import numpy as np
import pytest

import light_schedule
import oracle
import synth
from synth import special


def _loops(g, a, b, vcap, sort_cap):
    n, rp, col = g
    adj = [list(col[rp[x]:rp[x + 1]]) for x in range(n)]
    deg = [len(l) for l in adj]
    m = sum(deg) // 2
    rank = lambda x: (deg[x], x)
    up = [sorted((y for y in adj[x] if rank(x) < rank(y)), key=rank) for x in range(n)]
    probes = gather = 0
    for u in range(n):
        heavy = deg[u] > 0 and b * b * deg[u] * deg[u] > a * a * m
        d = len(up[u])
        if heavy or d < 2:
            continue
        for k, v in enumerate(up[u]):
            dv = len(up[v])
            gather += dv
            ln = d - 1 - k if d <= sort_cap else d
            if ln == 0:
                continue
            probes += ln if ln <= dv <= vcap else dv
    return probes, gather


GRAPHS = {
    "k9": special.complete(9),
    "wheel15": special.wheel(15),
    "friend6": special.friendship(6),
    "kpart": special.complete_multipartite([3, 4, 5]),
    "gnm": synth.uniform_pairs(60, 500, 5),
    "cl": synth.chung_lu(400, 10.0, 2.2, seed=3),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("vcap", [0, 3, 1 << 30])
@pytest.mark.parametrize("split", [(1, 1), (1000, 1), (1, 4)])
def test_model_equals_loops(name, vcap, split):
    g = oracle.normalise(*GRAPHS[name])
    for cap in (light_schedule.SORT_CAP, 4):  # 4: some lists stay unsorted
        got = light_schedule.light_work(g, split[0], split[1], vcap, sort_cap=cap)
        assert (got["probes"], got["gather"]) == _loops(g, split[0], split[1], vcap, cap)


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_suffix_work_bounded_by_wedges(name):
    g = oracle.normalise(*GRAPHS[name])
    n, rp, col = g
    deg = np.diff(np.asarray(rp, np.int64))
    key = deg * n + np.arange(n)
    row = np.repeat(np.arange(n), deg)
    up = key[row] < key[np.asarray(col, np.int64)]
    dplus = np.bincount(row[up], minlength=n)
    wedges = int((dplus * (dplus - 1) // 2).sum())
    # all vertices light, every pair free to take the shorter list
    w = light_schedule.light_work(g, 1, 0, 1 << 30)
    assert w["probes"] <= wedges
