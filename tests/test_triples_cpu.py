"""Pins of the oracle's triple sampling (section 3.2, "Triple Sampling"; the
Simple and Hybrid columns of Table 2) against facts that do not come from the
oracle: triangle counts by brute force over all vertex triples, the size of U
in closed form, U's order enumerated independently, the exact estimate on
complete graphs, unbiasedness over seeds; and the C ABI's argument checks."""
import ctypes
import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from paper_1011_0468_amd import _native
from synth import special

SMALL = {"k6": special.complete(6), "wheel9": special.wheel(9), "friend4": special.friendship(4),
         "kpart": special.complete_multipartite([2, 3, 4]), "gnm": synth.uniform_pairs(40, 260, 2),
         "cl": synth.chung_lu(120, 8.0, 2.1, seed=4), "star": special.star(12), "cycle": special.cycle(9)}


def _adj(g):
    n, rp, col = g
    return [set(int(c) for c in col[rp[x]:rp[x + 1]]) for x in range(n)], [list(col[rp[x]:rp[x + 1]]) for x in range(n)]


def _brute_T(g):
    sets, _ = _adj(g)
    return sum(1 for a, b, c in itertools.combinations(range(g[0]), 3) if b in sets[a] and c in sets[a] and c in sets[b])


def _enumerate_U(g, hybrid):
    # U in its documented order, with the closed flag and the weight
    n, rp, col = g
    sets, lists = _adj(g)
    m = len(col) // 2
    ext = [hybrid and len(lists[x]) ** 2 > m for x in range(n)]
    out = []
    for u in range(n):
        L = lists[u]
        if not ext[u]:
            for b in range(len(L)):  # colex: b outer, a inner
                for a in range(b):
                    x, y, z = L[a], u, L[b]
                    out.append(((x, y, z), z in sets[x]))
        else:
            for v in L:
                for w in lists[v]:
                    out.append(((u, v, w), w != u and w in sets[u]))
    res = []
    for (x, y, z), closed in out:
        res.append(((x, y, z), 60 // (3 + ext[x] + ext[y] + ext[z]) if closed else 0))
    return res


@pytest.mark.parametrize("name", sorted(SMALL))
@pytest.mark.parametrize("hybrid", [False, True])
def test_U_order_and_weights_match_enumeration(name, hybrid):
    g = oracle.normalise(*SMALL[name])
    size, pre = oracle.triples_size(g, hybrid, with_prefix=True)
    want = _enumerate_U(g, hybrid)
    assert size == len(want)
    got = [oracle.triple_at(g, hybrid, pre, r) for r in range(size)]
    assert got == want
    # every triangle's appearances weigh 60 in all
    assert sum(w for _, w in want) == 60 * _brute_T(g)


def test_U_size_closed_forms():
    for n in (3, 5, 8):
        g = oracle.normalise(*special.complete(n))
        assert oracle.triples_size(g, False) == n * math.comb(n - 1, 2)
        assert oracle.triples_size(g, True) == n * (n - 1) ** 2  # deg^2 > m for every vertex
    g = oracle.normalise(*special.star(10))  # 9 leaves; centre: 9^2 > m = 9; leaves: no wedges
    assert oracle.triples_size(g, False) == math.comb(9, 2)
    assert oracle.triples_size(g, True) == 9


@pytest.mark.parametrize("n", [4, 7, 12])
def test_simple_estimate_is_exact_on_complete_graphs(n):
    g = oracle.normalise(*special.complete(n))
    for s, seed in ((1, 0), (17, 3), (1000, 9)):
        size, wsum, closed = oracle.triple_sample(g, False, s, seed)
        assert closed == s and wsum == 20 * s
        assert oracle.triple_estimate(size, wsum, s) == math.comb(n, 3)


@pytest.mark.parametrize("hybrid", [False, True])
def test_estimate_is_unbiased_over_seeds(hybrid):
    g = oracle.normalise(*synth.chung_lu(300, 12.0, 2.1, seed=8))
    T = _brute_T(g) if g[0] <= 0 else oracle.count_bruteforce(oracle.dense_adjacency(g))
    s = 400
    est = [oracle.triple_estimate(*oracle.triple_sample(g, hybrid, s, seed)[:2], s) for seed in range(300)]
    se = np.std(est) / math.sqrt(len(est))
    assert abs(np.mean(est) - T) < 5 * se


def test_triangle_free_graph_estimates_zero():
    g = oracle.normalise(*special.complete_multipartite([5, 7]))  # bipartite
    for hybrid in (False, True):
        size, wsum, closed = oracle.triple_sample(g, hybrid, 500, 1)
        assert size > 0 and wsum == 0 and closed == 0


def test_sample_indices_in_range_and_spread():
    size = 1000003
    idx = [oracle.triple_index(5, i, size) for i in range(20000)]
    assert min(idx) >= 0 and max(idx) < size
    hist = np.bincount(np.array(idx) * 10 // size, minlength=10)
    assert hist.min() > 1700 and hist.max() < 2300


def test_abi_rejects_bad_arguments():
    L = _native.load()
    r = _native.TcTripleResult()
    assert L.tc_triple_estimate(None, 1.0, 0, 0, 10, 0, None, ctypes.byref(r)) == _native.TC_ERR_INVALID
