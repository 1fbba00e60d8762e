"""CPU pins of the oracle's semi-streaming variant (section 5.2): the triple
set U and its closure against brute force, |U| and the pass-1 draw count in
closed form, the candidate Lemma, unbiasedness over many seeds, and
triangle-free graphs."""
import math

import numpy as np
import pytest

import oracle
import synth


def _graphs():
    gs = {}
    n = 9
    gs["k9"] = oracle.normalise(n, *[a.astype(np.int32) for a in np.triu_indices(n, 1)])
    # wheel: hub 0 joined to a 12-cycle 1..12
    s = [0] * 12 + list(range(1, 13))
    d = list(range(1, 13)) + list(range(2, 13)) + [1]
    gs["wheel"] = oracle.normalise(13, np.array(s, np.int32), np.array(d, np.int32))
    gs["gnm"] = oracle.normalise(*synth.uniform_pairs(40, 300, seed=5))
    gs["cl"] = oracle.normalise(*synth.chung_lu(120, 10.0, 2.3, seed=2))
    return gs


GRAPHS = _graphs()


def _brute(g):
    return oracle.count_bruteforce(oracle.dense_adjacency(g))


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_every_triangle_has_three_closed_elements(name):
    # for any heavy set H, the closed elements of U (wedges at vertices
    # outside H, (vertex of H, edge) pairs) number exactly 3 t
    g = GRAPHS[name]
    n = g[0]
    T = _brute(g)
    rng = np.random.default_rng(7)
    for frac in (0.0, 0.2, 0.5, 1.0):
        heavy = rng.random(n) < frac
        assert oracle.stream_closed_all(g, heavy) == 3 * T, (name, frac)


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_sizes_in_closed_form(name):
    g = GRAPHS[name]
    n, rp, col = g
    m = len(col) // 2
    deg = np.diff(rp)
    for d, s, seed in ((1.0, 50, 0), (3.0, 200, 11)):
        r, heavy = oracle.stream_estimate(g, d, s, seed)
        assert r["m"] == m
        want_draws = math.ceil(d * math.sqrt(m) * math.log(n)) if n >= 2 and m >= 1 else 0
        assert r["draws1"] == want_draws
        # H holds only candidates above the split, |U| = |L| + |H| m
        assert all(int(deg[x]) ** 2 > m for x in np.nonzero(heavy)[0])
        L = sum(int(deg[u]) * (int(deg[u]) - 1) // 2 for u in range(n) if not heavy[u])
        assert r["heavy"] == int(heavy.sum()) and r["light_size"] == L
        assert r["size"] == L + r["heavy"] * m
        assert r["candidates"] >= r["heavy"]
        assert 0 <= r["closed"] <= s and r["queries"] <= 2 * s


def test_candidates_find_every_heavy_vertex():
    # the Lemma of section 5.2: with d m^(1/2) ln n draws every vertex of
    # degree above m^(1/2) is an endpoint of a drawn edge with probability at
    # least 1 - n^(1-d)
    for seed in range(5):
        g = oracle.normalise(*synth.chung_lu(3000, 16.0, 2.1, seed=seed + 1))
        n, rp, col = g
        m = len(col) // 2
        deg = np.diff(rp)
        want = {int(x) for x in np.nonzero(deg.astype(np.int64) ** 2 > m)[0]}
        assert want
        r, heavy = oracle.stream_estimate(g, 3.0, 10, seed)
        assert set(int(x) for x in np.nonzero(heavy)[0]) == want


def test_mean_is_unbiased():
    g = oracle.normalise(*synth.chung_lu(300, 14.0, 2.3, seed=9))
    T = _brute(g)
    s = 400
    ests = np.array([oracle.stream_estimate(g, 2.0, s, seed)[0]["estimate"] for seed in range(300)])
    se = ests.std(ddof=1) / math.sqrt(len(ests))
    assert abs(ests.mean() - T) < 5 * se, (ests.mean(), T, se)


def test_triangle_free_graphs_close_nothing():
    n = 40
    s = np.arange(n, dtype=np.int32)
    cyc = oracle.normalise(n, s, (s + 1) % n)
    a, b = np.meshgrid(np.arange(10), np.arange(10, 25))
    bip = oracle.normalise(25, a.ravel().astype(np.int32), b.ravel().astype(np.int32))
    for g in (cyc, bip):
        for seed in range(5):
            r, _ = oracle.stream_estimate(g, 3.0, 500, seed)
            assert r["closed"] == 0 and r["estimate"] == 0.0
