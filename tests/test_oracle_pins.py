"""Pins of the CPU oracle against facts fixed outside the oracle itself:
published SplitMix64 outputs, closed-form triangle counts, brute force on tiny
graphs, dense linear algebra (trace of A^3), statistical laws of the edge coin
and of the Rademacher projection, and hand-worked median-of-means cases."""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
import synth
from synth import special

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def _set_graph(n, src, dst):
    """Plain definition of the simple undirected graph: a set of 2-sets."""
    return {frozenset((int(u), int(v))) for u, v in zip(src, dst) if u != v}


def _dense(n, edges):
    A = np.zeros((n, n), np.int64)
    for e in edges:
        u, v = tuple(e)
        A[u, v] = A[v, u] = 1
    return A


def _brute(n, edges):
    """All vertex triples, checked one by one."""
    E = edges
    t = 0
    for a, b, c in itertools.combinations(range(n), 3):
        if frozenset((a, b)) in E and frozenset((b, c)) in E and frozenset((a, c)) in E:
            t += 1
    return t


# ---------------------------------------------------------------- hash ----

def test_mix64_matches_published_splitmix64_outputs():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) if not l.startswith("#")]
    assert len(rows) == 5
    for k, out in rows:
        assert oracle.mix64((int(k) * GAMMA) & M64) == int(out, 16)


def test_keep_threshold_values():
    assert oracle.keep_threshold(1.0) == 1 << 53
    assert oracle.keep_threshold(0.5) == 1 << 52
    assert oracle.keep_threshold(0.25) == 1 << 51
    assert oracle.keep_threshold(0.1) == math.floor(0.1 * 2 ** 53)


# ------------------------------------------------------------ normalise ----

@pytest.mark.parametrize("seed", [1, 2, 3])
def test_normalise_matches_set_definition(seed):
    n, s, d = synth.uniform_pairs(40, 300, seed)
    g = oracle.normalise(n, s, d)
    E = _set_graph(n, s, d)
    _, rp, col = g
    assert rp[n] == 2 * len(E)
    got = set()
    for u in range(n):
        row = col[rp[u]:rp[u + 1]]
        assert np.all(np.diff(row) > 0), "rows sorted, no duplicates"
        assert u not in row
        for v in row:
            got.add(frozenset((u, int(v))))
            assert u in col[rp[v]:rp[v + 1]], "symmetric"
    assert got == E


def test_normalise_rejects_out_of_range():
    with pytest.raises(ValueError):
        oracle.normalise(4, np.array([0, 4], np.int32), np.array([1, 1], np.int32))


def test_normalise_empty_and_isolated():
    n, rp, col = oracle.normalise(5, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert list(rp) == [0] * 6 and len(col) == 0
    n, rp, col = oracle.normalise(3, np.array([1, 1], np.int32), np.array([1, 1], np.int32))
    assert list(rp) == [0, 0, 0, 0]


# ---------------------------------------------------------------- count ----

def _named(name, args):
    if name == "complete":
        return special.complete(int(args))
    if name == "multipartite":
        return special.complete_multipartite([int(x) for x in args.split(",")])
    if name == "wheel":
        return special.wheel(int(args))
    if name == "friendship":
        return special.friendship(int(args))
    if name == "star":
        return special.star(int(args))
    if name == "cycle":
        return special.cycle(int(args))
    if name == "path":
        return special.path(int(args))
    if name == "petersen":
        return special.petersen()
    raise KeyError(name)


def _closed_forms():
    rows = []
    for l in open(os.path.join(GOLDEN, "closed_forms.txt")):
        if l.startswith("#") or not l.strip():
            continue
        name, args, t = l.split()
        rows.append((name, args, int(t)))
    return rows


@pytest.mark.parametrize("name,args,t", _closed_forms())
def test_count_closed_forms(name, args, t):
    g = oracle.normalise(*_named(name, args))
    assert oracle.count(g) == t
    assert oracle.count_idorder(g) == t
    assert oracle.count_split(g)["triangles"] == t


def test_complete_graph_formula_many_n():
    for n in range(0, 26):
        g = oracle.normalise(*special.complete(n)) if n >= 2 else oracle.normalise(max(n, 1), np.zeros(0, np.int32), np.zeros(0, np.int32))
        assert oracle.count(g) == math.comb(n, 3)


@pytest.mark.parametrize("seed", range(6))
def test_count_equals_brute_force_small_random(seed):
    n = 18 + 7 * seed
    n, s, d = synth.uniform_pairs(n, 4 * n, 100 + seed)
    E = _set_graph(n, s, d)
    g = oracle.normalise(n, s, d)
    assert oracle.count(g) == _brute(n, E)


@pytest.mark.parametrize("seed", range(3))
def test_count_equals_trace_a3_over_6(seed):
    n, s, d = synth.chung_lu(600, 14.0, 2.3, seed=seed + 11)
    g = oracle.normalise(n, s, d)
    A = oracle.dense_adjacency(g).astype(np.float64)
    tr = np.trace(A @ A @ A)
    assert tr % 6 == 0
    assert oracle.count(g) == int(tr) // 6
    assert oracle.count_idorder(g) == int(tr) // 6


def test_per_vertex_counts_sum_and_locate():
    n, s, d = synth.chung_lu(300, 10.0, 2.4, seed=5)
    g = oracle.normalise(n, s, d)
    T, pv = oracle.count(g, per_vertex=True)
    assert pv.sum() == T
    _, rp, col = g
    deg = np.diff(rp)
    E = _set_graph(n, s, d)
    brute = np.zeros(n, np.int64)
    for a, b, c in itertools.combinations(range(n), 3):
        if frozenset((a, b)) in E and frozenset((b, c)) in E and frozenset((a, c)) in E:
            low = min((a, b, c), key=lambda x: (deg[x], x))
            brute[low] += 1
    assert np.array_equal(brute, pv)


def test_count_additive_and_relabel_invariant():
    g1 = special.wheel(9)
    g2 = special.complete(7)
    g3 = synth.uniform_pairs(30, 120, 7)
    t = [oracle.count(oracle.normalise(*g)) for g in (g1, g2, g3)]
    u = special.disjoint_union(g1, g2, g3)
    assert oracle.count(oracle.normalise(*u)) == sum(t)
    perm = np.random.default_rng(3).permutation(u[0])
    assert oracle.count(oracle.normalise(*special.relabel(u, perm))) == sum(t)


# ---------------------------------------------------------------- split ----

def test_split_invariants_and_heavy_brute_force():
    n, s, d = synth.chung_lu(400, 16.0, 2.1, seed=9)
    g = oracle.normalise(n, s, d)
    _, rp, col = g
    deg = np.diff(rp)
    m = len(col) // 2
    T = oracle.count(g)
    E = _set_graph(n, s, d)
    for a, b in [(1, 1), (1, 2), (2, 1), (1, 4), (0, 1), (1000, 1)]:
        r = oracle.count_split(g, a, b)
        assert r["triangles"] == T and r["light"] + r["heavy"] == T and r["m"] == m
        H = [v for v in range(n) if b * b * deg[v] ** 2 > a * a * m]
        assert r["n_heavy"] == len(H)
        EH = {e for e in E if all(x in set(H) for x in e)}
        Hs = sorted(H)
        idx = {v: i for i, v in enumerate(Hs)}
        A = _dense(len(Hs), {frozenset(idx[x] for x in e) for e in EH}).astype(np.float64)
        assert r["heavy"] == int(np.trace(A @ A @ A)) // 6
    assert oracle.count_split(g, 0, 1)["heavy"] == oracle.count_split(g, 0, 1)["triangles"]
    assert oracle.count_split(g, 1000, 1)["heavy"] == 0
    h = oracle.count_split(g, 1, 1)["n_heavy"]
    assert h < 2 * math.sqrt(m)


def test_is_heavy_tie_is_light():
    # deg = sqrt(m) exactly: "at most m^(1/2)" is light (section 3.2)
    assert not oracle.is_heavy(10, 100, 1, 1)
    assert oracle.is_heavy(11, 100, 1, 1)
    assert not oracle.is_heavy(20, 100, 2, 1)
    assert oracle.is_heavy(6, 100, 1, 2)


def test_is_heavy_exact_where_64_bit_products_wrap():
    # the test deg > c m^(1/2), c = a/b, as b^2 deg^2 > a^2 m in exact
    # integers (section 3.2): checked against Python's unbounded integers on
    # operands whose 64-bit products would wrap
    cases = [(1, 1 << 24, 1 << 20, 1),             # a^2 m = 2^64: light
             ((1 << 31) - 1, 1 << 29, 1, 1 << 15),  # b^2 deg^2 ~ 2^92: heavy
             (1 << 30, (1 << 30) - 1, 1 << 15, 1 << 15),
             (46341, (1 << 31) - 1, 1, 1), (46340, (1 << 31) - 1, 1, 1),
             (3037000500, 1 << 62, 1, 2), ((1 << 31) - 1, (1 << 30) - 1, (1 << 31) - 1, 1)]
    for deg, m, a, b in cases:
        assert oracle.is_heavy(deg, m, a, b) == (b * b * deg * deg > a * a * m), (deg, m, a, b)


# --------------------------------------------------------------- sample ----

def test_sample_p1_keeps_all_and_symmetry():
    g = oracle.normalise(*synth.chung_lu(2000, 12.0, 2.5, seed=3))
    gp = oracle.sample(g, 1.0, 17)
    assert np.array_equal(g[1], gp[1]) and np.array_equal(g[2], gp[2])
    rng = np.random.default_rng(0)
    for _ in range(200):
        u, v = (int(x) for x in rng.integers(0, 1 << 31, 2))
        for p in (0.5, 0.1):
            assert oracle.keep(u, v, 5, p) == oracle.keep(v, u, 5, p)
    _, rpp, colp = oracle.sample(g, 0.3, 1)
    for u in range(g[0]):
        for v in colp[rpp[u]:rpp[u + 1]]:
            assert u in colp[rpp[v]:rpp[v + 1]]


@pytest.mark.parametrize("p", [0.5, 0.1, 0.05])
def test_sample_size_in_binomial_band(p):
    g = oracle.normalise(*synth.chung_lu(20000, 16.0, 2.5, seed=4))
    m = len(g[2]) // 2
    sizes = []
    for seed in range(3):
        mp = len(oracle.sample(g, p, seed)[2]) // 2
        sizes.append(mp)
        assert abs(mp - m * p) < 6 * math.sqrt(m * p * (1 - p))
    assert len(set(sizes)) == 3, "different seeds keep different sets"


def test_sampled_count_mean_and_variance_closed_form():
    """E[T_p] = p^3 T (section 3.1) and Var[T_p] = T(p^3-p^6) + 2 P1 (p^5-p^6),
    P1 = sum over edges of C(Delta(e), 2): distinct triangles share at most one edge."""
    g = oracle.normalise(*synth.chung_lu(400, 20.0, 2.3, seed=8))
    n, rp, col = g
    T = oracle.count(g)
    P1 = 0
    for u in range(n):
        Nu = set(col[rp[u]:rp[u + 1]].tolist())
        for v in col[rp[u]:rp[u + 1]]:
            if v > u:
                de = len(Nu & set(col[rp[v]:rp[v + 1]].tolist()))
                P1 += de * (de - 1) // 2
    p, S = 0.5, 3000
    xs = np.array([oracle.count(oracle.sample(g, p, s)) for s in range(S)], np.float64)
    mean = T * p ** 3
    var = T * (p ** 3 - p ** 6) + 2 * P1 * (p ** 5 - p ** 6)
    assert abs(xs.mean() - mean) < 5 * math.sqrt(var / S)
    assert abs(xs.var(ddof=1) / var - 1.0) < 0.2


# ------------------------------------------------------------- estimate ----

def test_estimate_rescale():
    assert oracle.estimate(123456789, 1.0) == 123456789.0
    assert oracle.estimate(1000, 0.5) == 8000.0
    assert oracle.estimate(7, 0.25) == 448.0
    for T in (1, 97, 10 ** 9):
        e = oracle.estimate(T, 0.1)
        assert abs(e * 0.1 ** 3 - T) <= 1e-12 * T


def test_median_of_means_hand_cases():
    # 8 seeds, 4 groups of 2: sums 3, 7, 11, 15 -> middle two 7 + 11 = 18 -> 18 / (2*2*p^3)
    assert oracle.median_of_means([1, 2, 3, 4, 5, 6, 7, 8], 4, 1.0) == 4.5
    # 6 seeds, 3 groups of 2: sums 10, 2, 6 -> median 6 -> 6 / (2 * 0.125)
    assert oracle.median_of_means([4, 6, 1, 1, 3, 3], 3, 0.5) == 24.0
    # one group: plain mean
    assert oracle.median_of_means([2, 4, 9], 1, 1.0) == 5.0
    # a single outlier group does not move the median
    assert oracle.median_of_means([5, 5, 5, 5, 5, 5, 5, 1000], 8, 1.0) == 5.0


# -------------------------------------------------------------------- RP ----

@pytest.mark.parametrize("seed", [0, 3])
def test_rp_q_equals_dense_quadratic_form(seed):
    g = oracle.normalise(*synth.chung_lu(250, 12.0, 2.4, seed=seed + 21))
    n = g[0]
    A = oracle.dense_adjacency(g).astype(np.int64)
    A3 = A @ A @ A
    k = 70
    q, est = oracle.rp_trace(g, k, seed)
    for l in range(k):
        x = np.array([oracle.rp_sign(seed, l, i) for i in range(n)], np.int64)
        assert q[l] == int(x @ A3 @ x)
        assert q[l] == oracle.rp_q(g, l, seed)
    assert est == float(int(q.sum())) / (6.0 * k)


def test_rp_exhaustive_average_is_trace():
    """Averaging x^T A^3 x over all 2^n sign vectors gives tr(A^3) = 6 t exactly."""
    g = oracle.normalise(*synth.uniform_pairs(11, 30, 4))
    n = g[0]
    tot = 0
    for bits in range(1 << n):
        x = np.array([1 - 2 * ((bits >> i) & 1) for i in range(n)], np.int64)
        tot += oracle.quadform_a3(g, x)
    assert tot % (1 << n) == 0
    assert tot // (1 << n) == 6 * oracle.count(g)


def test_rp_signs_balanced_and_variance_law():
    """Rademacher x: Var[x^T B x] = 2 (tr(B^2) - sum_i B_ii^2), B = A^3."""
    g = oracle.normalise(*synth.chung_lu(120, 10.0, 2.5, seed=2))
    n = g[0]
    signs = np.array([oracle.rp_sign(9, l, i) for l in range(64) for i in range(n)])
    assert abs(signs.mean()) < 6 / math.sqrt(signs.size)
    A = oracle.dense_adjacency(g).astype(np.float64)
    B = A @ A @ A
    var = 2 * (np.trace(B @ B) - np.sum(np.diag(B) ** 2))
    k = 4000
    q, est = oracle.rp_trace(g, k, 9)
    assert abs(q.mean() - np.trace(B)) < 5 * math.sqrt(var / k)
    assert abs(q.var(ddof=1) / var - 1) < 0.15
