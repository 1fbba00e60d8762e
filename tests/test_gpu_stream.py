"""The semi-streaming variant (section 5.2) on the GPU against the oracle:
every count of the three passes (draws, candidates, |H|, |L|, |U|, lookups,
closed draws, m) equal and the estimate bit for bit, on graphs with and
without heavy vertices, triangle-free and degenerate ones."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import special

pytestmark = pytest.mark.gpu

GRAPHS = {"cl16k": synth.workload("cl16k"), "cl_dense": synth.chung_lu(3000, 120.0, 2.1, seed=5),
          "rmat14": synth.rmat(14, seed=3), "k65": special.complete(65), "star": special.star(3000),
          "wheel": special.wheel(200), "multi_loops": synth.uniform_pairs(300, 5000, 3), "cycle": special.cycle(100),
          "bipartite": special.complete_multipartite([20, 30])}

CASES = ((1.0, 1 << 16, 3), (3.0, 50000, 11), (0.2, 1, 5), (2.0, 0, 1), (0.5, 777, 2 ** 64 - 1))


def _check(gpu, g, og, d, s, seed, label):
    sys.stdout.write("stream %s d=%g s=%d seed=%d\n" % (label, d, s, seed))
    sys.stdout.flush()
    got = gpu.tc_stream_estimate(g, d, s, seed=seed)
    want, _ = oracle.stream_estimate(og, d, s, seed)
    assert got == want, (label, d, s, seed)
    return got


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_stream_matches_oracle(gpu, name):
    n, s, d = GRAPHS[name]
    g = gpu.tc_build_csr(n, s, d)
    og = oracle.normalise(n, s, d)
    for dd, S, seed in CASES:
        _check(gpu, g, og, dd, S, seed, name)
    g.free()


def test_heavy_set_found_and_used(gpu):
    # a dense Chung-Lu graph has vertices above m^(1/2): with d = 3 they are
    # all candidates, so X is not empty and both kinds of draws occur
    n, s, d = GRAPHS["cl_dense"]
    og = oracle.normalise(n, s, d)
    m = len(og[2]) // 2
    deg = np.diff(og[1])
    g = gpu.tc_build_csr(n, s, d)
    r = _check(gpu, g, og, 3.0, 200000, 4, "cl_dense")
    assert r["heavy"] == int((deg.astype(np.int64) ** 2 > m).sum()) > 0
    assert r["size"] > r["light_size"] > 0
    T = oracle.count(og)
    # 200000 draws: within 10 % of the exact count
    assert abs(r["estimate"] - T) < 0.1 * T
    g.free()


def test_complete_graph_closes_every_drawn_wedge(gpu):
    # K_n: every wedge and every pair (h; e) with h outside e is closed
    g = gpu.tc_build_csr(*special.complete(40))
    r = gpu.tc_stream_estimate(g, 1.0, 10000, seed=8)
    n, m = 40, 40 * 39 // 2
    assert r["m"] == m and r["draws1"] == math.ceil(math.sqrt(m) * math.log(n))
    # every draw that asks for edges is closed: one or two lookups per closed draw
    assert 0 < r["closed"] <= 10000 and r["closed"] <= r["queries"] <= 2 * r["closed"]
    want, _ = oracle.stream_estimate(oracle.normalise(*special.complete(40)), 1.0, 10000, 8)
    assert r == want
    g.free()


def test_degenerate_graphs(gpu):
    for label, graph in (("no_edges", (10, np.zeros(0, np.int32), np.zeros(0, np.int32))),
                         ("one_vertex", (1, np.zeros(1, np.int32), np.zeros(1, np.int32))),
                         ("one_edge", (2, np.array([0], np.int32), np.array([1], np.int32))),
                         ("path", special.path(50))):
        g = gpu.tc_build_csr(*graph)
        og = oracle.normalise(*graph)
        for dd, S, seed in CASES:
            r = _check(gpu, g, og, dd, S, seed, label)
            assert r["closed"] == 0 and r["estimate"] == 0.0
        g.free()


def test_ragged_sample_counts(gpu):
    # sample counts around the grid's block and the table's growth steps
    n, s, d = GRAPHS["rmat14"]
    g = gpu.tc_build_csr(n, s, d)
    og = oracle.normalise(n, s, d)
    for S in (255, 256, 257, 1023, 1024, 65537):
        _check(gpu, g, og, 1.0, S, 21, "rmat14")
    g.free()


def test_invalid_arguments(gpu):
    g = gpu.tc_build_csr(*special.complete(5))
    for dd, S in ((0.0, 10), (-1.0, 10), (float("nan"), 10), (float("inf"), 10), (1.0, -1)):
        with pytest.raises(gpu.TcError):
            gpu.tc_stream_estimate(g, dd, S)
    with pytest.raises(gpu.TcError):
        gpu.tc_stream_estimate(g, 1.0, (1 << 28) + 1)
    g.free()
