"""Triple sampling on the GPU against the oracle: the same |U|, weight sum,
closed samples and m', and the estimate bit for bit, for Simple and Hybrid,
on the graph and on its sparsified copies."""
import sys

import pytest

import oracle
import synth
from synth import special

pytestmark = pytest.mark.gpu

GRAPHS = {"cl16k": synth.workload("cl16k"), "cl_dense": synth.chung_lu(3000, 120.0, 2.1, seed=5),
          "k65": special.complete(65), "star": special.star(3000), "multi_loops": synth.uniform_pairs(300, 5000, 3),
          "cycle": special.cycle(100)}


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("hybrid", [False, True])
def test_triples_match_oracle(gpu, name, hybrid):
    n, s, d = GRAPHS[name]
    g = gpu.tc_build_csr(n, s, d)
    og = oracle.normalise(n, s, d)
    for p, sseed, tseed, S in ((1.0, 0, 3, 1 << 16), (0.5, 7, 11, 50000), (0.1, 2, 5, 1)):
        sys.stdout.write("triples %s hybrid=%d p=%g\n" % (name, hybrid, p))
        sys.stdout.flush()
        got = gpu.tc_triple_estimate(g, p, S, hybrid=hybrid, sample_seed=sseed, triple_seed=tseed)
        gs = og if p == 1.0 else oracle.sample(og, p, sseed)
        size, wsum, closed = oracle.triple_sample(gs, hybrid, S, tseed)
        assert (got["size"], got["weight_sum"], got["closed"], got["m"]) == (size, wsum, closed, len(gs[2]) // 2)
        assert got["estimate"] == oracle.triple_estimate(size, wsum, S, p)
    g.free()


def test_simple_is_exact_on_complete_graph(gpu):
    import math
    g = gpu.tc_build_csr(*special.complete(200))
    r = gpu.tc_triple_estimate(g, 1.0, 123457, hybrid=False, triple_seed=9)
    assert r["closed"] == 123457 and r["estimate"] == math.comb(200, 3)
    g.free()


def test_invalid_arguments(gpu):
    g = gpu.tc_build_csr(*special.complete(5))
    for bad in (dict(p=0.0, num_samples=10), dict(p=1.0, num_samples=0), dict(p=float("nan"), num_samples=5)):
        with pytest.raises(gpu.TcError):
            gpu.tc_triple_estimate(g, bad["p"], bad["num_samples"])
    g.free()
