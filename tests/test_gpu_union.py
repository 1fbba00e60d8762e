"""Batched seeds as one union count: every seed's counts (all statistics
included) equal those of the seed counted alone, and the triangle counts
equal the oracle's, on graphs that exercise every phase: light-only,
all-heavy, mixed splits, isolated vertices, stars, and samples that keep
nothing."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _log(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


def _graphs():
    out = {}
    out["cl16k"] = synth.workload("cl16k")
    out["cl3000_dense"] = synth.chung_lu(3000, 40.0, 2.1, seed=5)
    n = 60
    iu = np.triu_indices(n, 1)
    out["k60"] = (n, iu[0].astype(np.int32), iu[1].astype(np.int32))
    out["star"] = (3001, np.zeros(3000, np.int32), np.arange(1, 3001, dtype=np.int32))
    out["rmat14"] = synth.rmat(14)
    _, s, d = synth.uniform_pairs(500, 4000, seed=3)
    out["isolated_tail"] = (5000, s, d)  # vertices 500..4999 isolated
    return out


GRAPHS = _graphs()


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("heavy", [(1, 1), (1, 4), (0, 1)])
def test_union_batch_equals_single_seeds(gpu, name, heavy):
    tc = gpu
    n, s, d = GRAPHS[name]
    g = tc.tc_build_csr(n, s, d)
    og = oracle.normalise(n, s, d)
    seeds = [0, 1, 2, 3, 4, 5, 6, 7, 11, 1000]
    for p in (0.3, 0.75):
        _log("union %s heavy %s p=%g" % (name, heavy, p))
        per, ests, mom = tc.tc_estimate(g, p, seeds, num_groups=5, heavy=heavy)
        singles = [tc.tc_estimate(g, p, [sd], heavy=heavy) for sd in seeds]
        for sd, c, e, (sp, se, _) in zip(seeds, per, ests, singles):
            assert c == sp[0], (name, heavy, p, sd, c, sp[0])
            assert e == se[0]
        want = [oracle.count(oracle.sample(og, p, sd)) for sd in seeds]
        assert [c["triangles"] for c in per] == want
        assert mom == oracle.median_of_means(want, 5, p)
    g.free()


def test_union_batch_of_empty_samples(gpu):
    tc = gpu
    n, s, d = GRAPHS["cl16k"]
    g = tc.tc_build_csr(n, s, d)
    per, ests, mom = tc.tc_estimate(g, 1e-9, list(range(8)), num_groups=2)
    assert all(c["m"] == 0 and c["triangles"] == 0 for c in per) and mom == 0.0
    singles = [tc.tc_estimate(g, 1e-9, [sd])[0][0] for sd in range(8)]
    assert per == singles
    g.free()
