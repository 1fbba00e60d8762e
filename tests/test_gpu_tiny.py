"""Graphs whose light anchors are mostly tiny (at most 8 out-neighbours, 8
iterated lists and 64 streamed positions, closed by lane groups without
tables) or sit just past those limits: counts and splits equal to the
oracle's, single and batched."""
import sys

import numpy as np
import pytest

import oracle
import synth
from synth import special

pytestmark = pytest.mark.gpu


def _cliques(k, copies):
    # disjoint copies of K_k: every anchor has d+ <= k - 1
    return special.disjoint_union(*[special.complete(k) for _ in range(copies)])


GRAPHS = {
    "k5_x2000": _cliques(5, 2000),      # d+ <= 4: all tiny
    "k9_x500": _cliques(9, 500),        # d+ <= 8: at the key limit
    "k10_x400": _cliques(10, 400),      # d+ up to 9: past it
    "k12_x200": _cliques(12, 200),      # positions past 64 for some anchors
    "gnm_low": synth.uniform_pairs(20000, 60000, 17),
    "cl_low": synth.chung_lu(30000, 5.0, 2.4, seed=3),
    "friendship": special.friendship(3000),
}


def _split(g):
    return oracle.count_split(g, 1, 1)


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_counts_match_oracle(gpu, name):
    n, s, d = GRAPHS[name]
    g = gpu.tc_build_csr(n, s, d)
    og = oracle.normalise(n, s, d)
    for p, seed in ((1.0, 0), (0.6, 1), (0.3, 2)):
        sys.stdout.write("tiny %s p=%g\n" % (name, p))
        sys.stdout.flush()
        want = _split(og if p == 1.0 else oracle.sample(og, p, seed))
        got = gpu.tc_count_exact(g) if p == 1.0 else gpu.tc_estimate(g, p, [seed])[0][0]
        for k in ("triangles", "light", "heavy", "n_heavy", "m"):
            assert got[k] == want[k], (name, p, k, got[k], want[k])
    g.free()


@pytest.mark.parametrize("name", ["k5_x2000", "cl_low", "k12_x200"])
def test_batched_equals_single_calls(gpu, name):
    n, s, d = GRAPHS[name]
    g = gpu.tc_build_csr(n, s, d)
    seeds = list(range(16))
    per, _, mom = gpu.tc_estimate(g, 0.5, seeds, num_groups=4)
    one = [gpu.tc_estimate(g, 0.5, [sd])[0][0] for sd in seeds]
    assert [c["triangles"] for c in per] == [c["triangles"] for c in one]
    assert [c["light"] for c in per] == [c["light"] for c in one]
    og = oracle.normalise(n, s, d)
    want = [oracle.count(oracle.sample(og, 0.5, sd)) for sd in seeds]
    assert [c["triangles"] for c in per] == want
    assert mom == oracle.median_of_means(want, 4, 0.5)
    g.free()


def test_clique_closed_forms(gpu):
    # K_k copies: C(k, 3) triangles each
    for k, copies in ((5, 2000), (9, 500), (12, 200)):
        g = gpu.tc_build_csr(*_cliques(k, copies))
        assert gpu.tc_count_exact(g)["triangles"] == copies * (k * (k - 1) * (k - 2) // 6)
        g.free()
