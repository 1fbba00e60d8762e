"""Adaptive keep probability on the GPU against the oracle: the same stages
(p, the median of means bit for bit, the edges counted) and the same balance
point (through libm, so to 1e-12)."""
import sys

import pytest

import oracle
import synth
from synth import special

pytestmark = pytest.mark.gpu

GRAPHS = {"cl16k": synth.workload("cl16k"), "k60": special.complete(60), "cycle": special.cycle(500)}

# (graph, p0, tol, seed0, seeds per stage, groups)
CASES = [("cl16k", 1 / 64, 0.02, 5, 8, 4), ("cl16k", 1 / 8, 0.0, 9, 4, 2), ("cl16k", 0.3, 0.5, 77, 3, 3),
         ("k60", 1 / 32, 0.05, 1, 6, 3), ("cycle", 1 / 4, 0.1, 0, 2, 1)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-p0=%g-tol=%g" % c[:3])
def test_adaptive_matches_oracle(gpu, case):
    name, p0, tol, seed0, S, G = case
    sys.stdout.write("adaptive %s p0=%g tol=%g\n" % (name, p0, tol))
    sys.stdout.flush()
    n, s, d = GRAPHS[name]
    g = gpu.tc_build_csr(n, s, d)
    stages, pb = gpu.tc_estimate_adaptive(g, p0, tol, seed0, S, G)
    ostages, opb = oracle.estimate_adaptive(oracle.normalise(n, s, d), p0, tol, seed0, S, G)
    assert [(x["p"], x["estimate"], x["m_sum"]) for x in stages] == ostages
    assert pb == pytest.approx(opb, rel=1e-12)
    g.free()


def test_adaptive_with_tuned_launches(gpu):
    # the launch table of each stage's p is used; the stages do not change
    n, s, d = GRAPHS["cl16k"]
    g = gpu.tc_build_csr(n, s, d)
    for p in (1 / 16, 1 / 8, 1 / 4, 1 / 2, 1.0):
        gpu.tc_tune_set(g, p, heavy=(1, 2), vmajor_cap=4, small_dmax=32, blocks_per_cu=2)
    tuned, _ = gpu.tc_estimate_adaptive(g, 1 / 16, 0.03, 2, 4, 2, tuned=True)
    plain, _ = gpu.tc_estimate_adaptive(g, 1 / 16, 0.03, 2, 4, 2)
    assert tuned == plain
    g.free()
