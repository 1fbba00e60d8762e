"""Pins of the oracle's adaptive keep probability and balance point (the
remarks after Table 2; section 3.3) against facts that do not come from the
oracle itself: the balance equation, closed-form counts, the doubling
schedule; and the C ABI's argument checks (no device work)."""
import ctypes
import math

import pytest

import oracle
from paper_1011_0468_amd import _native
from synth import special


@pytest.mark.parametrize("m,n,t,eps", [(10 ** 8, 10 ** 6, 10 ** 9, 0.1), (64153168, 4194304, 2.1e9, 0.02),
                                       (5000, 300, 4.0e6, 0.05)])
def test_balance_point_solves_the_balance_equation(m, n, t, eps):
    p = oracle.balance_p(m, n, t, eps)
    assert 0 < p < 1
    sampling = p * m
    counting = m ** 1.5 * math.log(n) / (p ** 1.5 * t * eps * eps)
    assert sampling == pytest.approx(counting, rel=1e-12)


def test_balance_point_caps():
    assert oracle.balance_p(100, 50, 1.0, 0.01) == 1.0  # the balance would need p > 1
    assert oracle.balance_p(100, 50, 0.0, 0.1) == 1.0
    assert oracle.balance_p(100, 50, 5.0, 0.0) == 1.0


def test_triangle_free_graph_runs_to_the_exact_count():
    # an estimate of 0 never counts as settled
    g = oracle.normalise(*special.cycle(40))
    stages, pb = oracle.estimate_adaptive(g, 1 / 16, 0.01, 3, 4, 2)
    assert [s[0] for s in stages] == [1 / 16, 1 / 8, 1 / 4, 1 / 2, 1.0]
    assert all(s[1] == 0.0 for s in stages) and stages[-1][2] == 4 * 40 and pb == 1.0


def test_p0_one_is_the_exact_count():
    g = oracle.normalise(*special.complete(7))
    stages, _ = oracle.estimate_adaptive(g, 1.0, 0.5, 0, 4, 2)
    assert stages == [(1.0, 35.0, 4 * 21)]


def test_zero_tolerance_doubles_to_the_exact_count():
    g = oracle.normalise(*special.complete(30))
    stages, _ = oracle.estimate_adaptive(g, 1 / 8, 0.0, 11, 6, 3)
    assert [s[0] for s in stages] == [0.125, 0.25, 0.5, 1.0]
    assert stages[-1][1] == math.comb(30, 3)
    assert len({s[1] for s in stages}) == 4  # no two stages agreed exactly


def test_stage_cap():
    g = oracle.normalise(*special.complete(30))
    stages, _ = oracle.estimate_adaptive(g, 1 / 64, 0.5, 1, 2, 1, max_stages=3)
    assert [s[0] for s in stages] == [1 / 64, 1 / 32, 1 / 16]


def test_abi_rejects_bad_arguments():
    L = _native.load()
    st = (_native.TcStage * 4)()
    ns = ctypes.c_int32(7)
    assert L.tc_estimate_adaptive(None, 0.5, 0.1, 0, 4, 2, 4, None, None, st, ctypes.byref(ns), None) == \
        _native.TC_ERR_INVALID
    assert ns.value == 0
