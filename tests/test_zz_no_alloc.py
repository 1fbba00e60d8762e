"""The allocation-free single-seed estimate (tc_estimate_noalloc) through the C
ABI: two calls in a row, the second on a smaller graph, each bit-identical to
tc_estimate with the same (graph, p, seed, params); counts that need more
than the fixed scratch array are refused before any device work."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _log(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


def _same(tc, g, p, seed, heavy=(1, 1)):
    got, est = tc.tc_estimate_noalloc(g, p, seed, heavy=heavy)
    per, ests, _ = tc.tc_estimate(g, p, [seed], heavy=heavy)
    assert got == per[0], (p, seed, heavy)
    assert est == ests[0]
    return got


def test_noalloc_matches_estimate_on_consecutive_calls(gpu):
    tc = gpu
    big = synth.chung_lu(16384, 12.0, 2.5, seed=1)
    small = synth.chung_lu(3000, 16.0, 2.3, seed=7)
    gb = tc.tc_build_csr(*big)
    gs = tc.tc_build_csr(*small)
    assert gs.info()["m"] < gb.info()["m"]
    for p, seed in ((1.0, 0), (0.25, 0), (0.5, 3)):
        _log("noalloc: large graph p=%g seed %d, then small graph" % (p, seed))
        a = _same(tc, gb, p, seed)
        b = _same(tc, gs, p, seed)
        assert a["m"] > b["m"] > 0 or p < 1.0
    # a split with heavy vertices in play, and the all-heavy block
    _same(tc, gb, 1.0, 0, heavy=(1, 4))
    _same(tc, gs, 1.0, 0, heavy=(0, 1))
    gb.free()
    gs.free()


def test_noalloc_refuses_counts_beyond_the_scratch_array(gpu):
    tc = gpu
    n, s, d = synth.rmat(18)
    g = tc.tc_build_csr(n, s, d)
    _log("noalloc: R-MAT s18 (m=%d) must not fit" % g.info()["m"])
    with pytest.raises(tc.TcError) as e:
        tc.tc_estimate_noalloc(g, 1.0, 0)
    assert e.value.status == 5 and "scratch" in str(e.value)
    # the refusal leaves the array usable: a small count right after
    small = synth.chung_lu(3000, 16.0, 2.3, seed=7)
    gs = tc.tc_build_csr(*small)
    _same(tc, gs, 0.5, 1)
    gs.free()
    g.free()
