"""Host-side checks of the serving engine: the admission bound, argument
checks, budget rejection and allocator failure, all before any device work."""
import ctypes

import numpy as np
import pytest

import paper_1011_0468_amd as tc
from paper_1011_0468_amd import _native
import synth


def _pairs(P, n=1 << 10):
    return np.zeros(P, np.int32), np.ones(P, np.int32) % n


def test_request_bytes_bounds_the_csr_and_grows_with_size():
    prev = 0
    for P in (0, 1, 1000, 16 << 10, 1 << 20):
        s, d = _pairs(P)
        b = tc.tc_request_bytes(1.0, n=1 << 10, src=s, dst=d)
        # at least the staging copy, the radix keys and the CSR itself
        assert b >= 8 * P + 2 * 4 * 2 * P + 4 * (2 * 2 * P) + 4 * (1 << 10)
        assert b % 256 == 0
        assert b >= prev
        prev = b


def test_request_bytes_sampled_needs_more_than_exact():
    s, d = _pairs(50000)
    exact = tc.tc_request_bytes(1.0, n=4096, src=s, dst=d)
    sampled = tc.tc_request_bytes(0.5, n=4096, src=s, dst=d)
    # the compacted sample: keep bits and prefixes, row pointers, degrees, col and src
    assert sampled > exact + 2 * 4 * 2 * 50000


def test_request_bytes_serving_mix_fits_eight_gib():
    scales, ps = synth.serving_requests(1000)
    assert scales.min() == 10 and scales.max() == 20
    # largest request of the mix: scale 20, p < 1
    P = 16 << 20
    r = _native.TcRequest()
    r.n, r.num_pairs, r.p = 1 << 20, P, 0.1
    r.src = r.dst = 1  # not dereferenced
    out = ctypes.c_int64(0)
    assert _native.load().tc_request_bytes(ctypes.byref(r), ctypes.byref(out)) == _native.TC_OK
    assert 64 * P < out.value < (8 << 30) // 2


@pytest.mark.parametrize("p", [0.0, -0.5, 1.5, float("nan"), float("inf")])
def test_request_bytes_rejects_bad_p(p):
    s, d = _pairs(10)
    with pytest.raises(tc.TcError) as e:
        tc.tc_request_bytes(p, n=16, src=s, dst=d)
    assert e.value.status == _native.TC_ERR_INVALID


def test_request_bytes_overflow_and_null():
    L = _native.load()
    r = _native.TcRequest()
    r.p = 1.0
    r.n = 1 << 31
    out = ctypes.c_int64(0)
    assert L.tc_request_bytes(ctypes.byref(r), ctypes.byref(out)) == _native.TC_ERR_OVERFLOW
    r.n, r.num_pairs = 10, 5
    assert L.tc_request_bytes(ctypes.byref(r), ctypes.byref(out)) == _native.TC_ERR_INVALID  # NULL src/dst
    assert L.tc_request_bytes(None, ctypes.byref(out)) == _native.TC_ERR_INVALID


@pytest.mark.parametrize("lanes", [0, 17, -1])
def test_server_rejects_bad_lane_count(lanes):
    with pytest.raises(tc.TcError) as e:
        tc.Server(0, lanes=lanes)
    assert e.value.status == _native.TC_ERR_INVALID


def test_zero_budget_rejects_every_request():
    with tc.Server(0, lanes=2) as sv:
        for P in (0, 3, 1000):
            s, d = _pairs(P)
            with pytest.raises(tc.TcError) as e:
                sv.submit(P, 1.0, 0, n=64, src=s, dst=d)
            assert e.value.status == _native.TC_ERR_BUDGET
        st = sv.stats()
        assert st["rejected"] == 3 and st["submitted"] == 0 and st["queued"] == 0
        assert sv.poll(8, 0.0) == []
        assert sv.clock() >= 0.0


def test_submit_checks_arguments():
    with tc.Server(0, lanes=1) as sv:
        s, d = _pairs(4)
        with pytest.raises(tc.TcError) as e:
            sv.submit(1, 2.0, 0, n=8, src=s, dst=d)
        assert e.value.status == _native.TC_ERR_INVALID
        with pytest.raises(tc.TcError) as e:
            sv.submit(2, 0.5, 0, arrival_s=float("nan"), n=8, src=s, dst=d)
        assert e.value.status == _native.TC_ERR_INVALID
        assert sv.stats()["rejected"] == 0


def test_arena_allocation_failure_is_oom():
    L = _native.load()
    calls = []

    @_native.ALLOC_FN
    def failing_alloc(nbytes, stream, ctx):
        calls.append(nbytes)
        return None

    @_native.FREE_FN
    def no_free(ptr, stream, ctx):
        pass

    assert L.tc_set_allocator(failing_alloc, no_free, None) == _native.TC_OK
    try:
        with pytest.raises(tc.TcError) as e:
            tc.Server(1 << 20, lanes=2)
        assert e.value.status == _native.TC_ERR_OOM
        assert calls == [1 << 20]
    finally:
        assert L.tc_set_allocator(_native.ALLOC_FN(0), _native.FREE_FN(0), None) == _native.TC_OK


def test_poll_and_stats_argument_checks():
    L = _native.load()
    got = ctypes.c_int32(0)
    assert L.tc_server_poll(None, None, 0, 0.0, ctypes.byref(got)) == _native.TC_ERR_INVALID
    with tc.Server(0, lanes=1) as sv:
        assert L.tc_server_poll(sv._h, None, 4, 0.0, ctypes.byref(got)) == _native.TC_ERR_INVALID
        assert L.tc_server_poll(sv._h, None, 0, 0.0, ctypes.byref(got)) == _native.TC_OK and got.value == 0
        assert L.tc_server_stats(sv._h, None) == _native.TC_ERR_INVALID
    L.tc_server_destroy(None)  # ignored
