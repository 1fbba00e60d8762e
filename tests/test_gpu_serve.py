"""Serving engine on the GPU: every request's counts equal the stand-alone
call's and the oracle's, whatever else is in flight; admission keeps the arena
within its budget and every allocation inside its reservation."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _log(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


def _mix(count, lo, hi, seed):
    scales, ps = synth.serving_requests(count, lo, hi, seed)
    reqs = []
    for i in range(count):
        n, s, d = synth.serving_graph(i, scales[i])
        reqs.append(dict(id=i, n=n, src=s, dst=d, p=float(ps[i]), seed=i))
    return reqs


def _alone(tc, r):
    g = tc.tc_build_csr(r["n"], r["src"], r["dst"])
    per, ests, _ = tc.tc_estimate(g, r["p"], [r["seed"]])
    g.free()
    return per[0], ests[0]


def _oracle_T(r):
    og = oracle.normalise(r["n"], r["src"], r["dst"])
    if r["p"] < 1.0:
        og = oracle.sample(og, r["p"], r["seed"])
    return oracle.count(og)


def _check_intervals(res, lanes):
    # at no time are more than `lanes` requests between admission and completion
    ev = sorted([(x["start_s"], 1) for x in res] + [(x["done_s"], -1) for x in res], key=lambda e: (e[0], e[1]))
    cur = peak = 0
    for _, d in ev:
        cur += d
        peak = max(peak, cur)
    assert peak <= lanes


def test_mix_equals_alone_and_oracle(gpu):
    tc = gpu
    reqs = _mix(48, 6, 13, seed=7)
    bounds = [tc.tc_request_bytes(r["p"], n=r["n"], src=r["src"], dst=r["dst"]) for r in reqs]
    budget = int(2.5 * max(bounds))  # admission pressure: a few requests at a time
    _log("serve mix: 48 requests, budget %d" % budget)
    with tc.Server(budget, lanes=4) as sv:
        for r in reqs:
            sv.submit(r["id"], r["p"], r["seed"], n=r["n"], src=r["src"], dst=r["dst"])
        res = sv.drain()
        st = sv.stats()
    assert len(res) == len(reqs)
    assert st["completed"] == len(reqs) and st["queued"] == 0 and st["running"] == 0
    assert st["arena_peak"] <= st["arena_bytes"] and st["spilled_bytes"] == 0
    _check_intervals(res, 4)
    by_id = {x["id"]: x for x in res}
    for r, b in zip(reqs, bounds):
        x = by_id[r["id"]]
        assert x["status"] == 0, x["message"]
        assert x["reserved_bytes"] == b and 0 < x["peak_bytes"] <= b and x["spilled_bytes"] == 0
        assert x["arrival_s"] <= x["start_s"] <= x["done_s"]
        counts, est = _alone(tc, r)
        assert x["counts"] == counts, r["id"]
        assert x["estimate"] == est
        assert x["counts"]["triangles"] == _oracle_T(r), r["id"]


def test_one_lane_serves_in_arrival_order(gpu):
    tc = gpu
    reqs = _mix(12, 6, 11, seed=3)
    with tc.Server(1 << 30, lanes=1) as sv:
        for r in reqs:
            sv.submit(r["id"], r["p"], r["seed"], n=r["n"], src=r["src"], dst=r["dst"])
        res = sv.drain()
    assert [x["id"] for x in res] == [r["id"] for r in reqs]
    for a, b in zip(res, res[1:]):
        assert a["done_s"] <= b["start_s"]
    assert all(x["lane"] == 0 and x["status"] == 0 for x in res)


def test_resident_graphs_and_future_arrivals(gpu):
    tc = gpu
    n, s, d = synth.workload("cl16k")
    g = tc.tc_build_csr(n, s, d)
    og = oracle.normalise(n, s, d)
    points = [(1.0, 0), (0.5, 1), (0.5, 2), (0.1, 3), (0.25, 4), (0.75, 5)]
    with tc.Server(1 << 30, lanes=3) as sv:
        t0 = sv.clock()
        for k, (p, seed) in enumerate(points):
            sv.submit(100 + k, p, seed, arrival_s=t0 + 0.02 * k, graph=g)
        res = sv.drain()
    assert len(res) == len(points)
    for x in res:
        p, seed = points[x["id"] - 100]
        assert x["status"] == 0
        assert x["arrival_s"] >= t0 + 0.02 * (x["id"] - 100) - 1e-9
        assert x["start_s"] >= x["arrival_s"]
        per, ests, _ = tc.tc_estimate(g, p, [seed])
        assert x["counts"] == per[0] and x["estimate"] == ests[0]
        want = oracle.count(og if p == 1.0 else oracle.sample(og, p, seed))
        assert x["counts"]["triangles"] == want
    g.free()


def test_failed_request_does_not_disturb_the_mix(gpu):
    tc = gpu
    reqs = _mix(6, 6, 9, seed=11)
    bad = dict(id=999, n=10, src=np.array([0, 1, 50], np.int32), dst=np.array([1, 2, 3], np.int32), p=1.0, seed=0)
    with tc.Server(1 << 30, lanes=2) as sv:
        for r in reqs[:3] + [bad] + reqs[3:]:
            sv.submit(r["id"], r["p"], r["seed"], n=r["n"], src=r["src"], dst=r["dst"])
        res = sv.drain()
        st = sv.stats()
    by_id = {x["id"]: x for x in res}
    assert by_id[999]["status"] == 1 and "outside" in by_id[999]["message"]
    assert st["arena_used"] == 0
    for r in reqs:
        assert by_id[r["id"]]["status"] == 0
        assert by_id[r["id"]]["counts"] == _alone(tc, r)[0]


def test_serving_workload_largest_request(gpu):
    # the scale-20 end of the serving mix under the default 8 GiB budget, at
    # the mix's three keep probabilities: every request against the oracle's
    # counts stored in tests/golden/serve20.json and against the stand-alone call
    import json
    import os
    tc = gpu
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "serve20.json")))
    want = {c["seed"]: c for c in gold["counts"]}
    n, s, d = synth.serving_graph(0, 20)
    assert n == gold["n"] and len(s) == gold["pairs"]
    with tc.Server(8 << 30, lanes=4) as sv:
        for k, c in want.items():
            sv.submit(k, c["p"], k, n=n, src=s, dst=d)
        res = sv.drain()
    g = tc.tc_build_csr(n, s, d)
    assert len(res) == len(want)
    for x in res:
        w = want[x["id"]]
        p = w["p"]
        assert x["status"] == 0 and x["spilled_bytes"] == 0 and x["peak_bytes"] <= x["reserved_bytes"]
        for k in ("triangles", "light", "heavy", "n_heavy", "m"):
            assert x["counts"][k] == w[k], (p, k, x["counts"][k], w[k])
        assert x["estimate"] == oracle.estimate(w["triangles"], p)
        per, _, _ = tc.tc_estimate(g, p, [x["id"]])
        assert x["counts"] == per[0]
        _log("scale 20 p=%g: T=%d latency %.1f ms, peak %.0f MiB of %.0f MiB reserved"
             % (p, x["counts"]["triangles"], 1e3 * (x["done_s"] - x["arrival_s"]), x["peak_bytes"] / 2**20,
                x["reserved_bytes"] / 2**20))
    g.free()


def _groups(res):
    # requests that ran as one fused group share their admission and completion times
    by = {}
    for x in res:
        by.setdefault((x["lane"], x["start_s"], x["done_s"]), []).append(x["id"])
    return [g for g in by.values() if len(g) > 1]


def test_fused_small_requests_equal_alone_and_oracle(gpu):
    # small requests fused into one union build and count: every result equals
    # the request run alone and the oracle's count, whatever it was fused with
    tc = gpu
    reqs = _mix(40, 6, 12, seed=19)
    with tc.Server(1 << 30, lanes=2, fuse_max_pairs=1 << 16) as sv:
        for r in reqs:
            sv.submit(r["id"], r["p"], r["seed"], n=r["n"], src=r["src"], dst=r["dst"])
        res = sv.drain()
        st = sv.stats()
    assert len(res) == len(reqs) and st["spilled_bytes"] == 0
    groups = _groups(res)
    _log("fused: %d groups, sizes %s" % (len(groups), sorted(len(g) for g in groups)))
    assert groups, "no request was fused"
    by_id = {x["id"]: x for x in res}
    for r in reqs:
        x = by_id[r["id"]]
        assert x["status"] == 0, x["message"]
        assert 0 < x["peak_bytes"] <= x["reserved_bytes"] and x["spilled_bytes"] == 0
        counts, est = _alone(tc, r)
        assert x["counts"] == counts, r["id"]
        assert x["estimate"] == est
        assert x["counts"]["triangles"] == _oracle_T(r), r["id"]


def test_fused_group_with_a_bad_request(gpu):
    tc = gpu
    reqs = _mix(6, 6, 9, seed=23)
    bad = dict(id=999, n=10, src=np.array([0, 1, 50], np.int32), dst=np.array([1, 2, 3], np.int32), p=0.5, seed=0)
    with tc.Server(1 << 30, lanes=1, fuse_max_pairs=1 << 16) as sv:
        for r in reqs[:3] + [bad] + reqs[3:]:
            sv.submit(r["id"], r["p"], r["seed"], n=r["n"], src=r["src"], dst=r["dst"])
        res = sv.drain()
    by_id = {x["id"]: x for x in res}
    assert by_id[999]["status"] == 1 and "outside" in by_id[999]["message"]
    for r in reqs:
        assert by_id[r["id"]]["status"] == 0
        assert by_id[r["id"]]["counts"] == _alone(tc, r)[0]


def test_fusion_leaves_large_requests_alone(gpu):
    # requests above the threshold run alone; the small ones around them fuse
    tc = gpu
    reqs = _mix(16, 8, 14, seed=29)
    with tc.Server(1 << 30, lanes=2, fuse_max_pairs=1 << 14) as sv:
        for r in reqs:
            sv.submit(r["id"], r["p"], r["seed"], n=r["n"], src=r["src"], dst=r["dst"])
        res = sv.drain()
    by_id = {x["id"]: x for x in res}
    for g in _groups(res):
        assert all(len(by_id[i]["counts"]) and next(r for r in reqs if r["id"] == i)["src"].size <= 1 << 14 for i in g)
    for r in reqs:
        assert by_id[r["id"]]["status"] == 0
        assert by_id[r["id"]]["counts"] == _alone(tc, r)[0]
