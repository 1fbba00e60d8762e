"""Full-size parity on the R-MAT scale-22 workload, in the launch
configuration the benchmark times: the device CSR against the oracle's
normalised graph, the sampled CSR at p = 0.1 against the oracle's sample, and
the counts at p in {1, 0.5, 0.1, 0.05} (seed 0) against the oracle values
stored in tests/golden/rmat22.json (written by tests/golden/make_golden.py)."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _log(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rmat22(gpu):
    import torch
    n, s, d = synth.workload("rmat22")
    _log("rmat22: building device CSR")
    g = gpu.tc_build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    return n, s, d, g


@pytest.fixture(scope="module")
def rmat22_oracle(rmat22):
    # the oracle's normalised graph, built once per module (host work)
    n, s, d, g = rmat22
    _log("rmat22: oracle normalise")
    return oracle.normalise(n, s, d)


def test_rmat22_csr_and_sample_match_oracle(gpu, rmat22, rmat22_oracle):
    n, s, d, g = rmat22
    og = rmat22_oracle
    rp, col, deg = gpu.tc_graph_read(g)
    assert np.array_equal(rp.astype(np.int64), og[1])
    assert np.array_equal(col, og[2])
    _log("rmat22: sample p=0.1 seed 0")
    gs = gpu.tc_sample(g, 0.1, 0)
    rps, cols, _ = gpu.tc_graph_read(gs)
    ogs = oracle.sample(og, 0.1, 0)
    assert np.array_equal(rps.astype(np.int64), ogs[1])
    assert np.array_equal(cols, ogs[2])


def test_rmat22_counts_match_golden(gpu, rmat22):
    n, s, d, g = rmat22
    gold = json.load(open(os.path.join(GOLDEN, "rmat22.json")))
    for want in gold["counts"]:
        p = want["p"]
        _log("rmat22: count p=%g" % p)
        if p == 1.0:
            got = gpu.tc_count_exact(g)
            est = float(got["triangles"])
        else:
            per, ests, _ = gpu.tc_estimate(g, p, [want["seed"]])
            got, est = per[0], ests[0]
        for k in ("triangles", "light", "heavy", "n_heavy", "m"):
            assert got[k] == want[k], (p, k, got[k], want[k])
        assert est == oracle.estimate(want["triangles"], p)


def test_rmat22_split_invariance(gpu, rmat22):
    n, s, d, g = rmat22
    gold = json.load(open(os.path.join(GOLDEN, "rmat22.json")))
    want = [c for c in gold["counts"] if c["p"] == 0.1][0]
    for a, b in [(1, 2), (2, 1), (1, 4)]:
        _log("rmat22: p=0.1 split %d/%d" % (a, b))
        per, _, _ = gpu.tc_estimate(g, 0.1, [0], heavy=(a, b))
        assert per[0]["triangles"] == want["triangles"]


def test_rmat22_every_operating_split_matches_golden(gpu, rmat22):
    # the light/heavy split at each operating point of the benchmark for every
    # heavy multiplier the autotuner may choose (c = 1/4, 1/2, 2; c = 1 is
    # covered above), against the oracle (tests/golden/rmat22_splits.json)
    n, s, d, g = rmat22
    gold = json.load(open(os.path.join(GOLDEN, "rmat22_splits.json")))
    for want in gold["counts"]:
        p, (a, b) = want["p"], want["split"]
        _log("rmat22: p=%g split %d/%d" % (p, a, b))
        if p == 1.0:
            got = gpu.tc_count_exact(g, heavy=(a, b))
        else:
            got = gpu.tc_estimate(g, p, [want["seed"]], heavy=(a, b))[0][0]
        for k in ("triangles", "light", "heavy", "n_heavy", "m"):
            assert got[k] == want[k], (p, a, b, k, got[k], want[k])


def test_rmat22_stream_estimate_matches_golden(gpu, rmat22):
    # the semi-streaming estimate (section 5.2) in the benchmark's
    # configuration (d = 1, 2^24 pass-2 draws), every count and the estimate
    # against the oracle's stored runs (tests/golden/stream22.json)
    n, s, d, g = rmat22
    gold = json.load(open(os.path.join(GOLDEN, "stream22.json")))
    keys = ("draws1", "candidates", "heavy", "light_size", "size", "queries", "closed", "m", "estimate")
    for want in gold["runs"]:
        _log("rmat22: stream d=%g s=%d seed %d" % (want["d"], want["num_samples"], want["seed"]))
        got = gpu.tc_stream_estimate(g, want["d"], want["num_samples"], seed=want["seed"])
        assert got == {k: want[k] for k in keys}
    # sampled relative error at 2^24 draws (about 40 closed draws per 10^6)
    assert abs(got["estimate"] / gold["exact"] - 1.0) < 0.02


def _timed(label, fn):
    import time
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    _log("%s: %.1f ms" % (label, (time.perf_counter() - t) * 1e3))
    return out


@pytest.fixture(scope="module")
def rmat24(gpu):
    import torch
    n, s, d = synth.workload("rmat24")
    _log("rmat24: building device CSR")
    g = gpu.tc_build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    synth._CACHE.pop("rmat24", None)
    return n, g


def test_rmat24_rp_vectors_match_golden(gpu, rmat24):
    """k = 256 Rademacher vectors on R-MAT scale 24: every q_l, which the
    oracle computed one by one (tests/golden/rmat24.json), must match exactly."""
    n, g = rmat24
    gold = json.load(open(os.path.join(GOLDEN, "rmat24.json")))
    assert g.info()["m"] == gold["m"]
    q, est = _timed("rmat24 rp k=256", lambda: gpu.tc_rp_trace(g, gold["k"], gold["seed"]))
    want = np.array(gold["q"], dtype=np.int64)
    assert len(want) == gold["k"] == len(q)
    bad = np.nonzero(q != want)[0]
    assert len(bad) == 0, [(int(l), int(q[l]), int(want[l])) for l in bad[:5]]
    assert est == float(int(q.sum())) / (6.0 * gold["k"])


def test_rmat24_exact_count_matches_golden(gpu, rmat24):
    n, g = rmat24
    want = json.load(open(os.path.join(GOLDEN, "rmat24_count.json")))["exact"]
    got = _timed("rmat24 exact", lambda: gpu.tc_count_exact(g))
    for k in ("triangles", "light", "heavy", "n_heavy", "m"):
        assert got[k] == want[k], (k, got[k], want[k])


def test_cl20_batched_median_of_means_matches_golden(gpu):
    import torch
    gold = json.load(open(os.path.join(GOLDEN, "cl20.json")))
    n, s, d = synth.workload("cl20")
    g = gpu.tc_build_csr(n, torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda())
    per, ests, mom = _timed("cl20 64 seeds", lambda: gpu.tc_estimate(g, gold["p"], gold["seeds"],
                                                                      num_groups=gold["groups"]))
    assert [c["triangles"] for c in per] == gold["triangles"]
    assert mom == gold["median_of_means"]
    assert gpu.tc_count_exact(g)["triangles"] == gold["exact"]["triangles"]


@pytest.mark.parametrize("h", [1000, 2048, 4096, 17000])
def test_top_degree_block_all_heavy_matches_oracle(gpu, rmat22, rmat22_oracle, h):
    # the dense subgraph induced by the h highest-degree vertices of R-MAT s22,
    # counted with every vertex heavy: the whole count runs in the int8-MFMA
    # block (h = 1000 leaves a ragged last macro tile; h = 17000 pads to 17024,
    # so the rows of U are built in two LDS chunks of columns).  The oracle's
    # count of the largest block is stored (tests/golden/make_golden.py).
    import torch
    n, s, d, g = rmat22
    deg = np.diff(rmat22_oracle[1])
    order = np.lexsort((np.arange(n), deg))[::-1][:h]
    lab = np.full(n, -1, np.int64)
    lab[order] = np.arange(h)
    keep = (lab[s] >= 0) & (lab[d] >= 0)
    hs, hd = lab[s[keep]].astype(np.int32), lab[d[keep]].astype(np.int32)
    stored = json.load(open(os.path.join(GOLDEN, "rmat22_top.json")))["blocks"]
    if str(h) in stored:
        want = stored[str(h)]["triangles"]
    else:
        want = oracle.count(oracle.normalise(h, hs, hd))
    sg = gpu.tc_build_csr(h, torch.from_numpy(hs).cuda(), torch.from_numpy(hd).cuda())
    c = gpu.tc_count_exact(sg, heavy=(0, 1))
    _log("top-%d block: m=%d T=%d n_heavy=%d" % (h, c["m"], c["triangles"], c["n_heavy"]))
    if str(h) in stored:
        assert c["m"] == stored[str(h)]["m"]
    if h > 16384:
        assert c["n_heavy"] > 16384  # more than one LDS chunk per row of U
    assert c["triangles"] == want and c["heavy"] == want and c["light"] == 0
    assert gpu.tc_count_exact(sg)["triangles"] == want
    sg.free()
