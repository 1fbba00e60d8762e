"""Write the oracle's expected values for the full-size workloads.

Calls only the CPU oracle (oracle/) on inputs from the seeded generators
(synth/); nothing here touches the device path.  Usage:

    python tests/golden/make_golden.py rmat22 rmat22_splits cl20 rmat24 rmat24_count rmat22_top serve20 stream22 cl16k

Each section writes tests/golden/<name>.json.
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

_G = {}


def _graph(name):
    if name not in _G:
        _G[name] = oracle.normalise(*synth.workload(name))
    return _G[name]


def _count_job(args):
    name, p, seed = args
    g = _graph(name)
    t = time.time()
    gp = g if p == 1.0 else oracle.sample(g, p, seed)
    r = oracle.count_split(gp, 1, 1)
    r.update(p=p, seed=seed, oracle_seconds=round(time.time() - t, 2))
    return r


def rmat22():
    jobs = [("rmat22", p, 0) for p in (1.0, 0.5, 0.1, 0.05)]
    with mp.Pool(4) as pool:
        res = pool.map(_count_job, jobs)
    return {"workload": "R-MAT scale 22, edge factor 16, a/b/c = .57/.19/.19, generator seed 1",
            "split": [1, 1], "counts": res}


def cl20():
    g = _graph("cl20")
    counts = []
    for s in range(64):
        counts.append(oracle.count(oracle.sample(g, 0.05, s)))
    return {"workload": "Chung-Lu n=2^20, avg degree 32, beta 2.2, generator seed 1",
            "p": 0.05, "seeds": list(range(64)), "groups": 8, "triangles": counts,
            "median_of_means": oracle.median_of_means(counts, 8, 0.05),
            "exact": oracle.count_split(g, 1, 1)}


def _rp_job(args):
    name, l, seed = args
    return oracle.rp_q(_graph(name), l, seed)


def rmat24():
    # every one of the k = 256 vectors, one by one; the graph is normalised in
    # the parent so that the forked workers share it
    k = 256
    g = _graph("rmat24")
    with mp.Pool(8) as pool:
        qs = pool.map(_rp_job, [("rmat24", l, 0) for l in range(k)], chunksize=4)
    return {"workload": "R-MAT scale 24, edge factor 16, a/b/c = .57/.19/.19, generator seed 1",
            "k": k, "seed": 0, "q": [int(q) for q in qs], "m": int(len(g[2]) // 2)}


def _split_job(args):
    name, p, seed, a, b = args
    g = _graph(name)
    t = time.time()
    gp = g if p == 1.0 else oracle.sample(g, p, seed)
    r = oracle.count_split(gp, a, b)
    r.update(p=p, seed=seed, split=[a, b], oracle_seconds=round(time.time() - t, 2))
    return r


def rmat22_splits():
    # the light/heavy split of every operating point of the benchmark (p = 1,
    # 0.5, 0.1, 0.05, seed 0) for every heavy multiplier c = a/b the autotuner
    # may pick (1/4, 1/2, 2; c = 1 is in rmat22.json)
    _graph("rmat22")
    jobs = [("rmat22", p, 0, a, b) for p in (1.0, 0.5, 0.1, 0.05) for a, b in ((1, 4), (1, 2), (2, 1))]
    with mp.Pool(6) as pool:
        res = pool.map(_split_job, jobs, chunksize=1)
    return {"workload": "R-MAT scale 22, edge factor 16, a/b/c = .57/.19/.19, generator seed 1",
            "counts": res}


def serve20():
    # the scale-20 end of the serving mix (request 0's generator seed) at the
    # three keep probabilities of the mix, sample seeds 0, 1, 2
    n, s, d = synth.serving_graph(0, 20)
    g = oracle.normalise(n, s, d)
    out = []
    for seed, p in enumerate((1.0, 0.5, 0.1)):
        gp = g if p == 1.0 else oracle.sample(g, p, seed)
        r = oracle.count_split(gp, 1, 1)
        r.update(p=p, seed=seed)
        out.append(r)
    return {"workload": "R-MAT scale 20, edge factor 16, a/b/c = .57/.19/.19, generator seed 1000 (serving request 0)",
            "n": n, "pairs": int(len(s)), "counts": out}


def rmat24_count():
    g = _graph("rmat24")
    return {"workload": "R-MAT scale 24, edge factor 16, a/b/c = .57/.19/.19, generator seed 1",
            "split": [1, 1], "exact": oracle.count_split(g, 1, 1)}


def rmat22_top():
    # the subgraph induced by the h highest-degree vertices (degree, then id,
    # descending) of R-MAT s22, relabelled 0..h-1 in that order; counted by the
    # oracle (about a minute for h = 17000)
    import numpy as np
    n, s, d = synth.workload("rmat22")
    deg = np.diff(_graph("rmat22")[1])
    out = {}
    for h in (17000,):
        order = np.lexsort((np.arange(n), deg))[::-1][:h]
        lab = np.full(n, -1, np.int64)
        lab[order] = np.arange(h)
        keep = (lab[s] >= 0) & (lab[d] >= 0)
        sub = oracle.normalise(h, lab[s[keep]].astype(np.int32), lab[d[keep]].astype(np.int32))
        out[str(h)] = {"m": int(len(sub[2]) // 2), "triangles": int(oracle.count(sub))}
    return {"workload": "R-MAT scale 22 (generator seed 1), subgraph induced by the top-h degree vertices",
            "blocks": out}


def cl16k():
    # the small Chung-Lu configuration: exact count and the p = 0.25 sample
    # of seed 0, with the light/heavy split at c = 1
    g = _graph("cl16k")
    out = []
    for p, seed in ((1.0, 0), (0.25, 0)):
        gp = g if p == 1.0 else oracle.sample(g, p, seed)
        r = oracle.count_split(gp, 1, 1)
        r.update(p=p, seed=seed)
        out.append(r)
    return {"workload": "Chung-Lu n=16384, avg degree 12, beta 2.5, generator seed 1", "counts": out}


def stream22():
    # the semi-streaming estimate (section 5.2) of the benchmark's stream
    # workload: d = 1, 2^24 pass-2 draws, seeds 0 and 1
    g = _graph("rmat22")
    runs = []
    for seed in (0, 1):
        t = time.time()
        r, heavy = oracle.stream_estimate(g, 1.0, 1 << 24, seed)
        r.update(d=1.0, num_samples=1 << 24, seed=seed, oracle_seconds=round(time.time() - t, 2))
        runs.append(r)
    return {"workload": "R-MAT scale 22, edge factor 16, a/b/c = .57/.19/.19, generator seed 1", "runs": runs,
            "exact": oracle.count(g)}


if __name__ == "__main__":
    for name in sys.argv[1:]:
        t = time.time()
        out = globals()[name]()
        out["generated_by"] = "tests/golden/make_golden.py (CPU oracle only)"
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f, indent=1)
        print(name, "done in %.1fs" % (time.time() - t), flush=True)
