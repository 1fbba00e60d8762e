"""Write the oracle's expected values for the full-size workloads.

Calls only the CPU oracle (oracle/) on inputs from the seeded generators
(synth/); nothing here touches the device path.  Usage:

    python tests/golden/make_golden.py rmat22 cl20 rmat24 rmat24_count rmat22_top

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
    ls = [0, 1, 63, 64, 127, 200, 255]
    with mp.Pool(4) as pool:
        qs = pool.map(_rp_job, [("rmat24", l, 0) for l in ls])
    g = _graph("rmat24")
    return {"workload": "R-MAT scale 24, edge factor 16, a/b/c = .57/.19/.19, generator seed 1",
            "k": 256, "seed": 0, "sampled_q": {str(l): int(q) for l, q in zip(ls, qs)},
            "m": int(len(g[2]) // 2)}


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


if __name__ == "__main__":
    for name in sys.argv[1:]:
        t = time.time()
        out = globals()[name]()
        out["generated_by"] = "tests/golden/make_golden.py (CPU oracle only)"
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f, indent=1)
        print(name, "done in %.1fs" % (time.time() - t), flush=True)
