"""Small named graphs with known triangle counts, as raw (n, src, dst) edge lists.

Closed forms used by the tests: K_n has C(n,3) triangles; the complete
tripartite K_{a,b,c} has a*b*c; the wheel W_n (hub plus a cycle on n-1 >= 4
rim vertices) has n-1; the friendship graph F_k has k; bipartite graphs,
trees, stars, even cycles and the Petersen graph have none.
"""
import itertools

import numpy as np


def _pack(n, pairs):
    if len(pairs) == 0:
        return n, np.zeros(0, np.int32), np.zeros(0, np.int32)
    a = np.asarray(pairs, dtype=np.int32)
    return n, a[:, 0].copy(), a[:, 1].copy()


def complete(n):
    return _pack(n, list(itertools.combinations(range(n), 2)))


def complete_multipartite(sizes):
    parts, base = [], 0
    for s in sizes:
        parts.append(list(range(base, base + s)))
        base += s
    pairs = []
    for i in range(len(parts)):
        for j in range(i + 1, len(parts)):
            pairs += [(u, v) for u in parts[i] for v in parts[j]]
    return _pack(base, pairs)


def wheel(n):
    """Hub 0 joined to a cycle on vertices 1..n-1."""
    rim = n - 1
    pairs = [(0, i) for i in range(1, n)]
    pairs += [(1 + i, 1 + (i + 1) % rim) for i in range(rim)]
    return _pack(n, pairs)


def friendship(k):
    """k triangles sharing the single vertex 0."""
    pairs = []
    for i in range(k):
        a, b = 1 + 2 * i, 2 + 2 * i
        pairs += [(0, a), (0, b), (a, b)]
    return _pack(2 * k + 1, pairs)


def star(n):
    return _pack(n, [(0, i) for i in range(1, n)])


def cycle(n):
    return _pack(n, [(i, (i + 1) % n) for i in range(n)])


def path(n):
    return _pack(n, [(i, i + 1) for i in range(n - 1)])


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return _pack(10, outer + spokes + inner)


def disjoint_union(*graphs):
    n_tot, srcs, dsts = 0, [], []
    for n, s, d in graphs:
        srcs.append(s + n_tot)
        dsts.append(d + n_tot)
        n_tot += n
    return n_tot, np.concatenate(srcs).astype(np.int32), np.concatenate(dsts).astype(np.int32)


def relabel(graph, perm):
    n, s, d = graph
    perm = np.asarray(perm, dtype=np.int32)
    return n, perm[s], perm[d]
