"""CPU oracle (TEST INFRASTRUCTURE ONLY).

Python bindings for ``oracle/tc_oracle.c``: a plain, slow, single-threaded
implementation of what the device path computes, written from the paper
(Kolountzakis, Miller, Peng, Tsourakakis, arXiv:1011.0468).  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import this module;
the product package never does.  It imports nothing from the product package.

All functions take / return numpy arrays.  A normalised graph is the tuple
``(n, row_ptr int64[n+1], col int32[2m])`` with sorted neighbour lists.
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build():
    """Compile the oracle with gcc: no fast-math, no floating-point contraction."""
    src = os.path.join(_HERE, "tc_oracle.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
                           "-fno-fast-math", "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    L = ctypes.CDLL(_SO)
    i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    P = ctypes.POINTER
    L.or_normalise.argtypes = [i64, i64, P(i32), P(i32), P(i64), P(i32), P(i64)]
    L.or_normalise.restype = ctypes.c_int
    L.or_mix64.argtypes = [u64]
    L.or_mix64.restype = u64
    L.or_keep_threshold.argtypes = [dbl]
    L.or_keep_threshold.restype = u64
    L.or_keep.argtypes = [i32, i32, u64, u64]
    L.or_keep.restype = ctypes.c_int
    L.or_sample.argtypes = [i64, P(i64), P(i32), dbl, u64, P(i64), P(i32)]
    L.or_sample.restype = i64
    L.or_count_triangles.argtypes = [i64, P(i64), P(i32), P(i64)]
    L.or_count_triangles.restype = i64
    L.or_count_triangles_idorder.argtypes = [i64, P(i64), P(i32)]
    L.or_count_triangles_idorder.restype = i64
    L.or_count_bruteforce.argtypes = [i64, P(ctypes.c_uint8)]
    L.or_count_bruteforce.restype = i64
    L.or_is_heavy.argtypes = [i64, i64, i32, i32]
    L.or_is_heavy.restype = ctypes.c_int
    L.or_count_split.argtypes = [i64, P(i64), P(i32), i32, i32, P(i64)]
    L.or_count_split.restype = ctypes.c_int
    L.or_estimate.argtypes = [i64, dbl]
    L.or_estimate.restype = dbl
    L.or_median_of_means.argtypes = [P(i64), i32, i32, dbl]
    L.or_median_of_means.restype = dbl
    L.or_rp_sign.argtypes = [u64, i64, i64]
    L.or_rp_sign.restype = ctypes.c_int
    L.or_quadform_a3.argtypes = [i64, P(i64), P(i32), P(i64)]
    L.or_quadform_a3.restype = i64
    L.or_rp_trace.argtypes = [i64, P(i64), P(i32), i32, u64, P(i64), P(dbl)]
    L.or_rp_trace.restype = ctypes.c_int
    L.or_rp_q.argtypes = [i64, P(i64), P(i32), i64, u64]
    L.or_rp_q.restype = i64
    L.or_triples_size.argtypes = [i64, P(i64), P(i32), ctypes.c_int, P(i64)]
    L.or_triples_size.restype = i64
    L.or_triple_at.argtypes = [i64, P(i64), P(i32), ctypes.c_int, P(i64), i64, P(i32), P(i32), P(i32)]
    L.or_triple_at.restype = i64
    L.or_triple_index.argtypes = [u64, i64, i64]
    L.or_triple_index.restype = i64
    L.or_triple_sample.argtypes = [i64, P(i64), P(i32), ctypes.c_int, i64, u64, P(i64)]
    L.or_triple_sample.restype = ctypes.c_int
    L.or_triple_estimate.argtypes = [i64, i64, i64, dbl]
    L.or_triple_estimate.restype = dbl
    L.or_stream_draws.argtypes = [i64, i64, dbl]
    L.or_stream_draws.restype = i64
    L.or_stream_closed_all.argtypes = [i64, P(i64), P(i32), P(ctypes.c_uint8)]
    L.or_stream_closed_all.restype = i64
    L.or_stream_estimate.argtypes = [i64, P(i64), P(i32), dbl, i64, u64, P(i64), P(ctypes.c_uint8)]
    L.or_stream_estimate.restype = ctypes.c_int
    L.or_stream_value.argtypes = [i64, i64, i64]
    L.or_stream_value.restype = dbl
    _lib = L
    return L


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _i64(a):
    return _p(a, ctypes.c_int64)


def _i32(a):
    return _p(a, ctypes.c_int32)


def normalise(n, src, dst):
    """Simple undirected graph of the pairs: returns (n, row_ptr, col)."""
    L = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    rp = np.empty(n + 1, np.int64)
    col = np.empty(max(2 * len(src), 1), np.int32)
    m = ctypes.c_int64(0)
    rc = L.or_normalise(n, len(src), _i32(src), _i32(dst), _i64(rp), _i32(col), ctypes.byref(m))
    if rc == 1:
        raise ValueError("vertex id out of range")
    if rc:
        raise MemoryError("oracle normalise")
    return n, rp, col[: 2 * m.value].copy()


def mix64(z):
    return int(_load().or_mix64(z & 0xFFFFFFFFFFFFFFFF))


def keep_threshold(p):
    return int(_load().or_keep_threshold(p))


def keep(u, v, seed, p):
    L = _load()
    return bool(L.or_keep(u, v, seed, L.or_keep_threshold(p)))


def sample(g, p, seed):
    """G_p as (n, row_ptr_p, col_p); m' = len(col_p) // 2."""
    n, rp, col = g
    L = _load()
    rpp = np.empty(n + 1, np.int64)
    colp = np.empty(max(len(col), 1), np.int32)
    L.or_sample(n, _i64(rp), _i32(col), p, seed, _i64(rpp), _i32(colp))
    return n, rpp, colp[: rpp[n]].copy()


def count(g, per_vertex=False):
    """Triangle count (degree-ordered merge); optionally per lowest-ranked vertex."""
    n, rp, col = g
    L = _load()
    pv = np.zeros(n, np.int64) if per_vertex else None
    t = L.or_count_triangles(n, _i64(rp), _i32(col), _i64(pv) if per_vertex else None)
    if t < 0:
        raise MemoryError("oracle count")
    return (int(t), pv) if per_vertex else int(t)


def count_idorder(g):
    n, rp, col = g
    return int(_load().or_count_triangles_idorder(n, _i64(rp), _i32(col)))


def count_bruteforce(adj):
    adj = np.ascontiguousarray(adj, dtype=np.uint8)
    return int(_load().or_count_bruteforce(adj.shape[0], _p(adj, ctypes.c_uint8)))


def is_heavy(deg, m, a=1, b=1):
    return bool(_load().or_is_heavy(deg, m, a, b))


def count_split(g, a=1, b=1):
    """dict(triangles, light, heavy, n_heavy, m) for the light/heavy split a/b."""
    n, rp, col = g
    out = np.zeros(5, np.int64)
    rc = _load().or_count_split(n, _i64(rp), _i32(col), a, b, _i64(out))
    if rc:
        raise MemoryError("oracle split")
    return dict(triangles=int(out[0]), light=int(out[1]), heavy=int(out[2]),
                n_heavy=int(out[3]), m=int(out[4]))


def estimate(T, p):
    return float(_load().or_estimate(int(T), float(p)))


def median_of_means(counts, num_groups, p):
    c = np.ascontiguousarray(counts, dtype=np.int64)
    return float(_load().or_median_of_means(_i64(c), len(c), num_groups, float(p)))


def triples_size(g, hybrid, with_prefix=False):
    """|U| of section 3.2's triple sampling (wedges; extensions for deg^2 > m
    when hybrid), and the start of each vertex's triples if with_prefix."""
    n, rp, col = g
    pre = np.zeros(n + 1, np.int64)
    size = int(_load().or_triples_size(n, _i64(rp), _i32(col), 1 if hybrid else 0, _i64(pre)))
    return (size, pre) if with_prefix else size


def triple_at(g, hybrid, prefix, r):
    """((x, y, z), weight if closed else 0) of triple r of U."""
    n, rp, col = g
    x, y, z = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    w = _load().or_triple_at(n, _i64(rp), _i32(col), 1 if hybrid else 0, _i64(prefix), int(r), ctypes.byref(x),
                             ctypes.byref(y), ctypes.byref(z))
    return (x.value, y.value, z.value), int(w)


def triple_index(seed, i, size):
    return int(_load().or_triple_index(seed & (2 ** 64 - 1), i, size))


def triple_sample(g, hybrid, s, seed):
    """(|U|, weight sum, closed samples) of s samples of U."""
    n, rp, col = g
    out = np.zeros(3, np.int64)
    if _load().or_triple_sample(n, _i64(rp), _i32(col), 1 if hybrid else 0, s, seed & (2 ** 64 - 1), _i64(out)):
        raise MemoryError("oracle triples")
    return int(out[0]), int(out[1]), int(out[2])


def triple_estimate(size, wsum, s, p=1.0):
    return float(_load().or_triple_estimate(size, wsum, s, float(p)))


def balance_p(m, n, t, eps):
    """Section 3.3: the p at which the sampling term p m equals the counting
    term m^(3/2) log n / (p^(3/2) t eps^2), i.e. (m^(1/2) ln n / (t eps^2))^(2/5),
    capped at 1 (1 when t <= 0 or eps = 0; natural logarithm)."""
    if t <= 0 or eps == 0:
        return 1.0
    return min(1.0, (math.sqrt(m) * math.log(n) / (t * (eps * eps))) ** 0.4)


def estimate_adaptive(g, p0, tol, seed0, num_seeds, num_groups, max_stages=32):
    """Vary p until the estimate settles (the remarks after Table 2): stage k
    samples with p = min(1, p0 2^k) and the seeds seed0 + k num_seeds + i,
    counts each sample exactly and takes the median of means (section 3.1
    rescaling); the search ends after the first stage k >= 1 with E_k > 0 and
    |E_k - E_(k-1)| <= tol E_k, after the stage at p = 1, or after
    max_stages stages.  An estimate of 0 never counts as settled (a sample
    without triangles says nothing about the rate).  Returns ([(p, estimate,
    sum of m')], balance_p of the last estimate)."""
    n, rp, col = g
    m = len(col) // 2
    stages = []
    prev = 0.0
    for k in range(max_stages):
        p = min(1.0, math.ldexp(p0, k))
        counts, msum = [], 0
        for i in range(num_seeds):
            seed = (seed0 + k * num_seeds + i) % (1 << 64)
            gs = g if p >= 1.0 else sample(g, p, seed)
            counts.append(count(gs))
            msum += len(gs[2]) // 2
        est = median_of_means(counts, num_groups, p)
        stages.append((p, est, msum))
        if p >= 1.0 or (k >= 1 and est > 0.0 and abs(est - prev) <= tol * est):
            break
        prev = est
    return stages, balance_p(m, n, stages[-1][1], tol)


def rp_sign(seed, l, i):
    return int(_load().or_rp_sign(seed, l, i))


def quadform_a3(g, x):
    n, rp, col = g
    x = np.ascontiguousarray(x, dtype=np.int64)
    return int(_load().or_quadform_a3(n, _i64(rp), _i32(col), _i64(x)))


def rp_trace(g, k, seed):
    """(q int64[k], triangle estimate)."""
    n, rp, col = g
    q = np.zeros(k, np.int64)
    est = ctypes.c_double(0.0)
    rc = _load().or_rp_trace(n, _i64(rp), _i32(col), k, seed, _i64(q), ctypes.byref(est))
    if rc:
        raise MemoryError("oracle rp")
    return q, est.value


def rp_q(g, l, seed):
    n, rp, col = g
    return int(_load().or_rp_q(n, _i64(rp), _i32(col), l, seed))


def dense_adjacency(g):
    n, rp, col = g
    A = np.zeros((n, n), np.uint8)
    for u in range(n):
        A[u, col[rp[u]:rp[u + 1]]] = 1
    return A


def stream_draws(n, m, d):
    """Pass 1 of the semi-streaming variant: ceil(d m^(1/2) ln n) edge draws."""
    return int(_load().or_stream_draws(n, m, float(d)))


def stream_closed_all(g, heavy):
    """Closed elements among all of the semi-streaming triple set U for the
    heavy set given by the flags ``heavy`` (every element counted once)."""
    n, rp, col = g
    h = np.ascontiguousarray(heavy, dtype=np.uint8)
    return int(_load().or_stream_closed_all(n, _i64(rp), _i32(col), _p(h, ctypes.c_uint8)))


def stream_estimate(g, d, s, seed):
    """Semi-streaming three-pass estimate (section 5.2): dict(draws1,
    candidates, heavy, light_size, size, queries, closed, m, estimate) and
    the flags of the heavy set."""
    n, rp, col = g
    out = np.zeros(8, np.int64)
    heavy = np.zeros(max(n, 1), np.uint8)
    rc = _load().or_stream_estimate(n, _i64(rp), _i32(col), float(d), int(s), seed & (2 ** 64 - 1), _i64(out),
                                    _p(heavy, ctypes.c_uint8))
    if rc:
        raise MemoryError("oracle stream")
    keys = ("draws1", "candidates", "heavy", "light_size", "size", "queries", "closed", "m")
    r = {k: int(v) for k, v in zip(keys, out)}
    r["estimate"] = float(_load().or_stream_value(r["size"], r["closed"], int(s))) if s > 0 else 0.0
    return r, heavy[:n].astype(bool)
