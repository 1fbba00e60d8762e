"""Work statistics of the light phase's schedule, from a normalised graph
(n, row_ptr, col): what the closure kernels must stream for a given heavy
split and v-major staging cap.  Test-side model of the scheduling rule (not
of the count, which the oracle fixes):

  orientation u -> v iff (deg u, u) < (deg v, v); light sources are the light
  vertices with d+ >= 2 (heavy iff b^2 deg^2 > a^2 m);
  N+(u) of a light source in rank order when d+(u) <= sort_cap;
  pair (u, v), v at position k of N+(u): len = d+(u) - 1 - k (sorted) or
  d+(u) (unsorted); no work if len = 0; else len entries streamed if
  len <= d+(v) <= vcap (v-major), d+(v) entries otherwise;
  gather = sum of d+(v) over all pairs.
"""
import numpy as np

SORT_CAP = 1024


def light_work(g, a, b, vcap, sort_cap=SORT_CAP):
    n, rp, col = g
    rp = np.asarray(rp, np.int64)
    col = np.asarray(col, np.int64)
    deg = np.diff(rp)
    m = len(col) // 2
    row = np.repeat(np.arange(n, dtype=np.int64), deg)
    key = deg * n + np.arange(n, dtype=np.int64)
    up = key[row] < key[col]
    u, v = row[up], col[up]
    dplus = np.bincount(u, minlength=n)
    heavy = (deg > 0) & (b * b * deg * deg > a * a * m)
    srcv = (~heavy) & (dplus >= 2)
    sel = srcv[u]
    u, v = u[sel], v[sel]
    o = np.lexsort((key[v], u))
    u, v = u[o], v[o]
    k = np.arange(len(u)) - np.searchsorted(u, u, side="left")
    d = dplus[u]
    dv = dplus[v]
    ln = np.where(d <= sort_cap, d - 1 - k, d)
    vm = (ln <= dv) & (dv <= vcap)
    probes = np.where(ln == 0, 0, np.where(vm, ln, dv))
    return dict(probes=int(probes.sum()), gather=int(dv.sum()), vmajor=int((vm & (ln > 0)).sum()),
                skipped=int((ln == 0).sum()))
