"""Seeded synthetic inputs shared by the oracle, the device path, the tests and
the benchmark.

Everything here produces *raw* edge lists (int32 ``src``/``dst`` numpy arrays
that may contain duplicate pairs and self-loops) or request traces.  No part of
the triangle-counting method lives here.

Workload recipes (shapes follow the paper's power-law social/web graphs,
Table 1 and section 4.1):

* ``rmat(scale, edge_factor=16, a=.57, b=.19, c=.19, seed=1)``: R-MAT with
  ``edge_factor * 2**scale`` pairs, 16-bit quadrant thresholds, no noise, then
  a seeded random relabelling of all ``2**scale`` vertices.
* ``chung_lu(n, avg_deg, beta, seed=1)``: Chung-Lu with weights
  ``w_i = C i^(-1/(beta-1))`` and ``P(ij) = min(1, w_i w_j / sum w)``; exact
  per-pair coins for ``n <= 65536``, the Miller-Hagberg skipping method above,
  then a seeded relabelling.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None


def build():
    """Compile the generator library with gcc (host code only)."""
    src = os.path.join(_HERE, "gen.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.synth_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_uint64, ctypes.c_int32, i32p, i32p]
    lib.synth_chung_lu.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, i32p, i32p,
                                   ctypes.POINTER(ctypes.c_int64)]
    lib.synth_uniform_pairs.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, i32p, i32p]
    lib.synth_poisson_arrivals.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                           ctypes.POINTER(ctypes.c_double)]
    lib.synth_uniform_ints.argtypes = [ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, i32p]
    for f in (lib.synth_rmat, lib.synth_chung_lu, lib.synth_uniform_pairs,
              lib.synth_poisson_arrivals, lib.synth_uniform_ints):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def rmat(scale, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=1, permute=True):
    """Return (n, src, dst) for an R-MAT graph of 2**scale vertices."""
    lib = _load()
    ne = int(edge_factor) << int(scale)
    src = np.empty(ne, dtype=np.int32)
    dst = np.empty(ne, dtype=np.int32)
    rc = lib.synth_rmat(scale, ne, a, b, c, seed, 1 if permute else 0, _p32(src), _p32(dst))
    if rc:
        raise RuntimeError("synth_rmat failed: %d" % rc)
    return 1 << int(scale), src, dst


def chung_lu(n, avg_deg, beta, seed=1, permute=True, exact=None):
    """Return (n, src, dst) for a Chung-Lu graph."""
    lib = _load()
    if exact is None:
        exact = n <= 65536
    cap = int(n * avg_deg * 0.75 + 64 * np.sqrt(n * avg_deg) + 1024)
    while True:
        src = np.empty(cap, dtype=np.int32)
        dst = np.empty(cap, dtype=np.int32)
        cnt = ctypes.c_int64(0)
        rc = lib.synth_chung_lu(n, avg_deg, beta, seed, 0 if exact else 1, 1 if permute else 0,
                                cap, _p32(src), _p32(dst), ctypes.byref(cnt))
        if rc == 3:
            cap *= 2
            continue
        if rc:
            raise RuntimeError("synth_chung_lu failed: %d" % rc)
        k = cnt.value
        return n, src[:k].copy(), dst[:k].copy()


def uniform_pairs(n, num_pairs, seed):
    """Uniform random (src, dst) pairs in [0,n): a multigraph with loops, for tests."""
    lib = _load()
    src = np.empty(num_pairs, dtype=np.int32)
    dst = np.empty(num_pairs, dtype=np.int32)
    rc = lib.synth_uniform_pairs(n, num_pairs, seed, _p32(src), _p32(dst))
    if rc:
        raise RuntimeError("synth_uniform_pairs failed")
    return n, src, dst


def poisson_arrivals(count, lam, seed):
    """Arrival times (seconds) of a Poisson process with rate ``lam`` per second."""
    lib = _load()
    out = np.empty(count, dtype=np.float64)
    rc = lib.synth_poisson_arrivals(count, lam, seed, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc:
        raise RuntimeError("synth_poisson_arrivals failed")
    return out


def uniform_ints(count, bound, seed, stream=0x494e5453):
    """``count`` integers uniform in [0, bound)."""
    lib = _load()
    out = np.empty(count, dtype=np.int32)
    rc = lib.synth_uniform_ints(count, bound, seed, stream, _p32(out))
    if rc:
        raise RuntimeError("synth_uniform_ints failed")
    return out


# ---- named workloads -------------------------------------------------------

_CACHE = {}


SERVE_P = (1.0, 0.5, 0.1)


def serving_requests(count, scale_lo=10, scale_hi=20, seed=12345):
    """Request mix of the serving workload: request i is an R-MAT graph of
    scale ``scale[i]`` uniform in [scale_lo, scale_hi] (edge factor 16,
    generator seed 1000 + i) counted at p uniform in {1, .5, .1} with sample
    seed i.  Returns (scales int32[count], p float64[count])."""
    scales = uniform_ints(count, scale_hi - scale_lo + 1, seed, stream=0x5343414C) + scale_lo
    pidx = uniform_ints(count, len(SERVE_P), seed, stream=0x50524F42)
    return scales.astype(np.int32), np.array([SERVE_P[k] for k in pidx], dtype=np.float64)


def serving_graph(i, scale):
    """Pairs of serving request i (R-MAT, edge factor 16, seed 1000 + i)."""
    return rmat(int(scale), 16, seed=1000 + int(i))


def workload(name):
    """Named synthetic workloads, cached per process.

    cl16k   : Chung-Lu n=16384, avg degree 12, beta 2.5 (exact per-pair coins)
    rmat22  : R-MAT scale 22, edge factor 16
    cl20    : Chung-Lu n=2**20, avg degree 32, beta 2.2 (skipping method)
    rmat24  : R-MAT scale 24, edge factor 16
    rmatS   : R-MAT scale S (serving requests use their own seeds, see ``rmat``)
    """
    if name in _CACHE:
        return _CACHE[name]
    if name == "cl16k":
        g = chung_lu(16384, 12.0, 2.5, seed=1)
    elif name == "cl20":
        g = chung_lu(1 << 20, 32.0, 2.2, seed=1)
    elif name.startswith("rmat"):
        g = rmat(int(name[4:]), 16, seed=1)
    else:
        raise KeyError(name)
    _CACHE[name] = g
    return g
