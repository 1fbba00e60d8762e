"""Degree-partitioned sampling triangle counter for one MI355X (gfx950).

Thin Python binding over the C ABI of ``libtc.so`` (``include/tc.h``): it only
marshals arguments.  Every step of the counting path runs in the library's
HIP kernels; PyTorch supplies device memory for inputs and the stream.

The method is Kolountzakis, Miller, Peng, Tsourakakis, "Efficient Triangle
Counting in Large Graphs via Degree-based Vertex Partitioning"
(arXiv:1011.0468): edge sparsification (section 3.1), light/heavy vertex
partition (section 3.2), exact count rescaled by 1/p^3, and the random
projection estimator of section 5.1.
"""
import ctypes

import numpy as np

from . import _native
from ._native import (TcCounts, TcError, TcParams, TcRequest, TcResult, TcServerConfig, TcServerInfo, TcStage, TcStreamResult, TcTripleResult, TcTuning,
                      check)

__all__ = ["Graph", "tc_build_csr", "tc_sample", "tc_count_exact", "tc_estimate", "tc_estimate_adaptive", "tc_triple_estimate", "tc_stream_estimate", "tc_rp_trace",
           "tc_graph_info", "tc_graph_read", "tc_tune_set", "tc_tune_get", "tc_autotune", "profile", "TcError",
           "Server", "tc_request_bytes"]


def _stream_ptr(stream):
    if stream is not None:
        return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    import torch
    if torch.cuda.is_available():
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(0)


def _params(heavy=(1, 1), tuned=False):
    return TcParams(int(heavy[0]), int(heavy[1]), 1 if tuned else 0)


class Graph:
    """Owning wrapper of a ``tc_graph`` handle (freed with the object)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def info(self):
        return tc_graph_info(self)

    def read(self, stream=None):
        return tc_graph_read(self, stream)

    def free(self):
        if self._h and self._h.value:
            _native.load().tc_graph_free(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def tc_build_csr(n, src, dst, stream=None):
    """Simple undirected graph of the pairs (src[i], dst[i]).

    ``src``/``dst``: int32 torch tensors (CUDA: read in place; CPU: copied in)
    or numpy arrays (copied in)."""
    L = _native.load()
    keep = []
    if isinstance(src, np.ndarray):
        s = np.ascontiguousarray(src, dtype=np.int32)
        d = np.ascontiguousarray(dst, dtype=np.int32)
        keep += [s, d]
        ps, pd, on_dev = s.ctypes.data, d.ctypes.data, 0
    else:
        import torch
        s = src.to(torch.int32).contiguous()
        d = dst.to(torch.int32).contiguous()
        keep += [s, d]
        ps, pd, on_dev = s.data_ptr(), d.data_ptr(), 1 if s.is_cuda else 0
    if len(s) != len(d):
        raise ValueError("src and dst differ in length")
    out = ctypes.c_void_p(0)
    check(L.tc_build_csr(int(n), len(s), ctypes.c_void_p(ps), ctypes.c_void_p(pd), on_dev, _stream_ptr(stream),
                         ctypes.byref(out)))
    return Graph(out.value)


def tc_graph_info(g):
    n, m, md = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    check(_native.load().tc_graph_info(g.handle, ctypes.byref(n), ctypes.byref(m), ctypes.byref(md)))
    return dict(n=n.value, m=m.value, max_deg=md.value)


def tc_graph_read(g, stream=None):
    """(row_ptr, col, deg) as host numpy int32 arrays."""
    inf = tc_graph_info(g)
    rp = np.empty(inf["n"] + 1, np.int32)
    col = np.empty(max(2 * inf["m"], 1), np.int32)
    deg = np.empty(max(inf["n"], 1), np.int32)
    check(_native.load().tc_graph_read(g.handle, ctypes.c_void_p(rp.ctypes.data), ctypes.c_void_p(col.ctypes.data),
                                       ctypes.c_void_p(deg.ctypes.data), 0, _stream_ptr(stream)))
    return rp, col[: 2 * inf["m"]], deg[: inf["n"]]


def tc_sample(g, p, seed, stream=None):
    out = ctypes.c_void_p(0)
    check(_native.load().tc_sample(g.handle, float(p), int(seed) & (2 ** 64 - 1), _stream_ptr(stream),
                                   ctypes.byref(out)))
    return Graph(out.value)


def tc_count_exact(g, heavy=(1, 1), tuned=False, stream=None):
    c = TcCounts()
    prm = _params(heavy, tuned)
    check(_native.load().tc_count_exact(g.handle, ctypes.byref(prm), _stream_ptr(stream), ctypes.byref(c)))
    return c.as_dict()


def tc_estimate(g, p, seeds, num_groups=1, heavy=(1, 1), tuned=False, stream=None):
    """Returns (per_seed counts list, per_seed estimates list, median of means)."""
    seeds = [int(s) & (2 ** 64 - 1) for s in seeds]
    S = len(seeds)
    arr = (ctypes.c_uint64 * S)(*seeds)
    per = (TcCounts * S)()
    ests = (ctypes.c_double * S)()
    mom = ctypes.c_double(0.0)
    prm = _params(heavy, tuned)
    check(_native.load().tc_estimate(g.handle, float(p), arr, S, int(num_groups), ctypes.byref(prm),
                                     _stream_ptr(stream), per, ests, ctypes.byref(mom)))
    return [c.as_dict() for c in per], list(ests), mom.value


def tc_estimate_noalloc(g, p, seed, heavy=(1, 1), tuned=False, stream=None):
    """Single-seed estimate whose buffers all live in the library's fixed
    device scratch array (no device allocation): (counts dict, estimate)."""
    c = TcCounts()
    est = ctypes.c_double(0.0)
    prm = _params(heavy, tuned)
    check(_native.load().tc_estimate_noalloc(g.handle, float(p), int(seed) & (2 ** 64 - 1), ctypes.byref(prm),
                                             _stream_ptr(stream), ctypes.byref(c), ctypes.byref(est)))
    return c.as_dict(), est.value


def tc_estimate_adaptive(g, p0, tol, seed0=0, num_seeds=8, num_groups=4, max_stages=32, heavy=(1, 1),
                         tuned=False, stream=None):
    """Stages of the adaptive keep probability (list of dicts p, estimate,
    m_sum; the last one is the answer) and the section 3.3 balance point."""
    st = (TcStage * int(max_stages))()
    ns = ctypes.c_int32(0)
    pb = ctypes.c_double(0.0)
    prm = _params(heavy, tuned)
    check(_native.load().tc_estimate_adaptive(g.handle, float(p0), float(tol), int(seed0) & (2 ** 64 - 1),
                                              int(num_seeds), int(num_groups), int(max_stages), ctypes.byref(prm),
                                              _stream_ptr(stream), st, ctypes.byref(ns), ctypes.byref(pb)))
    return [st[i].as_dict() for i in range(ns.value)], pb.value


def tc_triple_estimate(g, p, num_samples, hybrid=False, sample_seed=0, triple_seed=0, stream=None):
    """Triple sampling (Simple or Hybrid) on g or its (p, sample_seed) sample:
    dict(size, weight_sum, closed, m, estimate)."""
    r = TcTripleResult()
    check(_native.load().tc_triple_estimate(g.handle, float(p), int(sample_seed) & (2 ** 64 - 1), 1 if hybrid else 0,
                                            int(num_samples), int(triple_seed) & (2 ** 64 - 1), _stream_ptr(stream),
                                            ctypes.byref(r)))
    return r.as_dict()


def tc_stream_estimate(g, d, num_samples, seed=0, stream=None):
    """Semi-streaming three-pass estimate (section 5.2): dict(draws1,
    candidates, heavy, light_size, size, queries, closed, m, estimate)."""
    r = TcStreamResult()
    check(_native.load().tc_stream_estimate(g.handle, float(d), int(num_samples), int(seed) & (2 ** 64 - 1),
                                            _stream_ptr(stream), ctypes.byref(r)))
    return r.as_dict()


def tc_rp_trace(g, k, seed, stream=None):
    """(q int64[k] numpy array, triangle estimate)."""
    q = np.zeros(k, np.int64)
    est = ctypes.c_double(0.0)
    check(_native.load().tc_rp_trace(g.handle, int(k), int(seed) & (2 ** 64 - 1), _stream_ptr(stream),
                                     q.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(est)))
    return q, est.value


def tc_tune_set(g, p, heavy=(1, 1), small_dmax=128, vmajor_cap=1024, blocks_per_cu=8):
    t = TcTuning(int(heavy[0]), int(heavy[1]), int(small_dmax), int(vmajor_cap), int(blocks_per_cu))
    check(_native.load().tc_tune_set(g.handle, float(p), ctypes.byref(t)))


def tc_tune_get(g, p):
    t = TcTuning()
    check(_native.load().tc_tune_get(g.handle, float(p), ctypes.byref(t)))
    return t.as_dict()


def tc_autotune(g, p, seed=0, search_heavy=True, stream=None):
    t = TcTuning()
    check(_native.load().tc_autotune(g.handle, float(p), int(seed) & (2 ** 64 - 1), 1 if search_heavy else 0,
                                     _stream_ptr(stream), ctypes.byref(t)))
    return t.as_dict()


class profile:
    """Launch timing collected by the library with HIP events on the launch stream."""

    @staticmethod
    def enable(on=True):
        check(_native.load().tc_profile_enable(1 if on else 0))

    @staticmethod
    def select(names=None):
        """Restrict profiling to these kernel names (None: all)."""
        arg = None if not names else ",".join(names).encode()
        check(_native.load().tc_profile_select(arg))

    @staticmethod
    def reset():
        check(_native.load().tc_profile_reset())

    @staticmethod
    def read(kernel):
        ms, cnt = ctypes.c_double(0.0), ctypes.c_int64(0)
        check(_native.load().tc_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value


def _request(req_id, p, seed, arrival_s=0.0, graph=None, n=0, src=None, dst=None):
    r = TcRequest()
    r.id = int(req_id) & (2 ** 64 - 1)
    r.p = float(p)
    r.seed = int(seed) & (2 ** 64 - 1)
    r.arrival_s = float(arrival_s)
    if graph is not None:
        r.graph = graph.handle
    else:
        r.n = int(n)
        r.num_pairs = int(len(src))
        r.src = src.ctypes.data if len(src) else None
        r.dst = dst.ctypes.data if len(dst) else None
    return r


def _host_pairs(src, dst):
    src = np.ascontiguousarray(np.asarray(src), dtype=np.int32)
    dst = np.ascontiguousarray(np.asarray(dst), dtype=np.int32)
    if src.shape != dst.shape or src.ndim != 1:
        raise ValueError("src and dst must be 1-D arrays of equal length")
    return src, dst


def tc_request_bytes(p, graph=None, n=0, src=None, dst=None):
    """Arena bytes a serving request needs (no device work)."""
    if graph is None:
        src, dst = _host_pairs(src, dst)
    r = _request(0, p, 0, 0.0, graph, n, src, dst)
    out = ctypes.c_int64(0)
    check(_native.load().tc_request_bytes(ctypes.byref(r), ctypes.byref(out)))
    return out.value


class Server:
    """Serving engine (``tc_server_*``): a device arena of ``budget_bytes``,
    ``lanes`` concurrent requests, and requests of at most ``fuse_max_pairs``
    pairs fused with the small ones queued behind them (0: never).  Host arrays and graphs of submitted
    requests are kept referenced here until their results are polled."""

    def __init__(self, budget_bytes, lanes=4, fuse_max_pairs=0):
        cfg = TcServerConfig(int(budget_bytes), int(lanes), int(fuse_max_pairs))
        h = ctypes.c_void_p(0)
        check(_native.load().tc_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._held = {}

    def clock(self):
        t = ctypes.c_double(0.0)
        check(_native.load().tc_server_clock(self._h, ctypes.byref(t)))
        return t.value

    def submit(self, req_id, p, seed, arrival_s=0.0, graph=None, n=0, src=None, dst=None):
        """Queue a request: a resident ``graph``, or host pairs (``n``, ``src``, ``dst``)."""
        if graph is None:
            src, dst = _host_pairs(src, dst)
        if req_id in self._held:
            raise ValueError("request id %r is already in flight" % (req_id,))
        r = _request(req_id, p, seed, arrival_s, graph, n, src, dst)
        check(_native.load().tc_server_submit(self._h, ctypes.byref(r)))
        self._held[req_id] = (graph, src, dst)

    def poll(self, cap=64, timeout_s=-1.0):
        """Finished results (dicts), waiting up to ``timeout_s`` for the first."""
        buf = (TcResult * max(1, int(cap)))()
        got = ctypes.c_int32(0)
        check(_native.load().tc_server_poll(self._h, buf, int(cap), float(timeout_s), ctypes.byref(got)))
        out = []
        for i in range(got.value):
            d = buf[i].as_dict()
            self._held.pop(d["id"], None)
            out.append(d)
        return out

    def drain(self):
        """Every outstanding result."""
        out = []
        while self._held:
            part = self.poll(256, -1.0)
            if not part:
                break
            out.extend(part)
        return out

    def stats(self):
        st = TcServerInfo()
        check(_native.load().tc_server_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if self._h and self._h.value:
            _native.load().tc_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)
            self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
