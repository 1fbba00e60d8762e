"""ctypes declarations of libtc.so (the C ABI in include/tc.h).

The library is built in-tree by ``paper_1011_0468_amd.build``; importing this
module fails loudly if it is missing.  There is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libtc.so")
TORCH_ALLOC_PATH = os.path.join(HERE, "libtc_torch_alloc.so")

TC_OK, TC_ERR_INVALID, TC_ERR_OOM, TC_ERR_DEVICE, TC_ERR_OVERFLOW, TC_ERR_BUDGET = range(6)
STATUS_NAMES = {0: "TC_OK", 1: "TC_ERR_INVALID", 2: "TC_ERR_OOM", 3: "TC_ERR_DEVICE",
                4: "TC_ERR_OVERFLOW", 5: "TC_ERR_BUDGET"}


class TcParams(ctypes.Structure):
    _fields_ = [("heavy_num", ctypes.c_int32), ("heavy_den", ctypes.c_int32), ("use_tuned", ctypes.c_int32)]


class TcCounts(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("triangles", "light", "heavy", "m", "n_heavy", "light_sources", "light_out_edges",
                 "wedges", "gather", "probes", "items_small", "items_large", "model_bytes_small",
                 "model_bytes_large")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class TcTuning(ctypes.Structure):
    _fields_ = [("heavy_num", ctypes.c_int32), ("heavy_den", ctypes.c_int32), ("small_dmax", ctypes.c_int32),
                ("vmajor_cap", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class TcStage(ctypes.Structure):
    _fields_ = [("p", ctypes.c_double), ("estimate", ctypes.c_double), ("m_sum", ctypes.c_int64)]

    def as_dict(self):
        return {"p": self.p, "estimate": self.estimate, "m_sum": int(self.m_sum)}


class TcTripleResult(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int64), ("weight_sum", ctypes.c_int64), ("closed", ctypes.c_int64),
                ("m", ctypes.c_int64), ("estimate", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class TcStreamResult(ctypes.Structure):
    _fields_ = [("draws1", ctypes.c_int64), ("candidates", ctypes.c_int64), ("heavy", ctypes.c_int64),
                ("light_size", ctypes.c_int64), ("size", ctypes.c_int64), ("queries", ctypes.c_int64),
                ("closed", ctypes.c_int64), ("m", ctypes.c_int64), ("estimate", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class TcServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("lanes", ctypes.c_int32), ("fuse_max_pairs", ctypes.c_int32)]


class TcRequest(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("graph", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("num_pairs", ctypes.c_int64), ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p),
                ("p", ctypes.c_double), ("seed", ctypes.c_uint64), ("arrival_s", ctypes.c_double)]


class TcResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("lane", ctypes.c_int32),
                ("counts", TcCounts), ("estimate", ctypes.c_double), ("arrival_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("done_s", ctypes.c_double), ("reserved_bytes", ctypes.c_int64),
                ("peak_bytes", ctypes.c_int64), ("spilled_bytes", ctypes.c_int64), ("message", ctypes.c_char * 96)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_ if name not in ("counts", "message")}
        d["counts"] = self.counts.as_dict()
        d["message"] = self.message.decode(errors="replace")
        return d


class TcServerInfo(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("submitted", "completed", "rejected", "queued", "running", "arena_bytes", "arena_used",
                 "arena_peak", "spilled_bytes")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class TcError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

# every symbol declared in include/tc.h
EXPORTS = ["tc_set_allocator", "tc_build_csr", "tc_graph_info", "tc_graph_csr", "tc_graph_read", "tc_sample",
           "tc_count_exact", "tc_estimate", "tc_estimate_noalloc", "tc_estimate_adaptive", "tc_triple_estimate", "tc_stream_estimate", "tc_rp_trace", "tc_tune_set", "tc_tune_get", "tc_autotune",
           "tc_graph_free", "tc_last_error",
           "tc_request_bytes", "tc_server_create", "tc_server_clock", "tc_server_submit", "tc_server_poll",
           "tc_server_stats", "tc_server_destroy",
           "tc_profile_enable", "tc_profile_select", "tc_profile_reset", "tc_profile_read"]

_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO_PATH):
        raise RuntimeError("libtc.so is not built (run __graft_entry__.build()); "
                           "there is no fallback path")
    L = ctypes.CDLL(SO_PATH)
    vp, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    P = ctypes.POINTER
    sigs = {
        "tc_set_allocator": [ALLOC_FN, FREE_FN, vp],
        "tc_build_csr": [i64, i64, vp, vp, i32, vp, P(vp)],
        "tc_graph_info": [vp, P(i64), P(i64), P(i32)],
        "tc_graph_csr": [vp, P(vp), P(vp)],
        "tc_graph_read": [vp, vp, vp, vp, i32, vp],
        "tc_sample": [vp, dbl, u64, vp, P(vp)],
        "tc_count_exact": [vp, P(TcParams), vp, P(TcCounts)],
        "tc_estimate": [vp, dbl, P(u64), i32, i32, P(TcParams), vp, P(TcCounts), P(dbl), P(dbl)],
        "tc_estimate_noalloc": [vp, dbl, u64, P(TcParams), vp, P(TcCounts), P(dbl)],
        "tc_estimate_adaptive": [vp, dbl, dbl, u64, i32, i32, i32, P(TcParams), vp, P(TcStage), P(i32), P(dbl)],
        "tc_triple_estimate": [vp, dbl, u64, i32, i64, u64, vp, P(TcTripleResult)],
        "tc_stream_estimate": [vp, dbl, i64, u64, vp, P(TcStreamResult)],
        "tc_rp_trace": [vp, i32, u64, vp, P(i64), P(dbl)],
        "tc_tune_set": [vp, dbl, P(TcTuning)],
        "tc_tune_get": [vp, dbl, P(TcTuning)],
        "tc_autotune": [vp, dbl, u64, i32, vp, P(TcTuning)],
        "tc_request_bytes": [P(TcRequest), P(i64)],
        "tc_server_create": [P(TcServerConfig), P(vp)],
        "tc_server_clock": [vp, P(dbl)],
        "tc_server_submit": [vp, P(TcRequest)],
        "tc_server_poll": [vp, P(TcResult), i32, dbl, P(i32)],
        "tc_server_stats": [vp, P(TcServerInfo)],
        "tc_profile_enable": [i32],
        "tc_profile_reset": [],
        "tc_profile_select": [ctypes.c_char_p],
        "tc_profile_read": [ctypes.c_char_p, P(dbl), P(i64)],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.tc_graph_free.argtypes = [vp]
    L.tc_graph_free.restype = None
    L.tc_server_destroy.argtypes = [vp]
    L.tc_server_destroy.restype = None
    L.tc_last_error.argtypes = []
    L.tc_last_error.restype = ctypes.c_char_p
    _install_torch_allocator(L)
    _lib = L
    return L


_torch_alloc = None  # the shim and its two function pointers, kept alive while installed


def _install_torch_allocator(L):
    """Route the library's device allocations through PyTorch's caching
    allocator (tc_set_allocator with the C functions of libtc_torch_alloc.so:
    no Python runs per allocation), so that one pool serves the caller's
    tensors and the library's buffers."""
    global _torch_alloc
    if not os.path.exists(TORCH_ALLOC_PATH):
        raise RuntimeError("libtc_torch_alloc.so is not built (run __graft_entry__.build())")
    import torch  # noqa: F401  (loads libc10_hip before the shim)
    A = ctypes.CDLL(TORCH_ALLOC_PATH)
    fa = ALLOC_FN(ctypes.cast(A.tc_torch_alloc, ctypes.c_void_p).value)
    ff = FREE_FN(ctypes.cast(A.tc_torch_free, ctypes.c_void_p).value)
    rc = L.tc_set_allocator(fa, ff, None)
    if rc != 0:
        raise RuntimeError("tc_set_allocator refused the torch allocator (status %d)" % rc)
    _torch_alloc = (A, fa, ff)


def allocator():
    """"torch" while PyTorch's caching allocator serves the library."""
    return "torch" if _torch_alloc is not None else "library"


def check(status):
    if status != TC_OK:
        msg = load().tc_last_error().decode(errors="replace")
        raise TcError(status, msg)
