"""ctypes binding of libskis.so (argument marshalling only).

Every computation runs in the library's HIP kernels; this module passes device pointers of
torch tensors and the current HIP stream.  torch supplies device memory and streams only.
If libskis.so is missing or cannot be loaded, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libskis.so")

SKIS_OK, SKIS_WDEGENERATE, SKIS_EINVAL, SKIS_ENOMEM, SKIS_EHIP = 0, 1, -1, -2, -3

EXPORTED = ("skis_default_options", "skis_preprocess", "skis_build_sketch", "skis_sketch_info",
            "skis_estimate", "skis_greedy_max_cover", "skis_sketch_export", "skis_inverse_export",
            "skis_node_q", "skis_sketch_free", "skis_last_error", "skis_server_default_options",
            "skis_server_create", "skis_server_submit", "skis_server_wait", "skis_server_replay",
            "skis_server_get_stats", "skis_server_destroy", "skis_probe_random_read", "skis_set_memory_limits",
            "skis_release_cached_memory", "skis_samples_for_estimate", "skis_estimate_noalloc", "skis_im_dssa",
            "skis_preprocess_lt")


class SkisError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libskis error %d: %s" % (code, msg))
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("form", ctypes.c_uint32), ("slots_per_block", ctypes.c_uint32),
                ("visited_threshold", ctypes.c_uint32), ("big_row", ctypes.c_uint32),
                ("build_inverse_index", ctypes.c_uint32), ("threads_per_block", ctypes.c_uint32),
                ("max_device_bytes", ctypes.c_uint64), ("staging_entries", ctypes.c_uint64),
                ("chunk_samples", ctypes.c_uint64), ("quads_per_lane", ctypes.c_uint32),
                ("entry_budget", ctypes.c_uint64), ("ris_mode", ctypes.c_uint32), ("model", ctypes.c_uint32)]


class DssaInfo(ctypes.Structure):
    _fields_ = [("T", ctypes.c_uint64), ("iterations", ctypes.c_uint32), ("stopped", ctypes.c_uint32),
                ("cov_select", ctypes.c_uint64), ("cov_check", ctypes.c_uint64), ("est_select", ctypes.c_double),
                ("est_check", ctypes.c_double), ("eps1", ctypes.c_double), ("eps2", ctypes.c_double),
                ("eps3", ctypes.c_double), ("eps_t", ctypes.c_double), ("Lambda", ctypes.c_double),
                ("N_max", ctypes.c_double), ("t_max", ctypes.c_double), ("Gamma", ctypes.c_double)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("pipeline_depth", ctypes.c_uint32), ("max_batch_queries", ctypes.c_uint32),
                ("max_batch_entries", ctypes.c_uint32), ("max_large_sets", ctypes.c_uint32),
                ("max_device_bytes", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_uint64), ("queries", ctypes.c_uint64), ("max_batch", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("batch_hist", ctypes.c_uint64 * 16)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32), ("T", ctypes.c_uint64),
                ("entries", ctypes.c_uint64), ("probed_total", ctypes.c_uint64),
                ("deferred", ctypes.c_uint64), ("C", ctypes.c_uint64), ("Gamma", ctypes.c_double),
                ("device_bytes", ctypes.c_uint64), ("ms_preprocess", ctypes.c_double),
                ("ms_roots", ctypes.c_double), ("ms_sample", ctypes.c_double),
                ("ms_compact", ctypes.c_double), ("ms_inverse", ctypes.c_double),
                ("ms_tier0", ctypes.c_double), ("ms_tier1", ctypes.c_double),
                ("ms_tier2", ctypes.c_double), ("ms_tier3", ctypes.c_double),
                ("deferred_global", ctypes.c_uint64), ("deferred_bitmap", ctypes.c_uint64),
                ("plain_levels", ctypes.c_uint32), ("graph_replays", ctypes.c_uint32),
                ("tier_samples", ctypes.c_uint64 * 4), ("tier_entries", ctypes.c_uint64 * 4),
                ("tier_probed", ctypes.c_uint64 * 4), ("tier_swept", ctypes.c_uint64 * 4),
                ("tier_items", ctypes.c_uint64 * 4)]


_lib = None


def lib():
    """Loads libskis.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libskis.so is not built (%s); run python -m paper_1709_03565_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.skis_default_options.argtypes = [ctypes.POINTER(Options)]
        L.skis_default_options.restype = None
        L.skis_preprocess.argtypes = [i32, i64, P, P, P, P, P, P, P, P, P, P, P]
        L.skis_preprocess.restype = ctypes.c_int
        L.skis_preprocess_lt.argtypes = [i32, i64, P, P, P, P, P, P, P, P, P, P, P]
        L.skis_preprocess_lt.restype = ctypes.c_int
        L.skis_build_sketch.argtypes = [i32, i64, P, P, P, u64, u64, ctypes.POINTER(Options), P,
                                        ctypes.POINTER(P)]
        L.skis_build_sketch.restype = ctypes.c_int
        L.skis_sketch_info.argtypes = [P, ctypes.POINTER(Info)]
        L.skis_sketch_info.restype = ctypes.c_int
        L.skis_estimate.argtypes = [P, i32, P, P, P, P, P]
        L.skis_estimate.restype = ctypes.c_int
        L.skis_estimate_noalloc.argtypes = [P, i32, P, P, P, P, P]
        L.skis_estimate_noalloc.restype = ctypes.c_int
        L.skis_greedy_max_cover.argtypes = [P, i32, P, P, P, P, P]
        L.skis_greedy_max_cover.restype = ctypes.c_int
        L.skis_sketch_export.argtypes = [P, P, P, P, P, P]
        L.skis_sketch_export.restype = ctypes.c_int
        L.skis_inverse_export.argtypes = [P, P, P, P]
        L.skis_inverse_export.restype = ctypes.c_int
        L.skis_probe_random_read.argtypes = [P, u64, ctypes.c_uint32, u64, ctypes.c_uint32, P, P]
        L.skis_probe_random_read.restype = ctypes.c_int
        L.skis_node_q.argtypes = [P, P, P]
        L.skis_node_q.restype = ctypes.c_int
        L.skis_sketch_free.argtypes = [P]
        L.skis_sketch_free.restype = None
        L.skis_last_error.argtypes = []
        L.skis_last_error.restype = ctypes.c_char_p
        L.skis_server_default_options.argtypes = [ctypes.POINTER(ServerOptions)]
        L.skis_server_default_options.restype = None
        L.skis_server_create.argtypes = [P, ctypes.POINTER(ServerOptions), ctypes.POINTER(P)]
        L.skis_server_create.restype = ctypes.c_int
        L.skis_server_submit.argtypes = [P, P, i32, ctypes.POINTER(u64)]
        L.skis_server_submit.restype = ctypes.c_int
        L.skis_server_wait.argtypes = [P, u64, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
        L.skis_server_wait.restype = ctypes.c_int
        L.skis_server_replay.argtypes = [P, i32, P, P, P, P, P, P]
        L.skis_server_replay.restype = ctypes.c_int
        L.skis_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
        L.skis_server_get_stats.restype = ctypes.c_int
        L.skis_server_destroy.argtypes = [P]
        L.skis_server_destroy.restype = None
        L.skis_set_memory_limits.argtypes = [u64, u64]
        L.skis_set_memory_limits.restype = ctypes.c_int
        L.skis_release_cached_memory.argtypes = []
        L.skis_release_cached_memory.restype = ctypes.c_int
        L.skis_samples_for_estimate.argtypes = [i32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, ctypes.POINTER(u64)]
        L.skis_samples_for_estimate.restype = ctypes.c_int
        L.skis_im_dssa.argtypes = [i32, i64, P, P, P, i32, ctypes.c_double, ctypes.c_double, u64,
                                   ctypes.POINTER(Options), P, P, ctypes.POINTER(DssaInfo)]
        L.skis_im_dssa.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(code: int) -> int:
    if code < 0:
        raise SkisError(code, lib().skis_last_error().decode())
    return code


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    return t.to(device="cuda", dtype=dtype).contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def default_options(**kw) -> Options:
    o = Options()
    lib().skis_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def preprocess(row_ptr, col, w, model: int = 0):
    """Rows a1-a3 into new device tensors: dict(P, q, W, thr, alias, C, Gamma, status).  model 1:
    the linear threshold model (skis_preprocess_lt), P holds the running sums S."""
    row_ptr, col, w = _dev(row_ptr, torch.int32), _dev(col, torch.int32), _dev(w, torch.float32)
    n, m = row_ptr.numel() - 1, col.numel()
    P = torch.empty(max(m, 1), dtype=torch.float64, device="cuda")
    q = torch.empty(n, dtype=torch.float64, device="cuda")
    W = torch.empty(n, dtype=torch.int64, device="cuda")
    thr = torch.empty(n, dtype=torch.int64, device="cuda")
    alias = torch.empty(n, dtype=torch.int32, device="cuda")
    C = ctypes.c_uint64()
    G = ctypes.c_double()
    fn = lib().skis_preprocess_lt if model else lib().skis_preprocess
    st = _check(fn(n, m, _ptr(row_ptr), _ptr(col), _ptr(w), _ptr(P), _ptr(q), _ptr(W),
                   _ptr(thr), _ptr(alias), ctypes.byref(C), ctypes.byref(G), _stream()))
    return dict(P=P[:m], q=q, W=W, thr=thr, alias=alias, C=C.value, Gamma=G.value, status=st)


@dataclass
class SketchInfo:
    n: int
    T: int
    entries: int
    probed_total: int
    deferred: int
    C: int
    Gamma: float
    device_bytes: int
    ms_preprocess: float
    ms_roots: float
    ms_sample: float
    ms_compact: float
    ms_inverse: float
    ms_tier0: float
    ms_tier1: float
    ms_tier2: float
    ms_tier3: float
    deferred_global: int
    deferred_bitmap: int
    plain_levels: int
    graph_replays: int
    tier_samples: tuple = (0, 0, 0, 0)
    tier_entries: tuple = (0, 0, 0, 0)
    tier_probed: tuple = (0, 0, 0, 0)
    tier_swept: tuple = (0, 0, 0, 0)
    tier_items: tuple = (0, 0, 0, 0)


class Sketch:
    """A device-resident SKIS sketch (owned by libskis; freed by free() or on GC)."""

    def __init__(self, handle, status):
        self._h = handle
        self.status = status

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def free(self):
        if self._h:
            lib().skis_sketch_free(self._h)
            self._h = None

    def info(self) -> SketchInfo:
        i = Info()
        _check(lib().skis_sketch_info(self._h, ctypes.byref(i)))
        return SketchInfo(i.n, i.T, i.entries, i.probed_total, i.deferred, i.C, i.Gamma, i.device_bytes,
                          i.ms_preprocess, i.ms_roots, i.ms_sample, i.ms_compact, i.ms_inverse,
                          i.ms_tier0, i.ms_tier1, i.ms_tier2, i.ms_tier3, i.deferred_global, i.deferred_bitmap,
                          i.plain_levels, i.graph_replays, tuple(i.tier_samples), tuple(i.tier_entries),
                          tuple(i.tier_probed), tuple(i.tier_swept), tuple(i.tier_items))

    def estimate(self, set_ptr, set_nodes):
        """(cov uint64[Q], est float64[Q]) device tensors for seed sets in CSR form."""
        set_ptr, set_nodes = _dev(set_ptr, torch.int64), _dev(set_nodes, torch.int32)
        Q = set_ptr.numel() - 1
        cov = torch.empty(max(Q, 1), dtype=torch.int64, device="cuda")
        est = torch.empty(max(Q, 1), dtype=torch.float64, device="cuda")
        _check(lib().skis_estimate(self._h, Q, _ptr(set_ptr), _ptr(set_nodes), _ptr(cov), _ptr(est), _stream()))
        return cov[:Q], est[:Q]

    def estimate_noalloc(self, set_ptr, set_nodes):
        """As estimate(), through skis_estimate_noalloc (no device allocation inside the call)."""
        set_ptr, set_nodes = _dev(set_ptr, torch.int64), _dev(set_nodes, torch.int32)
        Q = set_ptr.numel() - 1
        cov = torch.empty(max(Q, 1), dtype=torch.int64, device="cuda")
        est = torch.empty(max(Q, 1), dtype=torch.float64, device="cuda")
        _check(lib().skis_estimate_noalloc(self._h, Q, _ptr(set_ptr), _ptr(set_nodes), _ptr(cov), _ptr(est),
                                           _stream()))
        return cov[:Q], est[:Q]

    def greedy(self, k: int):
        """(seeds int32[k], marginal uint64[k], cov, est) of Alg. 3."""
        seeds = torch.empty(max(k, 1), dtype=torch.int32, device="cuda")
        marg = torch.empty(max(k, 1), dtype=torch.int64, device="cuda")
        cov, est = ctypes.c_uint64(), ctypes.c_double()
        _check(lib().skis_greedy_max_cover(self._h, k, _ptr(seeds), _ptr(marg), ctypes.byref(cov),
                                           ctypes.byref(est), _stream()))
        return seeds[:k], marg[:k], cov.value, est.value

    def export(self):
        """(sample_ptr int64[T+1], nodes int32[entries], roots int32[T], probed uint64[T])."""
        inf = self.info()
        sp = torch.empty(inf.T + 1, dtype=torch.int64, device="cuda")
        nodes = torch.empty(max(inf.entries, 1), dtype=torch.int32, device="cuda")
        roots = torch.empty(max(inf.T, 1), dtype=torch.int32, device="cuda")
        probed = torch.empty(max(inf.T, 1), dtype=torch.int64, device="cuda")
        _check(lib().skis_sketch_export(self._h, _ptr(sp), _ptr(nodes), _ptr(roots), _ptr(probed), _stream()))
        return sp, nodes[:inf.entries], roots[:inf.T], probed[:inf.T]

    def inverse(self):
        inf = self.info()
        node_ptr = torch.empty(inf.n + 1, dtype=torch.int64, device="cuda")
        ns = torch.empty(max(inf.entries, 1), dtype=torch.int32, device="cuda")
        _check(lib().skis_inverse_export(self._h, _ptr(node_ptr), _ptr(ns), _stream()))
        return node_ptr, ns[:inf.entries]

    def q(self):
        inf = self.info()
        q = torch.empty(inf.n, dtype=torch.float64, device="cuda")
        _check(lib().skis_node_q(self._h, _ptr(q), _stream()))
        return q


def im_dssa(row_ptr, col, w, k: int, eps: float, delta: float, seed: int, **kw):
    """D-SSA on SKIS sketches (skis_im_dssa): (seeds int32 numpy [k], info dict, status)."""
    import numpy as np
    row_ptr, col, w = _dev(row_ptr, torch.int32), _dev(col, torch.int32), _dev(w, torch.float32)
    n, m = row_ptr.numel() - 1, col.numel()
    opt = default_options(**kw)
    seeds = np.zeros(max(k, 1), np.int32)
    info = DssaInfo()
    st = _check(lib().skis_im_dssa(n, m, _ptr(row_ptr), _ptr(col), _ptr(w), k, eps, delta, seed, ctypes.byref(opt),
                                   _stream(), seeds.ctypes.data_as(ctypes.c_void_p), ctypes.byref(info)))
    return seeds[:k], {f: getattr(info, f) for f, _ in DssaInfo._fields_}, st


def samples_for_estimate(n: int, Gamma: float, I_lower: float, eps: float, delta: float) -> int:
    """Samples an (eps, delta)-estimate of every set with I(S) >= I_lower needs (Lemma lem:monte)."""
    T = ctypes.c_uint64()
    _check(lib().skis_samples_for_estimate(n, Gamma, I_lower, eps, delta, ctypes.byref(T)))
    return T.value


def set_memory_limits(cache_keep_bytes: int, pool_keep_bytes: int) -> None:
    """Limits on the device memory the library keeps for reuse (idle-block cache, pool)."""
    _check(lib().skis_set_memory_limits(cache_keep_bytes, pool_keep_bytes))


def release_cached_memory() -> None:
    """Gives the library's idle device memory back (after a device synchronisation)."""
    _check(lib().skis_release_cached_memory())


def build_sketch(row_ptr, col, w, num_samples: int, seed: int, options: Options | None = None, **kw) -> Sketch:
    """Builds a sketch of num_samples IIS samples on the current device and stream."""
    row_ptr, col, w = _dev(row_ptr, torch.int32), _dev(col, torch.int32), _dev(w, torch.float32)
    n, m = row_ptr.numel() - 1, col.numel()
    opt = options if options is not None else default_options(**kw)
    h = ctypes.c_void_p()
    st = _check(lib().skis_build_sketch(n, m, _ptr(row_ptr), _ptr(col), _ptr(w), num_samples, seed,
                                        ctypes.byref(opt), _stream(), ctypes.byref(h)))
    return Sketch(h, st)


class Server:
    """Continuous-batching estimate service over a resident sketch (skis_server_*).

    Host-side API: sets are numpy int32 arrays of node ids; results come back in host memory.
    The sketch must stay alive while the server runs."""

    def __init__(self, sketch: Sketch, **kw):
        o = ServerOptions()
        lib().skis_server_default_options(ctypes.byref(o))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        h = ctypes.c_void_p()
        _check(lib().skis_server_create(sketch._h, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._sketch = sketch

    def submit(self, nodes) -> int:
        a = np.ascontiguousarray(nodes, dtype=np.int32)
        t = ctypes.c_uint64()
        _check(lib().skis_server_submit(self._h, a.ctypes.data_as(ctypes.c_void_p), a.size, ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int):
        """(cov, est, latency_us) of a submitted set."""
        c, e, l = ctypes.c_uint64(), ctypes.c_double(), ctypes.c_double()
        _check(lib().skis_server_wait(self._h, ticket, ctypes.byref(c), ctypes.byref(e), ctypes.byref(l)))
        return c.value, e.value, l.value

    def replay(self, set_ptr, set_nodes, arrival_us):
        """Open-loop replay: (cov uint64[Q], est float64[Q], latency_us float64[Q]) numpy arrays."""
        sp = np.ascontiguousarray(set_ptr, dtype=np.int64)
        sn = np.ascontiguousarray(set_nodes, dtype=np.int32)
        at = np.ascontiguousarray(arrival_us, dtype=np.float64)
        Q = sp.size - 1
        cov = np.zeros(max(Q, 1), np.uint64)
        est = np.zeros(max(Q, 1), np.float64)
        lat = np.zeros(max(Q, 1), np.float64)
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(lib().skis_server_replay(self._h, Q, vp(sp), vp(sn) if sn.size else None, vp(at), vp(cov), vp(est),
                                        vp(lat)))
        return cov[:Q], est[:Q], lat[:Q]

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().skis_server_get_stats(self._h, ctypes.byref(st)))
        return {"batches": st.batches, "queries": st.queries, "max_batch": st.max_batch,
                "device_bytes": st.device_bytes, "batch_hist": list(st.batch_hist)}

    def close(self):
        if self._h:
            lib().skis_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def probe_random_read(table: torch.Tensor, row_bytes: int, reads: int, sink: torch.Tensor, seed: int = 1) -> None:
    """Reads `reads` rows of row_bytes bytes at uniformly random positions of the device
    tensor `table` (its bytes split into rows) on torch's current stream; a measurement aid
    for the random-access ceiling, timed by the caller.  sink: one int32 on the device."""
    if not (table.is_cuda and sink.is_cuda and table.is_contiguous()):
        raise ValueError("table and sink must be contiguous device tensors")
    rows = table.numel() * table.element_size() // row_bytes if row_bytes > 0 else 0
    _check(lib().skis_probe_random_read(_ptr(table), rows, row_bytes, reads, seed, _ptr(sink), _stream()))
