"""ctypes binding of libslim.so (include/slim.h).

Argument marshalling only: every step of Triangle p-1-Reduction and edge
sampling runs in the library's HIP kernels.  PyTorch provides device memory
(tensors) and the stream.  There is no CPU fallback: if libslim.so is not
built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# SLIM_LIBRARY may name another build of the same library (e.g. a variant
# compiled with different launch constants); the default is the in-tree one.
LIB_PATH = os.environ.get("SLIM_LIBRARY") or os.path.join(_HERE, "libslim.so")

OK, EINVAL, ENOMEM, EBUDGET, EDEVICE, EAGAIN = 0, -1, -2, -3, -4, -5
VALIDATE = 1
OP_TR, OP_ES, OP_TR2, OP_MCTR, OP_SPECTRAL, OP_EOTR = 1, 2, 3, 4, 5, 6
STAT_KEYS = ("n", "m_in", "triangles", "selected", "deleted", "m_out")
NOALLOC_WS_BYTES = 512 << 20  # the fixed workspace of slim_triangle_reduce_noalloc

# Exported symbols of libslim.so, in include/slim.h order.
SYMBOLS = ("slim_last_error", "slim_strerror", "slim_version", "slim_load_csr",
           "slim_graph_free", "slim_workspace_size", "slim_triangle_reduce",
           "slim_triangle_reduce_noalloc", "slim_edge_sample",
           "slim_compress", "slim_spectral_sparsify", "slim_batch_create", "slim_batch_workspace_size", "slim_batch_run", "slim_batch_set",
           "slim_batch_get", "slim_batch_tune", "slim_batch_stats", "slim_batch_free",
           "slim_serve_create", "slim_serve_submit", "slim_serve_poll", "slim_serve_wait",
           "slim_serve_next", "slim_serve_cancel", "slim_serve_copy", "slim_result_release", "slim_serve_stats",
           "slim_serve_reset_stats", "slim_serve_destroy",
           "slim_tune_set", "slim_tune_get", "slim_profile_enable", "slim_profile_read",
           "slim_degree_kl_workspace", "slim_degree_kl")


class Phase(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("ms", ctypes.c_float)]


class JobParams(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("pad", ctypes.c_int32), ("p", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class Out(ctypes.Structure):
    _fields_ = [("row_off", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("stats", ctypes.c_void_p), ("weight", ctypes.c_void_p)]


class ServeCfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_uint32),
                ("n_streams", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


class Job(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("pad", ctypes.c_int32), ("p", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("row_off", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("nnz", ctypes.c_uint64), ("where", ctypes.c_uint32),
                ("pad2", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in STAT_KEYS]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("pad", ctypes.c_int32), ("row_off", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("n", ctypes.c_uint64), ("stats", Stats),
                ("queue_ms", ctypes.c_double), ("latency_ms", ctypes.c_double)]


SERVE_STAT_KEYS = ("submitted", "completed", "failed", "cancelled", "queued", "running", "batches",
                   "mean_batch_jobs", "p50_ms", "p99_ms", "mean_ms", "max_ms", "jobs_per_s",
                   "edges_per_s", "hbm_in_use", "hbm_peak", "hbm_budget")


class ServeStats(ctypes.Structure):
    _fields_ = ([(k, ctypes.c_uint64) for k in SERVE_STAT_KEYS[:7]]
                + [(k, ctypes.c_double) for k in SERVE_STAT_KEYS[7:14]]
                + [(k, ctypes.c_uint64) for k in SERVE_STAT_KEYS[14:]])


HOST, DEVICE = 0, 1


class SlimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} ({code})")
        self.code = code


def _bind(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, u64, u32, dbl, i32 = (ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double,
                              ctypes.c_int)
    lib.slim_last_error.restype = ctypes.c_char_p
    lib.slim_last_error.argtypes = []
    lib.slim_strerror.restype = ctypes.c_char_p
    lib.slim_strerror.argtypes = [i32]
    lib.slim_version.restype = i32
    lib.slim_version.argtypes = []
    lib.slim_load_csr.restype = i32
    lib.slim_load_csr.argtypes = [vp, vp, u64, u64, u32, vp, ctypes.POINTER(vp)]
    lib.slim_graph_free.restype = None
    lib.slim_graph_free.argtypes = [vp]
    lib.slim_workspace_size.restype = i32
    lib.slim_workspace_size.argtypes = [vp, i32, ctypes.POINTER(u64)]
    for fn in (lib.slim_triangle_reduce, lib.slim_edge_sample):
        fn.restype = i32
        fn.argtypes = [vp, dbl, u64, vp, u64, vp, vp, vp, vp]
    lib.slim_triangle_reduce_noalloc.restype = i32
    lib.slim_triangle_reduce_noalloc.argtypes = [vp, dbl, u64, vp, vp, vp, vp]
    lib.slim_compress.restype = i32
    lib.slim_compress.argtypes = [vp, i32, dbl, u64, vp, u64, vp, vp, vp, vp]
    lib.slim_spectral_sparsify.restype = i32
    lib.slim_spectral_sparsify.argtypes = [vp, dbl, u64, vp, u64, vp, vp, vp, vp, vp]
    lib.slim_batch_create.restype = i32
    lib.slim_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(JobParams), u32,
                                      ctypes.POINTER(vp)]
    lib.slim_batch_workspace_size.restype = i32
    lib.slim_batch_workspace_size.argtypes = [vp, ctypes.POINTER(u64)]
    lib.slim_batch_run.restype = i32
    lib.slim_batch_run.argtypes = [vp, vp, u64, ctypes.POINTER(Out), vp]
    lib.slim_batch_set.restype = i32
    lib.slim_batch_set.argtypes = [vp, ctypes.c_char_p, ctypes.c_int64]
    lib.slim_batch_get.restype = i32
    lib.slim_batch_get.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)]
    lib.slim_batch_tune.restype = i32
    lib.slim_batch_tune.argtypes = [vp, vp, u64, ctypes.POINTER(Out), ctypes.c_char_p, vp]
    lib.slim_batch_stats.restype = i32
    lib.slim_batch_stats.argtypes = [vp, vp]
    lib.slim_batch_free.restype = None
    lib.slim_batch_free.argtypes = [vp]
    lib.slim_serve_create.restype = i32
    lib.slim_serve_create.argtypes = [ctypes.POINTER(ServeCfg), ctypes.POINTER(vp)]
    lib.slim_serve_submit.restype = i32
    lib.slim_serve_submit.argtypes = [vp, ctypes.POINTER(Job), ctypes.POINTER(u64)]
    for fn in (lib.slim_serve_poll, lib.slim_serve_wait):
        fn.restype = i32
        fn.argtypes = [vp, u64, ctypes.POINTER(Result)]
    lib.slim_serve_next.restype = i32
    lib.slim_serve_next.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(u64), ctypes.POINTER(Result)]
    lib.slim_serve_cancel.restype = i32
    lib.slim_serve_cancel.argtypes = [vp, u64]
    lib.slim_serve_copy.restype = i32
    lib.slim_serve_copy.argtypes = [vp, u64, vp, vp]
    lib.slim_result_release.restype = i32
    lib.slim_result_release.argtypes = [vp, u64]
    lib.slim_serve_stats.restype = i32
    lib.slim_serve_stats.argtypes = [vp, ctypes.POINTER(ServeStats)]
    lib.slim_serve_reset_stats.restype = i32
    lib.slim_serve_reset_stats.argtypes = [vp]
    lib.slim_serve_destroy.restype = None
    lib.slim_serve_destroy.argtypes = [vp]
    lib.slim_tune_set.restype = i32
    lib.slim_tune_set.argtypes = [ctypes.c_char_p, ctypes.c_int64]
    lib.slim_tune_get.restype = i32
    lib.slim_tune_get.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)]
    lib.slim_profile_enable.restype = i32
    lib.slim_profile_enable.argtypes = [i32]
    lib.slim_profile_read.restype = i32
    lib.slim_profile_read.argtypes = [ctypes.POINTER(Phase), i32, ctypes.POINTER(i32)]
    lib.slim_degree_kl_workspace.restype = i32
    lib.slim_degree_kl_workspace.argtypes = [u64, ctypes.POINTER(u64)]
    lib.slim_degree_kl.restype = i32
    lib.slim_degree_kl.argtypes = [vp, vp, u64, vp, u64, vp, vp]
    return lib


_lib = _bind()


def _check(rc: int):
    if rc != OK:
        raise SlimError(rc, _lib.slim_last_error().decode())


def _stream_handle(stream, device) -> int:
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return int(stream.cuda_stream)


def version() -> int:
    return int(_lib.slim_version())


def tune_set(key: str, value: int):
    """Set a scheduling knob (never changes results)."""
    _check(_lib.slim_tune_set(key.encode(), int(value)))


def tune_get(key: str) -> int:
    v = ctypes.c_int64(0)
    _check(_lib.slim_tune_get(key.encode(), ctypes.byref(v)))
    return int(v.value)


def profile_enable(on: bool = True):
    """Bracket each phase of the following compute calls with HIP events."""
    _check(_lib.slim_profile_enable(1 if on else 0))


def profile_read() -> list[tuple[str, float]]:
    """(phase, ms) of the most recent compute call (waits for its events)."""
    arr = (Phase * 32)()
    cnt = ctypes.c_int(0)
    _check(_lib.slim_profile_read(arr, 32, ctypes.byref(cnt)))
    return [(arr[i].name.decode(), float(arr[i].ms)) for i in range(min(cnt.value, 32))]


class Graph:
    """A device-resident CSR wrapped in a library handle.

    ``row_off``: int64 tensor [n+1]; ``col``: int32/uint32 tensor [nnz] holding
    uint32 vertex ids.  The tensors are kept alive by this object.
    """

    def __init__(self, row_off: torch.Tensor, col: torch.Tensor, validate: bool = False,
                 stream=None):
        if row_off.dtype != torch.int64 or not row_off.is_cuda or not row_off.is_contiguous():
            raise ValueError("row_off must be a contiguous int64 CUDA tensor")
        if col.element_size() != 4 or not col.is_cuda or not col.is_contiguous():
            raise ValueError("col must be a contiguous 32-bit CUDA tensor")
        self.row_off, self.col = row_off, col
        self.device = row_off.device
        self.n = int(row_off.numel() - 1)
        self.nnz = int(col.numel())
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = _lib.slim_load_csr(row_off.data_ptr(), col.data_ptr() if self.nnz else None,
                                    self.n, self.nnz, VALIDATE if validate else 0,
                                    _stream_handle(stream, self.device), ctypes.byref(h))
        _check(rc)
        self._h = h

    @classmethod
    def from_numpy(cls, row_off: np.ndarray, col: np.ndarray, device="cuda:0",
                   validate: bool = False) -> "Graph":
        ro = torch.from_numpy(np.ascontiguousarray(row_off, dtype=np.int64)).to(device)
        c = np.ascontiguousarray(col, dtype=np.uint32).view(np.int32)
        ct = torch.from_numpy(c).to(device) if c.size else torch.zeros(1, dtype=torch.int32,
                                                                     device=device)[:0]
        return cls(ro, ct, validate=validate)

    @classmethod
    def from_csr(cls, g, device="cuda:0", validate: bool = False) -> "Graph":
        return cls.from_numpy(g.row_off, g.col, device=device, validate=validate)

    @property
    def m(self) -> int:
        return self.nnz // 2

    def workspace_size(self, op: int) -> int:
        b = ctypes.c_uint64(0)
        _check(_lib.slim_workspace_size(self._h, op, ctypes.byref(b)))
        return int(b.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib.slim_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Buffers:
    """Workspace and output tensors for one graph and one operation, reusable
    across calls (the library itself allocates nothing)."""

    def __init__(self, g: Graph, op: int):
        self.g, self.op = g, op
        dev = g.device
        self.ws_bytes = g.workspace_size(op)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)
        self.out_row_off = torch.empty(g.n + 1, dtype=torch.int64, device=dev)
        self.out_col = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=dev)
        self.stats = torch.zeros(len(STAT_KEYS), dtype=torch.int64, device=dev)
        self.out_w = (torch.empty(max(g.nnz, 1), dtype=torch.float32, device=dev)
                      if op == OP_SPECTRAL else None)


def _run(fn, g: Graph, p: float, seed: int, bufs: Buffers | None, stream):
    if bufs is None:
        bufs = Buffers(g, OP_TR if fn is _lib.slim_triangle_reduce else OP_ES)
    with torch.cuda.device(g.device):
        rc = fn(g._h, float(p), int(seed) & (2**64 - 1), bufs.ws.data_ptr(), bufs.ws_bytes,
                bufs.out_row_off.data_ptr(), bufs.out_col.data_ptr(), bufs.stats.data_ptr(),
                _stream_handle(stream, g.device))
    _check(rc)
    return bufs


def triangle_reduce(g: Graph, p: float, seed: int, bufs: Buffers | None = None, stream=None):
    """Enqueue Triangle p-1-Reduction; returns the Buffers holding the output
    CSR (out_row_off, out_col) and stats (valid after stream sync)."""
    return _run(_lib.slim_triangle_reduce, g, p, seed, bufs, stream)


def edge_sample(g: Graph, p: float, seed: int, bufs: Buffers | None = None, stream=None):
    """Enqueue uniform edge sampling (p = deletion probability)."""
    return _run(_lib.slim_edge_sample, g, p, seed, bufs, stream)


def compress(g: Graph, op: int, p: float, seed: int, bufs: Buffers | None = None, stream=None):
    """Enqueue any operation by op code (OP_TR, OP_ES, OP_TR2, OP_MCTR, OP_SPECTRAL,
    OP_EOTR).  OP_EOTR returns once its output is complete (it waits for the
    stream)."""
    if bufs is None:
        bufs = Buffers(g, op)
    with torch.cuda.device(g.device):
        rc = _lib.slim_compress(g._h, int(op), float(p), int(seed) & (2**64 - 1), bufs.ws.data_ptr(),
                                bufs.ws_bytes, bufs.out_row_off.data_ptr(), bufs.out_col.data_ptr(),
                                bufs.stats.data_ptr(), _stream_handle(stream, g.device))
    _check(rc)
    return bufs


def spectral_sparsify(g: Graph, upsilon: float, seed: int, bufs: Buffers | None = None,
                      stream=None):
    """Enqueue spectral sparsification; the weights land in bufs.out_w."""
    if bufs is None:
        bufs = Buffers(g, OP_SPECTRAL)
    with torch.cuda.device(g.device):
        rc = _lib.slim_spectral_sparsify(
            g._h, float(upsilon), int(seed) & (2**64 - 1), bufs.ws.data_ptr(), bufs.ws_bytes,
            bufs.out_row_off.data_ptr(), bufs.out_col.data_ptr(),
            bufs.out_w.data_ptr() if bufs.out_w is not None else None, bufs.stats.data_ptr(),
            _stream_handle(stream, g.device))
    _check(rc)
    return bufs


def degree_kl(row_off_p, row_off_q, out=None, ws=None, stream=None):
    """Enqueue the Kullback-Leibler divergence (bits) of the degree
    distribution of CSR offsets ``row_off_q`` from that of ``row_off_p``
    (device int64 tensors of n+1 entries).  Returns the device float64
    tensor of one element that receives it."""
    n = row_off_p.numel() - 1
    if row_off_q.numel() != n + 1:
        raise ValueError("both graphs must have the same vertex count")
    dev = row_off_p.device
    need = ctypes.c_uint64(0)
    _check(_lib.slim_degree_kl_workspace(n, ctypes.byref(need)))
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(max(int(need.value), 1), dtype=torch.uint8, device=dev)
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=dev)
    with torch.cuda.device(dev):
        rc = _lib.slim_degree_kl(row_off_p.data_ptr(), row_off_q.data_ptr(), n, ws.data_ptr(),
                                 ws.numel(), out.data_ptr(), _stream_handle(stream, dev))
    _check(rc)
    return out


def weights_numpy(bufs: Buffers):
    """Synchronise and copy the output weights of a spectral sparsification."""
    torch.cuda.synchronize(bufs.g.device)
    k = int(bufs.out_row_off[-1].item())
    return bufs.out_w[:k].cpu().numpy()


def result_numpy(bufs: Buffers):
    """Synchronise and copy a result to host: (row_off, col, stats dict)."""
    torch.cuda.synchronize(bufs.g.device)
    ro = bufs.out_row_off.cpu().numpy()
    nnz_out = int(ro[-1])
    col = bufs.out_col[:nnz_out].cpu().numpy().view(np.uint32)
    st = dict(zip(STAT_KEYS, (int(x) for x in bufs.stats.cpu().numpy())))
    return ro, col, st


class Batch:
    """Many (graph, op, p, seed) jobs run as one graph set (slim_batch_*).

    ``jobs`` holds one ``(op, p, seed)`` per graph.  Output tensors for all
    graphs are allocated here as three flat tensors sliced per graph
    (``row_off``/``col``/``stats`` views), plus the workspace.
    """

    def __init__(self, graphs: list[Graph], jobs):
        if len(graphs) != len(jobs) or not graphs:
            raise ValueError("one job per graph, at least one graph")
        self.graphs = list(graphs)
        self.device = graphs[0].device
        hs = (ctypes.c_void_p * len(graphs))(*[g._h.value for g in graphs])
        js = (JobParams * len(jobs))(*[JobParams(int(op), 0, float(p), int(seed) & (2**64 - 1))
                                       for op, p, seed in jobs])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.slim_batch_create(hs, js, len(graphs), ctypes.byref(h)))
        self._h = h
        b = ctypes.c_uint64(0)
        _check(_lib.slim_batch_workspace_size(h, ctypes.byref(b)))
        self.ws_bytes = int(b.value)
        dev = self.device
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)
        ns = np.array([g.n for g in graphs], dtype=np.int64)
        nnzs = np.array([g.nnz for g in graphs], dtype=np.int64)
        self.ro_base = np.concatenate([[0], np.cumsum(ns + 1)])
        self.col_base = np.concatenate([[0], np.cumsum(nnzs)])
        self.row_off_all = torch.empty(int(self.ro_base[-1]), dtype=torch.int64, device=dev)
        self.col_all = torch.empty(max(int(self.col_base[-1]), 1), dtype=torch.int32, device=dev)
        self.stats_all = torch.zeros((len(graphs), len(STAT_KEYS)), dtype=torch.int64, device=dev)
        self.w_all = (torch.empty(max(int(self.col_base[-1]), 1), dtype=torch.float32, device=dev)
                      if any(int(op) == OP_SPECTRAL for op, _, _ in jobs) else None)
        rp, cp, sp = (self.row_off_all.data_ptr(), self.col_all.data_ptr(),
                      self.stats_all.data_ptr())
        wp = self.w_all.data_ptr() if self.w_all is not None else None
        self._outs = (Out * len(graphs))(*[
            Out(rp + 8 * int(self.ro_base[i]), cp + 4 * int(self.col_base[i]) if nnzs[i] else None,
                sp + 8 * len(STAT_KEYS) * i,
                wp + 4 * int(self.col_base[i]) if (wp and nnzs[i]) else None)
            for i in range(len(graphs))])

    def __len__(self):
        return len(self.graphs)

    def set(self, key: str, value: int):
        _check(_lib.slim_batch_set(self._h, key.encode(), int(value)))

    def get(self, key: str) -> int:
        v = ctypes.c_int64(0)
        _check(_lib.slim_batch_get(self._h, key.encode(), ctypes.byref(v)))
        return int(v.value)

    def run(self, stream=None):
        """Enqueue every job (results valid after stream sync)."""
        with torch.cuda.device(self.device):
            _check(_lib.slim_batch_run(self._h, self.ws.data_ptr(), self.ws_bytes, self._outs,
                                       _stream_handle(stream, self.device)))

    def tune(self, cache_path: str | None = None, stream=None):
        """Autotune the batch's knobs (runs it several times; synchronises)."""
        with torch.cuda.device(self.device):
            _check(_lib.slim_batch_tune(self._h, self.ws.data_ptr(), self.ws_bytes, self._outs,
                                        cache_path.encode() if cache_path else None,
                                        _stream_handle(stream, self.device)))

    def stats(self) -> list[dict]:
        """Per-graph counters of the most recent run (slim_batch_stats)."""
        out = np.zeros((len(self.graphs), len(STAT_KEYS)), dtype=np.uint64)
        _check(_lib.slim_batch_stats(self._h, out.ctypes.data))
        return [dict(zip(STAT_KEYS, (int(x) for x in row))) for row in out]

    def result_numpy(self, i: int):
        """Synchronise and copy graph i's result: (row_off, col, stats dict)."""
        torch.cuda.synchronize(self.device)
        a, b = int(self.ro_base[i]), int(self.ro_base[i + 1])
        ro = self.row_off_all[a:b].cpu().numpy()
        c0 = int(self.col_base[i])
        col = self.col_all[c0:c0 + int(ro[-1])].cpu().numpy().view(np.uint32)
        st = dict(zip(STAT_KEYS, (int(x) for x in self.stats_all[i].cpu().numpy())))
        return ro, col, st

    def close(self):
        if getattr(self, "_h", None):
            torch.cuda.synchronize(self.device)
            _lib.slim_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """In-process compression service (slim_serve_*): HBM-budget admission
    and continuously formed batches on ``n_streams`` worker streams."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 0, n_streams: int = 2,
                 max_batch: int = 0, device="cuda:0"):
        self.device = torch.device(device)
        cfg = ServeCfg(int(hbm_budget_bytes), int(max_slots), int(n_streams), int(max_batch), 0)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.slim_serve_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._keep = {}  # ticket -> arrays the job borrows

    def submit(self, graph, op: int, p: float, seed: int) -> int:
        """Queue a job on a host CSR (graphgen.CSR / numpy arrays, copied to the
        device by the server) or a device-resident Graph (borrowed)."""
        if isinstance(graph, Graph):
            ro, col, n, nnz, where = (graph.row_off.data_ptr(),
                                      graph.col.data_ptr() if graph.nnz else None,
                                      graph.n, graph.nnz, DEVICE)
            keep = graph
        else:
            ro_np = np.ascontiguousarray(graph.row_off, dtype=np.int64)
            col_np = np.ascontiguousarray(graph.col, dtype=np.uint32)
            ro, col = ro_np.ctypes.data, (col_np.ctypes.data if col_np.size else None)
            n, nnz, where = ro_np.size - 1, col_np.size, HOST
            keep = (ro_np, col_np)
        job = Job(int(op), 0, float(p), int(seed) & (2**64 - 1), ro, col, n, nnz, where, 0)
        t = ctypes.c_uint64(0)
        _check(_lib.slim_serve_submit(self._h, ctypes.byref(job), ctypes.byref(t)))
        self._keep[int(t.value)] = keep
        return int(t.value)

    def poll(self, ticket: int):
        r = Result()
        rc = _lib.slim_serve_poll(self._h, ticket, ctypes.byref(r))
        if rc == EAGAIN:
            return None
        _check(rc)
        return r

    def wait(self, ticket: int) -> Result:
        r = Result()
        _check(_lib.slim_serve_wait(self._h, ticket, ctypes.byref(r)))
        return r

    def next(self, timeout_ms: int = -1):
        """(ticket, Result) of the next job to finish, in completion order;
        None if none finished within timeout_ms (-1: wait without limit)."""
        r = Result()
        t = ctypes.c_uint64(0)
        rc = _lib.slim_serve_next(self._h, int(timeout_ms), ctypes.byref(t), ctypes.byref(r))
        if rc == EAGAIN:
            return None
        _check(rc)
        return int(t.value), r

    def cancel(self, ticket: int) -> bool:
        rc = _lib.slim_serve_cancel(self._h, ticket)
        if rc == EAGAIN:
            return False
        _check(rc)
        self._keep.pop(ticket, None)
        return True

    def result_numpy(self, ticket: int):
        """Wait for a job and copy its output: (row_off, col, stats dict)."""
        r = self.wait(ticket)
        if r.status != OK:
            raise SlimError(r.status, f"job {ticket} failed")
        st = {k: int(getattr(r.stats, k)) for k in STAT_KEYS}
        ro = np.empty(r.n + 1, dtype=np.int64)
        col = np.empty(max(2 * st["m_out"], 1), dtype=np.uint32)
        _check(_lib.slim_serve_copy(self._h, ticket, ro.ctypes.data, col.ctypes.data))
        return ro, col[:2 * st["m_out"]], st

    def release(self, ticket: int):
        _check(_lib.slim_result_release(self._h, ticket))
        self._keep.pop(ticket, None)

    def stats(self) -> dict:
        o = ServeStats()
        _check(_lib.slim_serve_stats(self._h, ctypes.byref(o)))
        return {k: getattr(o, k) for k in SERVE_STAT_KEYS}

    def reset_stats(self):
        _check(_lib.slim_serve_reset_stats(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.slim_serve_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
