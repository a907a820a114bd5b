"""CPU oracle (TEST INFRASTRUCTURE ONLY) -- ctypes front end of liboracle.so.

Plain single-threaded reference for Triangle p-1-Reduction (Slim Graph,
section 4.3), its p-2, Min-Count and Edge-Once variants, uniform edge
sampling (section 4.2.2), spectral sparsification (section 4.2.1) and the
degree-distribution Kullback-Leibler divergence of section 5 (in numpy).  Only tests/,
``__graft_entry__.smoke()`` and bench.py's ``cpu_baseline`` leg may import
this module; the product path never does.  It shares no code with the GPU
path.  The readings of the paper it implements are stated in the header of
``slim_oracle.c``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slim_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

STAT_KEYS = ("n", "m_in", "T", "selected", "deleted", "m_out")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (single-threaded, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", _SRC, "-o", tmp,
                        "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    vp, u64, dbl = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double
    lib.orc_philox4x32_10.argtypes = [vp, vp, vp]
    lib.orc_philox4x32_10.restype = None
    lib.orc_threshold.argtypes = [dbl, ctypes.POINTER(u64)]
    lib.orc_threshold.restype = ctypes.c_int
    lib.orc_validate.argtypes = [u64, vp, vp]
    lib.orc_validate.restype = ctypes.c_int
    lib.orc_list_triangles.argtypes = [u64, vp, vp, vp, u64, ctypes.POINTER(u64)]
    lib.orc_list_triangles.restype = ctypes.c_int
    for fn in (lib.orc_triangle_reduce, lib.orc_edge_sample):
        fn.argtypes = [u64, vp, vp, dbl, u64, vp, vp, vp]
        fn.restype = ctypes.c_int
    lib.orc_triangle_reduce_x.argtypes = [u64, vp, vp, dbl, u64, ctypes.c_int, vp, vp, vp]
    lib.orc_triangle_reduce_x.restype = ctypes.c_int
    lib.orc_triangle_reduce_eo.argtypes = [u64, vp, vp, dbl, u64, ctypes.c_uint32, vp, vp, vp]
    lib.orc_triangle_reduce_eo.restype = ctypes.c_int
    lib.orc_spectral_sparsify.argtypes = [u64, vp, vp, dbl, u64, vp, vp, vp, vp]
    lib.orc_spectral_sparsify.restype = ctypes.c_int
    lib.orc_tr_rows.argtypes = [u64, vp, vp, dbl, u64, vp, u64, vp, vp]
    lib.orc_tr_rows.restype = ctypes.c_int
    lib.orc_edge_triangle_counts.argtypes = [u64, vp, vp, vp]
    lib.orc_edge_triangle_counts.restype = ctypes.c_int
    _lib = lib
    return lib


def _arrays(g):
    ro = np.ascontiguousarray(g.row_off, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.uint32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.uint32)  # valid pointer for empty graphs
    return ro, col


def philox4x32_10(ctr, key):
    """Philox4x32-10 of a 4-word counter and 2-word key (uint32 words)."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return [int(x) for x in out]


def threshold(p: float) -> int:
    t = ctypes.c_uint64(0)
    if _load().orc_threshold(float(p), ctypes.byref(t)) != 0:
        raise ValueError(f"p must lie in [0, 1], got {p!r}")
    return int(t.value)


def validate(g) -> int:
    ro, col = _arrays(g)
    return int(_load().orc_validate(g.n, ro.ctypes.data, col.ctypes.data))


def list_triangles(g) -> np.ndarray:
    """All triangles as an (T, 3) uint32 array of id-sorted triples."""
    lib = _load()
    ro, col = _arrays(g)
    cnt = ctypes.c_uint64(0)
    lib.orc_list_triangles(g.n, ro.ctypes.data, col.ctypes.data, None, 0, ctypes.byref(cnt))
    out = np.zeros((max(int(cnt.value), 1), 3), dtype=np.uint32)
    lib.orc_list_triangles(g.n, ro.ctypes.data, col.ctypes.data, out.ctypes.data, cnt.value,
                           ctypes.byref(cnt))
    return out[: int(cnt.value)]


def _run(fn, g, p, seed):
    ro, col = _arrays(g)
    out_ro = np.zeros(g.n + 1, dtype=np.int64)
    out_col = np.zeros(max(g.nnz, 1), dtype=np.uint32)
    stats = np.zeros(6, dtype=np.uint64)
    rc = fn(g.n, ro.ctypes.data, col.ctypes.data, float(p), int(seed) & (2**64 - 1),
            out_ro.ctypes.data, out_col.ctypes.data, stats.ctypes.data)
    if rc == -1:
        raise ValueError(f"p must lie in [0, 1], got {p!r}")
    if rc != 0:
        raise RuntimeError(f"oracle failed rc={rc}")
    nnz_out = int(out_ro[-1])
    return out_ro, out_col[:nnz_out].copy(), dict(zip(STAT_KEYS, (int(x) for x in stats)))


def triangle_reduce(g, p: float, seed: int):
    """Triangle p-1-Reduction of CSR ``g``: (row_off, col, stats)."""
    return _run(_load().orc_triangle_reduce, g, p, seed)


def triangle_reduce_x(g, p: float, seed: int, variant: int):
    """Triangle p-x-Reduction variants: 1 = p-1, 2 = p-2 (a selected triangle
    keeps one uniform edge), 3 = Min-Count p-1 (removes its edge in the fewest
    input triangles, ties uniform), 4 = Edge-Once p-1 (selected triangles in
    priority order; one is considered only if none of its edges has been).
    Returns (row_off, col, stats)."""
    lib = _load()

    def fn(n, ro, col, p_, seed_, oro, ocol, st):
        return lib.orc_triangle_reduce_x(n, ro, col, p_, seed_, int(variant), oro, ocol, st)

    return _run(fn, g, p, seed)


def triangle_reduce_eo(g, p: float, seed: int, buckets: int = 1):
    """Edge-Once Triangle p-1-Reduction (variant 4 of ``triangle_reduce_x``),
    walking the selected triangles in ``buckets`` consecutive ranges of their
    priority word so that only one range is held in memory at a time; the
    result does not depend on ``buckets``.  Returns (row_off, col, stats)."""
    lib = _load()
    if int(buckets) < 1:
        raise ValueError("buckets must be >= 1")

    def fn(n, ro, col, p_, seed_, oro, ocol, st):
        return lib.orc_triangle_reduce_eo(n, ro, col, p_, seed_, int(buckets), oro, ocol, st)

    return _run(fn, g, p, seed)


def spectral_sparsify(g, upsilon: float, seed: int):
    """Spectral sparsification (keep {u,v} with p_uv = min(1, upsilon /
    min(d_u, d_v)), weight 1/p_uv): (row_off, col, weights float32, stats)."""
    lib = _load()
    ro, col = _arrays(g)
    out_ro = np.zeros(g.n + 1, dtype=np.int64)
    out_col = np.zeros(max(g.nnz, 1), dtype=np.uint32)
    out_w = np.zeros(max(g.nnz, 1), dtype=np.float32)
    stats = np.zeros(6, dtype=np.uint64)
    rc = lib.orc_spectral_sparsify(g.n, ro.ctypes.data, col.ctypes.data, float(upsilon),
                                   int(seed) & (2**64 - 1), out_ro.ctypes.data, out_col.ctypes.data,
                                   out_w.ctypes.data, stats.ctypes.data)
    if rc == -1:
        raise ValueError(f"upsilon must be >= 0, got {upsilon!r}")
    if rc != 0:
        raise RuntimeError(f"oracle failed rc={rc}")
    k = int(out_ro[-1])
    return out_ro, out_col[:k].copy(), out_w[:k].copy(), dict(zip(STAT_KEYS, (int(x) for x in stats)))


def edge_sample(g, p: float, seed: int):
    """Uniform edge sampling (p = deletion probability): (row_off, col, stats)."""
    return _run(_load().orc_edge_sample, g, p, seed)


def tr_rows(g, p: float, seed: int, rows):
    """Output rows of Triangle p-1-Reduction for the listed vertices only."""
    lib = _load()
    ro, col = _arrays(g)
    rows = np.ascontiguousarray(rows, dtype=np.uint32)
    total = int(sum(int(g.row_off[r + 1] - g.row_off[r]) for r in rows))
    out_off = np.zeros(len(rows) + 1, dtype=np.int64)
    out_col = np.zeros(max(total, 1), dtype=np.uint32)
    rc = lib.orc_tr_rows(g.n, ro.ctypes.data, col.ctypes.data, float(p),
                         int(seed) & (2**64 - 1), rows.ctypes.data, len(rows),
                         out_off.ctypes.data, out_col.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle tr_rows failed rc={rc}")
    return [out_col[out_off[i]:out_off[i + 1]].copy() for i in range(len(rows))]


def degree_distribution(row_off) -> dict:
    """{k: fraction of the vertices with degree k} of a CSR (degree = row
    length), in float64."""
    deg = np.diff(np.asarray(row_off, dtype=np.int64))
    n = deg.size
    out = {}
    for k, c in zip(*np.unique(deg, return_counts=True)):
        out[int(k)] = float(c) / n
    return out


def degree_kl(row_off_p, row_off_q) -> float:
    """Kullback-Leibler divergence D_KL(P||Q) = sum_k P(k) log2(P(k)/Q(k))
    (section 5, in bits) of the degree distribution Q of a compressed graph
    from the distribution P of its input; +inf if a degree of P is missing
    from Q, 0 for empty graphs."""
    if len(row_off_p) != len(row_off_q):
        raise ValueError("both graphs must have the same vertex count")
    if len(row_off_p) <= 1:
        return 0.0
    P, Q = degree_distribution(row_off_p), degree_distribution(row_off_q)
    total = 0.0
    for k in sorted(P):
        if k not in Q:
            return float("inf")
        total += P[k] * math.log2(P[k] / Q[k])
    return total


def edge_triangle_counts(g) -> np.ndarray:
    """t[j] = number of triangles containing the edge of CSR entry j."""
    ro, col = _arrays(g)
    t = np.zeros(max(g.nnz, 1), dtype=np.uint32)
    rc = _load().orc_edge_triangle_counts(g.n, ro.ctypes.data, col.ctypes.data, t.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle edge_triangle_counts failed rc={rc}")
    return t[: g.nnz]
