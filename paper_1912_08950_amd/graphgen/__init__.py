"""Seeded synthetic input graphs (G(n,q) and R-MAT) as symmetric sorted CSR.

This module draws inputs only; it holds none of the compression method's
arithmetic.  Both the GPU path and the CPU oracle consume what it returns.
The native part (``graphgen.c``) is built with gcc + OpenMP into
``libslimgen.so`` next to this file; output does not depend on thread count.

Workload recipes (the paper's real graphs are not available; these synthetic
graphs stand in for them):

* ``er(n, avg_degree, seed)`` -- G(n, q) with q = avg_degree / (n - 1).
* ``rmat(scale, edge_factor, seed)`` -- R-MAT with a,b,c,d = .57,.19,.19,.05,
  edge_factor * 2^scale directed samples, ids through a seeded bijection of
  [0, 2^scale), symmetrized, self-loops and duplicates removed.
* ``batch_mix(count, seed, ...)`` -- a mixed population of many graphs: half
  G(n, q), half R-MAT, n log-uniform in [n_lo, n_hi], average degree d
  uniform in [d_lo, d_hi].  An R-MAT member is drawn at scale ceil(log2 n)
  with endpoints >= n dropped; its sample count d/2 * n * (2^scale / n)^2
  makes up for the dropped samples, so its average degree is d before
  duplicate removal.  ``mix_seed(base, i)`` derives the per-graph seeds.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libslimgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libslimgen.so with gcc (-O3 -fopenmp)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
               "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    i64p = ctypes.POINTER(ctypes.POINTER(ctypes.c_int64))
    u32p = ctypes.POINTER(ctypes.POINTER(ctypes.c_uint32))
    u64 = ctypes.c_uint64
    lib.sg_gen_er.argtypes = [u64, ctypes.c_double, u64, i64p, u32p, ctypes.POINTER(u64)]
    lib.sg_gen_er.restype = ctypes.c_int
    lib.sg_gen_rmat.argtypes = [ctypes.c_int, u64, u64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int, u64, i64p, u32p,
                                ctypes.POINTER(u64)]
    lib.sg_gen_rmat.restype = ctypes.c_int
    lib.sg_pairs_csr.argtypes = [u64, ctypes.c_void_p, ctypes.c_void_p, u64, i64p, u32p,
                                 ctypes.POINTER(u64)]
    lib.sg_pairs_csr.restype = ctypes.c_int
    lib.sg_copy_free.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint32),
                                 u64, u64, ctypes.c_void_p, ctypes.c_void_p]
    lib.sg_copy_free.restype = None
    lib.sg_num_threads.restype = ctypes.c_int
    vp = ctypes.c_void_p
    lib.sg_gen_many.argtypes = [u64, vp, vp, vp, vp, vp, vp,
                                ctypes.POINTER(ctypes.POINTER(ctypes.c_int64)),
                                ctypes.POINTER(ctypes.POINTER(ctypes.c_uint32)), vp]
    lib.sg_gen_many.restype = ctypes.c_int
    _lib = lib
    return lib


@dataclass
class CSR:
    """Undirected simple graph: symmetric CSR, sorted rows, no self-loops."""
    row_off: np.ndarray  # int64 [n+1]
    col: np.ndarray      # uint32 [nnz]
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.row_off.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_off)


def _collect(rc, n, ro_p, col_p, nnz, name) -> CSR:
    lib = _load()
    if rc != 0:
        raise RuntimeError(f"graph generator failed (rc={rc}) for {name}")
    nnz = int(nnz.value)
    row_off = np.empty(n + 1, dtype=np.int64)
    col = np.empty(nnz, dtype=np.uint32)
    lib.sg_copy_free(ro_p, col_p, n, nnz, row_off.ctypes.data, col.ctypes.data)
    return CSR(row_off, col, name)


def er(n: int, avg_degree: float, seed: int) -> CSR:
    """G(n, q) with q = avg_degree / (n - 1)."""
    lib = _load()
    ro_p = ctypes.POINTER(ctypes.c_int64)()
    col_p = ctypes.POINTER(ctypes.c_uint32)()
    nnz = ctypes.c_uint64(0)
    rc = lib.sg_gen_er(n, float(avg_degree), seed, ctypes.byref(ro_p), ctypes.byref(col_p),
                       ctypes.byref(nnz))
    return _collect(rc, n, ro_p, col_p, nnz, f"er_n{n}_d{avg_degree:g}_s{seed}")


def rmat(scale: int, edge_factor: float, seed: int, n: int | None = None,
         abc=(0.57, 0.19, 0.19), permute: bool = True, samples: int | None = None) -> CSR:
    """R-MAT graph; n defaults to 2^scale (endpoints >= n are rejected)."""
    lib = _load()
    nn = (1 << scale) if n is None else int(n)
    if samples is None:
        samples = int(round(edge_factor * nn))
    ro_p = ctypes.POINTER(ctypes.c_int64)()
    col_p = ctypes.POINTER(ctypes.c_uint32)()
    nnz = ctypes.c_uint64(0)
    rc = lib.sg_gen_rmat(scale, nn, samples, abc[0], abc[1], abc[2], 1 if permute else 0, seed,
                         ctypes.byref(ro_p), ctypes.byref(col_p), ctypes.byref(nnz))
    return _collect(rc, nn, ro_p, col_p, nnz, f"rmat_s{scale}_ef{edge_factor:g}_s{seed}")


def from_pairs(n: int, pairs, name: str = "pairs") -> CSR:
    """CSR of the undirected simple graph spanned by a list of (u, v) pairs."""
    lib = _load()
    arr = np.asarray(pairs, dtype=np.uint32).reshape(-1, 2)
    pu = np.ascontiguousarray(arr[:, 0])
    pv = np.ascontiguousarray(arr[:, 1])
    ro_p = ctypes.POINTER(ctypes.c_int64)()
    col_p = ctypes.POINTER(ctypes.c_uint32)()
    nnz = ctypes.c_uint64(0)
    rc = lib.sg_pairs_csr(n, pu.ctypes.data, pv.ctypes.data, len(pu), ctypes.byref(ro_p),
                          ctypes.byref(col_p), ctypes.byref(nnz))
    return _collect(rc, n, ro_p, col_p, nnz, name)


# ---- small named families used by tests ---------------------------------

def complete(n: int) -> CSR:
    return from_pairs(n, [(u, v) for u in range(n) for v in range(u + 1, n)], f"K{n}")


def path(n: int) -> CSR:
    return from_pairs(n, [(i, i + 1) for i in range(n - 1)], f"P{n}")


def cycle(n: int) -> CSR:
    return from_pairs(n, [(i, (i + 1) % n) for i in range(n)], f"C{n}")


def star(n: int) -> CSR:
    return from_pairs(n, [(0, i) for i in range(1, n)], f"S{n}")


def grid(r: int, c: int) -> CSR:
    pairs = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                pairs.append((v, v + 1))
            if i + 1 < r:
                pairs.append((v, v + c))
    return from_pairs(r * c, pairs, f"grid{r}x{c}")


def complete_bipartite(a: int, b: int) -> CSR:
    return from_pairs(a + b, [(i, a + j) for i in range(a) for j in range(b)], f"K{a},{b}")


def friendship(k: int) -> CSR:
    """k triangles sharing the single vertex 0 (edge-disjoint triangles)."""
    pairs = []
    for t in range(k):
        x, y = 1 + 2 * t, 2 + 2 * t
        pairs += [(0, x), (0, y), (x, y)]
    return from_pairs(2 * k + 1, pairs, f"F{k}")


def empty(n: int) -> CSR:
    return CSR(np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.uint32), f"E{n}")


def num_threads() -> int:
    return int(_load().sg_num_threads())


def mix_seed(base: int, i: int) -> int:
    """Per-item seed from a base seed: the SplitMix64 output function applied
    to base + (i + 1) * 0x9E3779B97F4A7C15 (mod 2^64)."""
    m = (1 << 64) - 1
    z = (int(base) + (int(i) + 1) * 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def batch_mix(count: int, seed: int, n_lo: int = 1000, n_hi: int = 200000, d_lo: float = 4.0,
              d_hi: float = 64.0):
    """`count` graphs, even indices G(n, q) and odd indices R-MAT, with n
    log-uniform in [n_lo, n_hi] and average degree uniform in [d_lo, d_hi]
    (parameters from numpy's PCG64 seeded with `seed`; graph i's generator
    seed is mix_seed(seed, i)).  Generated in parallel across graphs; graph
    i equals what er() / rmat() return for its parameters.  Returns a list
    of CSR."""
    rng = np.random.default_rng(seed)
    ns = np.maximum(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), count)).astype(np.int64), 2)
    ds = rng.uniform(d_lo, d_hi, count)
    kind = np.array([i % 2 for i in range(count)], dtype=np.int32)
    seeds = np.array([mix_seed(seed, i) & 0x7FFFFFFFFFFFFFFF for i in range(count)], dtype=np.uint64)
    scales = np.array([max(1, int(np.ceil(np.log2(int(n))))) for n in ns], dtype=np.int32)
    samples = np.array([int(round(d / 2 * n * ((1 << int(s)) / n) ** 2))
                        for n, d, s in zip(ns, ds, scales)], dtype=np.uint64)
    lib = _load()
    ro_ps = (ctypes.POINTER(ctypes.c_int64) * count)()
    col_ps = (ctypes.POINTER(ctypes.c_uint32) * count)()
    nnzs = np.zeros(count, dtype=np.uint64)
    ns_u = ns.astype(np.uint64)
    rc = lib.sg_gen_many(count, kind.ctypes.data, ns_u.ctypes.data, ds.ctypes.data,
                         seeds.ctypes.data, scales.ctypes.data, samples.ctypes.data, ro_ps, col_ps,
                         nnzs.ctypes.data)
    out = []
    for i in range(count):
        n, nnz = int(ns[i]), int(nnzs[i])
        name = (f"er_n{n}_d{ds[i]:g}_s{int(seeds[i])}" if kind[i] == 0 else
                f"rmat_s{int(scales[i])}_n{n}_s{int(seeds[i])}")
        if not ro_ps[i]:
            raise RuntimeError(f"graph generator failed (rc={rc}) for {name}")
        row_off = np.empty(n + 1, dtype=np.int64)
        col = np.empty(nnz, dtype=np.uint32)
        lib.sg_copy_free(ro_ps[i], col_ps[i], n, nnz, row_off.ctypes.data, col.ctypes.data)
        out.append(CSR(row_off, col, name))
    if rc != 0:
        raise RuntimeError(f"graph generator failed (rc={rc})")
    return out


def batch_mix_params(count: int, seed: int, n_lo: int = 1000, n_hi: int = 200000,
                     d_lo: float = 4.0, d_hi: float = 64.0):
    """The per-graph (kind, n, d, generator seed, scale, samples) that
    batch_mix(count, seed, ...) draws, for checking it graph by graph."""
    rng = np.random.default_rng(seed)
    ns = np.maximum(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), count)).astype(np.int64), 2)
    ds = rng.uniform(d_lo, d_hi, count)
    out = []
    for i in range(count):
        n, d = int(ns[i]), float(ds[i])
        s = mix_seed(seed, i) & 0x7FFFFFFFFFFFFFFF
        scale = max(1, int(np.ceil(np.log2(n))))
        out.append(("er" if i % 2 == 0 else "rmat", n, d, s, scale,
                    int(round(d / 2 * n * ((1 << scale) / n) ** 2))))
    return out
