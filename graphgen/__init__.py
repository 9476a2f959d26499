"""Seeded synthetic graph inputs shared by the tests, the bench and the oracle
checks.

This module holds no graph-algorithm arithmetic: it generates edge lists
(R-MAT, uniform G(n, m), hand-made lists), turns them into CSR (neighbours
sorted, self-loops and duplicates dropped, optionally symmetrized) and draws
per-edge weights and root vertices.  All randomness is counter based
(SplitMix64 finaliser keyed by seed/stream/index), so results do not depend on
the thread count.

R-MAT parameters default to the paper's workload description: (A, B, C) =
(0.57, 0.19, 0.19), D = 0.05, 16 generated edges per vertex (section 5,
Table 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_intp = ctypes.POINTER(ctypes.c_int)

STREAM_ROOTS = 5


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.gg_rmat_csr.restype = ctypes.c_void_p
        lib.gg_rmat_csr.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                    ctypes.c_int, ctypes.c_int, _i64p, _intp]
        lib.gg_uniform_csr.restype = ctypes.c_void_p
        lib.gg_uniform_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                       ctypes.c_int, _i64p, _intp]
        lib.gg_edges_csr.restype = ctypes.c_void_p
        lib.gg_edges_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, _i32p, _i32p,
                                     ctypes.c_int, _i64p, _intp]
        lib.gg_take.restype = None
        lib.gg_take.argtypes = [ctypes.c_void_p, _i64p, _i32p]
        lib.gg_weights.restype = None
        lib.gg_weights.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_uint64,
                                   ctypes.c_int, ctypes.c_int32, ctypes.c_int32, _i32p]
        lib.gg_draws.restype = None
        lib.gg_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                 ctypes.c_int64, _u64p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


@dataclass
class CSR:
    """Host CSR graph: row_offsets int64[n+1], col_indices int32[nnz]."""
    n: int
    offsets: np.ndarray
    cols: np.ndarray
    symmetric: bool
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.offsets[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)


def _take(handle, n: int, nnz: int, err: int) -> tuple[np.ndarray, np.ndarray]:
    if not handle:
        raise MemoryError(f"graphgen failed with code {err}")
    off = np.empty(n + 1, dtype=np.int64)
    col = np.empty(max(nnz, 0), dtype=np.int32)
    _load().gg_take(handle, _ptr(off, _i64p), _ptr(col, _i32p))
    return off, col


def rmat(scale: int, edge_factor: int = 16, seed: int = 1, symmetrize: bool = True,
         permute: bool = True, a: float = 0.57, b: float = 0.19, c: float = 0.19) -> CSR:
    lib = _load()
    nnz = ctypes.c_int64(0)
    err = ctypes.c_int(0)
    h = lib.gg_rmat_csr(scale, edge_factor, a, b, c, seed, int(symmetrize), int(permute),
                        ctypes.byref(nnz), ctypes.byref(err))
    off, col = _take(h, 1 << scale, nnz.value, err.value)
    return CSR(1 << scale, off, col, symmetrize, f"rmat{scale}")


def uniform(n: int, m: int, seed: int = 1, symmetrize: bool = True) -> CSR:
    lib = _load()
    nnz = ctypes.c_int64(0)
    err = ctypes.c_int(0)
    h = lib.gg_uniform_csr(n, m, seed, int(symmetrize), ctypes.byref(nnz), ctypes.byref(err))
    off, col = _take(h, n, nnz.value, err.value)
    return CSR(n, off, col, symmetrize, f"uniform{n}")


def from_edges(n: int, src, dst, symmetrize: bool = True, name: str = "edges") -> CSR:
    lib = _load()
    s = np.ascontiguousarray(np.asarray(src, dtype=np.int32))
    d = np.ascontiguousarray(np.asarray(dst, dtype=np.int32))
    assert s.shape == d.shape
    nnz = ctypes.c_int64(0)
    err = ctypes.c_int(0)
    h = lib.gg_edges_csr(n, s.size, _ptr(s, _i32p), _ptr(d, _i32p), int(symmetrize),
                         ctypes.byref(nnz), ctypes.byref(err))
    off, col = _take(h, n, nnz.value, err.value)
    return CSR(n, off, col, symmetrize, name)


def weights(g: CSR, seed: int = 2, lo: int = 1, hi: int = 255) -> np.ndarray:
    """Uniform int32 weights in [lo, hi]; one draw per unordered pair when the
    graph is symmetric, one per directed edge otherwise."""
    w = np.empty(max(g.nnz, 0), dtype=np.int32)
    _load().gg_weights(g.n, _ptr(g.offsets, _i64p), _ptr(g.cols, _i32p), seed,
                       int(g.symmetric), lo, hi, _ptr(w, _i32p))
    return w


def draws(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().gg_draws(seed, stream, start, count, _ptr(out, _u64p))
    return out


def max_degree_vertex(g: CSR) -> int:
    """Highest out-degree vertex; ties go to the lowest id."""
    return int(np.argmax(g.degrees()))


def sample_roots(g: CSR, k: int, seed: int = 3) -> np.ndarray:
    """k distinct vertices of out-degree >= 1, chosen by smallest keyed draw."""
    cand = np.nonzero(g.degrees() > 0)[0]
    if cand.size == 0:
        return np.zeros(0, dtype=np.int32)
    keys = draws(seed, STREAM_ROOTS, 0, g.n)[cand]
    order = np.argsort(keys, kind="stable")[: min(k, cand.size)]
    return cand[order].astype(np.int32)


def workload(name: str) -> CSR:
    """Named inputs: 'rmatS' (symmetrized R-MAT at scale S, seed 1),
    'rmatS_dir' (directed R-MAT), 'uniformN' (G(2^N, 4*2^N) symmetrized)."""
    if name.startswith("rmat") and name.endswith("_dir"):
        return rmat(int(name[4:-4]), symmetrize=False)
    if name.startswith("rmat"):
        return rmat(int(name[4:]))
    if name.startswith("uniform"):
        s = int(name[7:])
        return uniform(1 << s, 4 << s, seed=1)
    raise ValueError(name)
