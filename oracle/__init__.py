"""The oracle — TEST INFRASTRUCTURE ONLY.

Plain CPU reference results for BFS levels, SSSP distances, PageRank,
Brandes betweenness centrality and connected components, computed in C
(``oracle.c``) from their plain definitions in fp64 / int64.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library and never imports it.

Readings of the paper that bind both sides (the paper leaves them open):
  * PageRank divides a vertex's rank by its out-degree (Page et al., cited in
    section 7.1; Figure 14 omits the division), starts from 1/N, updates
    synchronously, runs a fixed number of iterations, and by default spreads
    the rank held by out-degree-0 vertices uniformly ("uniform"); "drop"
    discards it as Figure 14 read literally does.
  * Betweenness follows Brandes' recurrence with the (1 + delta_w) term that
    Figure 18 omits; sums run over ordered pairs (no halving) and the source
    itself receives nothing.
  * Unreachable vertices get INT32_MAX as level/distance.  A finite SSSP
    distance >= INT32_MAX is reported as an overflow.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

INF = np.iinfo(np.int32).max
DANGLING = {"uniform": 0, "drop": 1}

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


class OracleError(RuntimeError):
    pass


class DistanceOverflow(OracleError):
    """A finite shortest-path distance does not fit below INT32_MAX."""


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_bfs.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int32, _i32p, _i32p]
        lib.oracle_sssp_dijkstra.argtypes = [ctypes.c_int64, _i64p, _i32p, _i32p,
                                             ctypes.c_int32, _i64p]
        lib.oracle_sssp_bellman_ford.argtypes = [ctypes.c_int64, _i64p, _i32p, _i32p,
                                                 ctypes.c_int32, _i64p]
        lib.oracle_pagerank.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_double,
                                        ctypes.c_int32, ctypes.c_int32, _f64p]
        lib.oracle_cc.argtypes = [ctypes.c_int64, _i64p, _i32p, _i32p]
        lib.oracle_bc.argtypes = [ctypes.c_int64, _i64p, _i32p, _i32p, ctypes.c_int32,
                                  _f64p, _f64p]
        for f in (lib.oracle_bfs, lib.oracle_sssp_dijkstra, lib.oracle_sssp_bellman_ford,
                  lib.oracle_pagerank, lib.oracle_bc):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _csr(offsets, cols):
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    col = np.ascontiguousarray(cols, dtype=np.int32)
    n = off.size - 1
    return n, off, col


def _check(rc: int):
    if rc != 0:
        raise OracleError(f"oracle call failed with code {rc}")


def bfs(offsets, cols, root: int, parents: bool = False):
    """Levels (int32, INF = unreachable) from `root`; optionally parents."""
    n, off, col = _csr(offsets, cols)
    lev = np.empty(n, dtype=np.int32)
    par = np.empty(n, dtype=np.int32) if parents else None
    _check(_load().oracle_bfs(n, off.ctypes.data_as(_i64p), col.ctypes.data_as(_i32p),
                              int(root), lev.ctypes.data_as(_i32p),
                              par.ctypes.data_as(_i32p) if parents else None))
    return (lev, par) if parents else lev


def sssp64(offsets, cols, weights, root: int, method: str = "dijkstra") -> np.ndarray:
    """Exact int64 distances; INT64_MAX = unreachable."""
    n, off, col = _csr(offsets, cols)
    w = np.ascontiguousarray(weights, dtype=np.int32)
    dist = np.empty(n, dtype=np.int64)
    fn = _load().oracle_sssp_dijkstra if method == "dijkstra" else _load().oracle_sssp_bellman_ford
    _check(fn(n, off.ctypes.data_as(_i64p), col.ctypes.data_as(_i32p),
              w.ctypes.data_as(_i32p), int(root), dist.ctypes.data_as(_i64p)))
    return dist


def sssp(offsets, cols, weights, root: int, method: str = "dijkstra") -> np.ndarray:
    """int32 distances with INF = INT32_MAX; raises DistanceOverflow when a
    finite distance is >= INT32_MAX."""
    d = sssp64(offsets, cols, weights, root, method)
    unreach = d == np.iinfo(np.int64).max
    if np.any(d[~unreach] >= INF):
        raise DistanceOverflow("finite distance >= INT32_MAX")
    out = np.where(unreach, INF, d).astype(np.int32)
    return out


def pagerank(offsets, cols, damping: float = 0.85, iterations: int = 10,
             dangling: str = "uniform") -> np.ndarray:
    n, off, col = _csr(offsets, cols)
    r = np.empty(n, dtype=np.float64)
    _check(_load().oracle_pagerank(n, off.ctypes.data_as(_i64p), col.ctypes.data_as(_i32p),
                                   float(damping), int(iterations), DANGLING[dangling],
                                   r.ctypes.data_as(_f64p)))
    return r


def bc(offsets, cols, sources: Sequence[int], return_sigma: bool = False):
    """Betweenness summed over `sources` (ordered pairs, not halved)."""
    n, off, col = _csr(offsets, cols)
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
    out = np.empty(n, dtype=np.float64)
    sig = np.empty(n, dtype=np.float64) if return_sigma else None
    _check(_load().oracle_bc(n, off.ctypes.data_as(_i64p), col.ctypes.data_as(_i32p),
                             src.ctypes.data_as(_i32p), src.size, out.ctypes.data_as(_f64p),
                             sig.ctypes.data_as(_f64p) if return_sigma else None))
    return (out, sig) if return_sigma else out



def cc(offsets, cols) -> np.ndarray:
    """Connected components of the undirected graph (edge direction ignored):
    labels[v] = smallest vertex id in v's component."""
    n, off, col = _csr(offsets, cols)
    lab = np.empty(n, dtype=np.int32)
    _check(_load().oracle_cc(n, off.ctypes.data_as(_i64p), col.ctypes.data_as(_i32p), lab.ctypes.data_as(_i32p)))
    return lab
