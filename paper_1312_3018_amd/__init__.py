"""Python binding of libtg (C ABI in include/tg.h).

Argument marshalling only: every step of every algorithm runs in the HIP
kernels of libtg.so.  PyTorch supplies device memory (output tensors) and
streams.  The functions carry the C names: graph_load_csr,
partition_by_degree, bfs, sssp, pagerank, bc, partition_info, tg_last_error,
tg_last_stats.  Importing the package does not load the library; the first
call does, and raises if libtg.so is missing (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtg.so")

TG_OK, TG_EINVAL, TG_ENOMEM, TG_EDEVICE, TG_ERANGE, TG_EUNSUPPORTED, TG_ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
TG_PTRS_DEVICE, TG_VALIDATE, TG_SYMMETRIC = 0x1, 0x2, 0x4
TG_INF = 2**31 - 1
STRATEGY = {"high": 0, "low": 1, "rand": 2}
DANGLING = {"uniform": 0, "drop": 1}

_c_i64p = ctypes.POINTER(ctypes.c_int64)
_c_i32p = ctypes.POINTER(ctypes.c_int32)


class TGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libtg.so not built at {LIB_PATH}; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.graph_load_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, vp, vp, vp, ctypes.c_uint32, vp,
                                   ctypes.POINTER(vp)]
    lib.partition_by_degree.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                        ctypes.c_char_p, ctypes.POINTER(vp)]
    lib.partition_retune.argtypes = [vp, ctypes.c_char_p]
    lib.bfs.argtypes = [vp, _c_i32p, ctypes.c_int32, vp, vp, vp]
    lib.sssp.argtypes = [vp, _c_i32p, ctypes.c_int32, vp, vp]
    lib.bfs_batched.argtypes = [vp, _c_i32p, ctypes.c_int32, vp, vp]
    lib.bc_batched.argtypes = [vp, _c_i32p, ctypes.c_int32, vp, vp]
    lib.bc_batched.restype = ctypes.c_int
    lib.sssp_batched.argtypes = [vp, _c_i32p, ctypes.c_int32, vp, vp]
    lib.pagerank.argtypes = [vp, ctypes.c_float, ctypes.c_int32, ctypes.c_int32, vp, vp]
    lib.bc.argtypes = [vp, _c_i32p, ctypes.c_int32, vp, vp]
    lib.bc_multi.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(_c_i32p), _c_i32p,
                             ctypes.POINTER(vp), vp]
    lib.bc_multi.restype = ctypes.c_int
    lib.cc.argtypes = [vp, vp, vp]
    lib.server_create.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
    lib.server_add_graph.argtypes = [vp, vp, _c_i32p]
    lib.server_submit.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                                  ctypes.POINTER(ctypes.c_uint64)]
    lib.server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
    lib.server_stats.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.server_destroy.argtypes = [vp]
    lib.server_destroy.restype = None
    for f in (lib.server_create, lib.server_add_graph, lib.server_submit, lib.server_wait, lib.server_stats):
        f.restype = ctypes.c_int
    lib.graph_free.argtypes = [vp]
    lib.partition_free.argtypes = [vp]
    lib.tg_last_error.restype = ctypes.c_char_p
    lib.partition_info.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.tg_last_stats.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    lib.bfs_noalloc.argtypes = [vp, _c_i32p, ctypes.c_int32, vp, vp]
    lib.tg_set_timing.argtypes = [ctypes.c_int]
    lib.tg_set_timing.restype = None
    for f in (lib.graph_load_csr, lib.partition_by_degree, lib.partition_retune, lib.bfs, lib.sssp, lib.pagerank, lib.bc,
              lib.bfs_batched, lib.sssp_batched,
              lib.partition_info, lib.tg_last_stats):
        f.restype = ctypes.c_int
    lib.graph_free.restype = None
    lib.partition_free.restype = None
    _lib = lib
    return lib


def require_native():
    """Load libtg.so or raise."""
    return _load()


def tg_last_error() -> str:
    return _load().tg_last_error().decode()


def _check(rc: int):
    if rc != TG_OK:
        raise TGError(rc, tg_last_error())


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _is_cuda_tensor(x) -> bool:
    return hasattr(x, "is_cuda") and x.is_cuda


class Graph:
    """Library-owned host copy of a CSR graph."""

    def __init__(self, handle, n: int, m: int, symmetric: bool, weighted: bool):
        self._h = handle
        self.n, self.m, self.symmetric, self.weighted = n, m, symmetric, weighted

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h:
            _load().graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Partition:
    """Degree-ordered partition(s) placed on the device; keeps its graph alive."""

    def __init__(self, handle, graph: Graph):
        self._h = handle
        self.graph = graph

    @property
    def handle(self):
        return self._h

    @property
    def n(self) -> int:
        return self.graph.n

    def info(self) -> dict:
        return partition_info(self)

    def free(self):
        if self._h:
            _load().partition_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def graph_load_csr(num_vertices: int, row_offsets, col_indices, weights=None, *, symmetric: bool = False,
                   validate: bool = True, stream=None) -> Graph:
    """Load CSR arrays (numpy host arrays, or torch CUDA tensors)."""
    lib = _load()
    flags = (TG_VALIDATE if validate else 0) | (TG_SYMMETRIC if symmetric else 0)
    if _is_cuda_tensor(row_offsets):
        import torch
        assert row_offsets.dtype == torch.int64 and col_indices.dtype == torch.int32
        flags |= TG_PTRS_DEVICE
        ptrs = (row_offsets.data_ptr(), col_indices.data_ptr() if col_indices.numel() else None,
                weights.data_ptr() if weights is not None else None)
        m = int(col_indices.numel())
        keep = (row_offsets, col_indices, weights)
        st = _stream_handle(stream)
    else:
        off = np.ascontiguousarray(row_offsets, dtype=np.int64)
        col = np.ascontiguousarray(col_indices, dtype=np.int32)
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.int32)
        ptrs = (off.ctypes.data, col.ctypes.data if col.size else None, None if w is None else w.ctypes.data)
        m = int(col.size)
        keep = (off, col, w)
        st = None
    out = ctypes.c_void_p()
    _check(lib.graph_load_csr(int(num_vertices), m, ptrs[0], ptrs[1], ptrs[2], flags, st, ctypes.byref(out)))
    del keep
    return Graph(out.value, int(num_vertices), m, symmetric, weights is not None)


def partition_by_degree(graph: Graph, strategy: str = "high", cpu_edge_share: float = 0.0, seed: int = 0,
                        tuning=None) -> Partition:
    lib = _load()
    tj = None
    if tuning is not None:
        tj = (tuning if isinstance(tuning, str) else json.dumps(tuning)).encode()
    out = ctypes.c_void_p()
    _check(lib.partition_by_degree(graph.handle, STRATEGY[strategy], float(cpu_edge_share), int(seed), tj,
                                   ctypes.byref(out)))
    return Partition(out.value, graph)


def partition_retune(part: Partition, tuning=None) -> None:
    """Re-derive bins and launch shapes of `part` from a tuning dict/JSON."""
    tj = None
    if tuning is not None:
        tj = (tuning if isinstance(tuning, str) else json.dumps(tuning)).encode()
    _check(_load().partition_retune(part.handle, tj))


def partition_info(part: Partition) -> dict:
    lib = _load()
    need = lib.partition_info(part.handle, None, 0)
    if need < 0:
        _check(need)
    buf = ctypes.create_string_buffer(need + 1)
    lib.partition_info(part.handle, buf, need + 1)
    return json.loads(buf.value.decode())


def tg_last_stats() -> dict:
    lib = _load()
    need = lib.tg_last_stats(None, 0)
    buf = ctypes.create_string_buffer(need + 1)
    lib.tg_last_stats(buf, need + 1)
    return json.loads(buf.value.decode())


def tg_set_timing(on: bool) -> None:
    """Per-kernel HIP-event timing on (reported by tg_last_stats) or off."""
    _load().tg_set_timing(1 if on else 0)


def _roots(roots) -> np.ndarray:
    return np.ascontiguousarray(np.atleast_1d(np.asarray(roots, dtype=np.int32)))


def _out(t, shape, dtype_name: str):
    import torch
    dt = getattr(torch, dtype_name)
    if t is None:
        return torch.empty(shape, dtype=dt, device="cuda")
    assert t.is_cuda and t.dtype == dt and t.is_contiguous() and t.numel() >= int(np.prod(shape))
    return t


def bfs(part: Partition, roots: Sequence[int], levels=None, parents=None, want_parents: bool = False,
        stream=None):
    """Levels [len(roots), V] int32 (TG_INF = unreachable); optionally parents."""
    r = _roots(roots)
    levels = _out(levels, (r.size, part.n), "int32")
    if want_parents:
        parents = _out(parents, (r.size, part.n), "int32")
    _check(_load().bfs(part.handle, r.ctypes.data_as(_c_i32p), r.size, levels.data_ptr(),
                       parents.data_ptr() if parents is not None else None, _stream_handle(stream)))
    return (levels, parents) if parents is not None else levels


def sssp(part: Partition, roots: Sequence[int], dist=None, stream=None):
    r = _roots(roots)
    dist = _out(dist, (r.size, part.n), "int32")
    _check(_load().sssp(part.handle, r.ctypes.data_as(_c_i32p), r.size, dist.data_ptr(), _stream_handle(stream)))
    return dist


def pagerank(part: Partition, damping: float = 0.85, iterations: int = 10, dangling: str = "uniform",
             rank=None, stream=None):
    rank = _out(rank, (part.n,), "float32")
    _check(_load().pagerank(part.handle, float(damping), int(iterations), DANGLING[dangling],
                            rank.data_ptr(), _stream_handle(stream)))
    return rank


def bc(part: Partition, sources: Sequence[int], scores=None, stream=None):
    s = _roots(sources)
    scores = _out(scores, (part.n,), "float32")
    _check(_load().bc(part.handle, s.ctypes.data_as(_c_i32p), s.size, scores.data_ptr(), _stream_handle(stream)))
    return scores


def cc(part: Partition, labels=None, stream=None):
    """Connected components: labels[v] = smallest original id in v's component
    (weak components of a directed graph)."""
    labels = _out(labels, (part.n,), "int32")
    _check(_load().cc(part.handle, labels.data_ptr(), _stream_handle(stream)))
    return labels


def bfs_batched(part: Partition, roots: Sequence[int], levels=None, stream=None):
    """bfs() for many roots through the 64-slot bitmask engine."""
    r = _roots(roots)
    levels = _out(levels, (r.size, part.n), "int32")
    _check(_load().bfs_batched(part.handle, r.ctypes.data_as(_c_i32p), r.size, levels.data_ptr(),
                               _stream_handle(stream)))
    return levels


def bc_batched(part: Partition, sources: Sequence[int], scores=None, stream=None):
    """bc() for many sources through the 64-source [vertex][source] layout."""
    s = _roots(sources)
    scores = _out(scores, (part.n,), "float32")
    _check(_load().bc_batched(part.handle, s.ctypes.data_as(_c_i32p), s.size, scores.data_ptr(),
                              _stream_handle(stream)))
    return scores


def bc_multi(parts: Sequence[Partition], sources: Sequence[Sequence[int]], scores=None, stream=None):
    """bc_batched() over several graphs in one call; returns one score tensor
    per graph."""
    lib = _load()
    k = len(parts)
    assert len(sources) == k
    srcs = [_roots(s) for s in sources]
    scores = [_out(None if scores is None else scores[i], (parts[i].n,), "float32") for i in range(k)]
    ph = (ctypes.c_void_p * k)(*[p.handle for p in parts])
    sp = (_c_i32p * k)(*[s.ctypes.data_as(_c_i32p) for s in srcs])
    ns = (ctypes.c_int32 * k)(*[s.size for s in srcs])
    op = (ctypes.c_void_p * k)(*[t.data_ptr() for t in scores])
    _check(lib.bc_multi(ph, k, sp, ns, op, _stream_handle(stream)))
    return scores


def sssp_batched(part: Partition, roots: Sequence[int], dist=None, stream=None):
    """sssp() for many roots through the 64-slot engine."""
    r = _roots(roots)
    dist = _out(dist, (r.size, part.n), "int32")
    _check(_load().sssp_batched(part.handle, r.ctypes.data_as(_c_i32p), r.size, dist.data_ptr(),
                                _stream_handle(stream)))
    return dist


TG_QUERY_BFS, TG_QUERY_SSSP = 0, 1


class Server:
    """Continuous-batching query server (server_* in the C ABI)."""

    def __init__(self, max_slots: int = 64, memory_cap_bytes: Optional[int] = None,
                 sssp_solo_min_vertices: Optional[int] = None,
                 sssp_solo_min_skew: Optional[float] = None):
        lib = _load()
        opts = {"max_slots": int(max_slots)}
        if memory_cap_bytes is not None:
            opts["memory_cap_bytes"] = int(memory_cap_bytes)
        if sssp_solo_min_vertices is not None:
            opts["sssp_solo_min_vertices"] = int(sssp_solo_min_vertices)
        if sssp_solo_min_skew is not None:
            opts["sssp_solo_min_skew"] = float(sssp_solo_min_skew)
        h = ctypes.c_void_p()
        _check(lib.server_create(json.dumps(opts).encode(), ctypes.byref(h)))
        self._h = h.value
        self._parts = []

    def add_graph(self, part: Partition) -> int:
        gid = ctypes.c_int32()
        _check(_load().server_add_graph(self._h, part.handle, ctypes.byref(gid)))
        self._parts.append(part)
        return gid.value

    def submit(self, graph_id: int, kind: int, root: int, out) -> int:
        t = ctypes.c_uint64()
        _check(_load().server_submit(self._h, graph_id, kind, int(root), out.data_ptr(), ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1) -> float:
        lat = ctypes.c_double()
        _check(_load().server_wait(self._h, ticket, int(timeout_us), ctypes.byref(lat)))
        return lat.value

    def stats(self) -> dict:
        lib = _load()
        n = lib.server_stats(self._h, None, 0)
        buf = ctypes.create_string_buffer(n + 1)
        lib.server_stats(self._h, buf, n + 1)
        return json.loads(buf.value.decode())

    def close(self):
        if self._h:
            _load().server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
