"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/tg.h declares, and rejects malformed graphs."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import graphgen
import paper_1312_3018_amd as tg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "tg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w \*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_library_exports_every_declared_symbol():
    lib = tg.require_native()
    names = declared_functions()
    assert {"graph_load_csr", "partition_by_degree", "bfs", "sssp", "pagerank", "bc"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", tg.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines())
    assert set(names) <= exported


def _load(n, off, col, w=None, symmetric=False):
    return tg.graph_load_csr(n, np.asarray(off, dtype=np.int64), np.asarray(col, dtype=np.int32),
                             None if w is None else np.asarray(w, dtype=np.int32), symmetric=symmetric)


def test_load_valid_graph_on_host():
    g = graphgen.rmat(8)
    G = tg.graph_load_csr(g.n, g.offsets, g.cols, graphgen.weights(g), symmetric=True)
    assert G.n == g.n and G.m == g.nnz
    G.free()


@pytest.mark.parametrize("off,col,msg", [
    ([0, 2, 1, 3], [1, 2, 0], "decrease"),
    ([1, 2, 3, 3], [1, 2, 0], "row_offsets[0]"),
    ([0, 1, 2, 4], [1, 2, 0], "num_edges"),
    ([0, 1, 2, 3], [1, 3, 0], "out of range"),
    ([0, 1, 2, 3], [1, -1, 0], "out of range"),
])
def test_malformed_csr_is_rejected(off, col, msg):
    with pytest.raises(tg.TGError) as ei:
        _load(3, off, col)
    assert ei.value.code == tg.TG_EINVAL
    assert msg in str(ei.value)


def test_bad_weights_and_false_symmetry_rejected():
    with pytest.raises(tg.TGError) as ei:
        _load(2, [0, 1, 2], [1, 0], w=[3, 0])
    assert ei.value.code == tg.TG_EINVAL
    with pytest.raises(tg.TGError) as ei:
        _load(3, [0, 1, 1, 1], [1], symmetric=True)
    assert "symmetric" in str(ei.value)
    with pytest.raises(tg.TGError):
        _load(2, [0, 1, 2], [1, 0], w=[3, 4], symmetric=True)  # unequal reverse weight


def test_sizes_checked():
    lib = tg.require_native()
    out = ctypes.c_void_p()
    assert lib.graph_load_csr(-1, 0, None, None, None, 0, None, ctypes.byref(out)) == tg.TG_EINVAL
    assert lib.graph_load_csr(2**31, 0, None, None, None, 0, None, ctypes.byref(out)) == tg.TG_EINVAL
    assert lib.graph_load_csr(1, 0, None, None, None, 0, None, ctypes.byref(out)) == tg.TG_EINVAL
    assert "row_offsets is NULL" in tg.tg_last_error()


@pytest.mark.parametrize("opts", ['{"max_slots": 0}', '{"max_slots": 65}', '{"memory_cap_bytes": -1}',
                                  '{"sssp_solo_min_vertices": -1}', '{"sssp_solo_min_skew": -0.5}'])
def test_server_options_checked_on_host(opts):
    """server_create rejects out-of-range options before it touches a device."""
    lib = tg._load()
    h = ctypes.c_void_p()
    assert lib.server_create(opts.encode(), ctypes.byref(h)) == tg.TG_EINVAL
    assert not h.value
