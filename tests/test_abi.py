"""The C ABI library: it loads, exports every declared symbol, and validates
arguments on the host (no device work is started by these calls)."""

import ctypes
import os
import re

import numpy as np
import pytest

from heavyhex import eagle127, ring

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2309_15642_amd import _lib
    return _lib.load()


def test_header_symbols_exported(lib):
    hdr = open(os.path.join(ROOT, "include", "gpeps.h")).read()
    declared = set(re.findall(r"\b(gpeps_[a-z_]+)\s*\(", hdr))
    from paper_2309_15642_amd import _lib
    assert declared == set(_lib.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def _ws(lib, graphs, goi, **kw):
    from paper_2309_15642_amd import _lib
    keep = []
    arr = (_lib.gpeps_graph * len(graphs))()
    for k, (n, edges, colour) in enumerate(graphs):
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        keep.append(e)
        arr[k].n_nodes = n
        arr[k].n_edges = e.shape[0]
        arr[k].edges = e.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        if colour is not None:
            c = np.ascontiguousarray(np.asarray(colour, dtype=np.int32))
            keep.append(c)
            arr[k].colour = c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    cfg = _lib.gpeps_config()
    cfg.d_max = kw.get("d_max", 16)
    cfg.precision = kw.get("precision", 0)
    cfg.trunc_rel = kw.get("trunc_rel", 1e-6)
    cfg.max_jacobi_sweeps = 40
    cfg.max_steps = kw.get("max_steps", 20)
    cfg.mode = kw.get("mode", 0)
    cfg.adjoint = kw.get("adjoint", 0)
    g = np.asarray(goi, dtype=np.int32)
    out = ctypes.c_size_t(0)
    st = lib.gpeps_workspace_size(arr, len(graphs), g.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(g),
                                  ctypes.byref(cfg), ctypes.byref(out))
    return st, out.value, lib.gpeps_last_error(None).decode()


def test_workspace_size_eagle(lib):
    g = eagle127()
    st, nbytes, _ = _ws(lib, [(g.n_nodes, g.edges, g.colour)], [0], d_max=32)
    assert st == 0
    # site tensors alone: 36 degree-3, 89 degree-2, 2 degree-1 qubits, complex64, D = 32
    gamma = (36 * 2 * 32 ** 3 + 89 * 2 * 32 ** 2 + 2 * 2 * 32) * 8
    assert gamma < nbytes < 3 * gamma


def test_library_colouring_matches_given(lib):
    g = eagle127()
    a = _ws(lib, [(g.n_nodes, g.edges, None)], [0])
    b = _ws(lib, [(g.n_nodes, g.edges, g.colour)], [0])
    assert a[0] == 0 and b[0] == 0 and a[1] == b[1]


@pytest.mark.parametrize("case,msg", [
    ("self_loop", "self-loop"),
    ("duplicate", "duplicate"),
    ("range", "out of range"),
    ("improper", "not proper"),
    ("degree4", "degree"),
    ("d_max", "d_max"),
    ("odd_cycle", "bipartite"),
])
def test_argument_errors(lib, case, msg):
    r = ring(12)
    graphs = [(12, r.edges, r.colour)]
    kw = {}
    if case == "self_loop":
        graphs = [(3, [(0, 1), (1, 1)], None)]
    elif case == "duplicate":
        graphs = [(3, [(0, 1), (1, 0)], None)]
    elif case == "range":
        graphs = [(3, [(0, 1), (1, 5)], None)]
    elif case == "improper":
        graphs = [(3, [(0, 1), (1, 2)], [0, 0])]
    elif case == "degree4":
        graphs = [(5, [(0, 1), (0, 2), (0, 3), (0, 4)], None)]
    elif case == "d_max":
        kw = {"d_max": 65}
    elif case == "odd_cycle":
        graphs = [(3, [(0, 1), (1, 2), (0, 2)], None)]
    st, _, err = _ws(lib, graphs, [0], **kw)
    assert st == -1
    assert msg in err


def test_bad_instance_index(lib):
    r = ring(12)
    st, _, err = _ws(lib, [(12, r.edges, r.colour)], [1])
    assert st == -1 and "graph_of_instance" in err


def test_init_rejects_missing_workspace(lib):
    from paper_2309_15642_amd import _lib
    r = ring(12)
    e = np.ascontiguousarray(r.edges.astype(np.int32))
    c = np.ascontiguousarray(r.colour.astype(np.int32))
    g = _lib.gpeps_graph(12, 12, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    cfg = _lib.gpeps_config(4, 1, 1e-12, 40, 5, 0)
    goi = (ctypes.c_int32 * 1)(0)
    th = (ctypes.c_double * 1)(0.5)
    tj = (ctypes.c_double * 1)(-1.5707963267948966)
    ctx = ctypes.c_void_p(0)
    st = lib.gpeps_init(ctypes.byref(ctx), ctypes.byref(g), 1, goi, 1, th, tj, ctypes.byref(cfg), None, 0, None)
    assert st == -2 and not ctx.value
    assert "workspace" in lib.gpeps_last_error(None).decode()


def test_tuning_calls_reject_null_context(lib):
    tiles = (ctypes.c_int32 * 3)(16, 2, 256)
    assert lib.gpeps_set_tiles(None, tiles) == -1
    assert lib.gpeps_autotune(None, 4, tiles) == -1
    assert "ctx is NULL" in lib.gpeps_last_error(None).decode()


def test_adjoint_modes_workspace(lib):
    """cfg.adjoint: 1 adds checkpoints and one set of per-class buffers; 2 keeps the per-class
    state and buffers of every step, so its extra size grows with max_steps; 3 is rejected."""
    g = eagle127()
    spec = [(g.n_nodes, g.edges, g.colour)]
    sizes = {}
    for adj in (0, 1, 2):
        for steps in (10, 20):
            st, n, _ = _ws(lib, spec, [0], adjoint=adj, max_steps=steps)
            assert st == 0
            sizes[(adj, steps)] = n
    grow = {adj: sizes[(adj, 20)] - sizes[(adj, 10)] for adj in (0, 1, 2)}
    assert sizes[(1, 20)] > sizes[(0, 20)] and sizes[(2, 20)] > sizes[(1, 20)]
    # one more step: a history row (0); plus a checkpoint (1); plus 3 class snapshots and buffers (2)
    assert grow[0] < grow[1] < grow[2]
    assert grow[2] - grow[1] > 10 * 3 * (g.n_nodes * 2 * 8)
    st, _, msg = _ws(lib, spec, [0], adjoint=3)
    assert st != 0 and "adjoint" in msg


def test_layer_kind_validation_without_context(lib):
    """Unknown layer kinds and a NULL context are errors before any device work."""
    assert lib.gpeps_apply_layer(None, 2, 1) != 0
    assert lib.gpeps_apply_layer(None, 7, 1) != 0
    assert lib.gpeps_bp_expect_z(None, 1, None, 0, None) != 0


def test_bond_cap_rules(lib):
    """d_max up to 64; above 32 the adjoint is refused and the cutoff must be >= 1e-10; 65 is refused."""
    g = eagle127()
    graphs = [(g.n_nodes, g.edges, g.colour)]
    st, n64, _ = _ws(lib, graphs, [0], d_max=64)
    st16, n16, _ = _ws(lib, graphs, [0], d_max=16)
    assert st == 0 and st16 == 0 and n64 > n16
    for kw, word in ((dict(d_max=65), "d_max"), (dict(d_max=64, adjoint=1), "adjoint"),
                     (dict(d_max=40, trunc_rel=1e-12), "trunc_rel")):
        st, _, msg = _ws(lib, graphs, [0], **kw)
        assert st == -1 and word in msg, (kw, msg)
    st, _, _ = _ws(lib, graphs, [0], d_max=32, trunc_rel=1e-12, adjoint=1)
    assert st == 0


def test_measurement_library_exports_and_validates():
    """libgpeps_peaks.so (peak-rate probes for the benchmark and the LDS fill the LDS-residue GPU
    test uses) loads and exports its entry points; the LDS fill rejects bad sizes on the host,
    before any HIP call."""
    path = os.path.join(ROOT, "paper_2309_15642_amd", "libgpeps_peaks.so")
    pk = ctypes.CDLL(path)
    for name in ("gpeps_peak_fma_f64", "gpeps_peak_mfma_f64", "gpeps_peak_copy", "gpeps_probe_fill_lds"):
        assert hasattr(pk, name), name
    pk.gpeps_probe_fill_lds.argtypes = [ctypes.c_ulonglong, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    pk.gpeps_probe_fill_lds.restype = ctypes.c_int
    invalid_value = 1  # hipErrorInvalidValue
    assert pk.gpeps_probe_fill_lds(0, 4, 1, None) == invalid_value    # fewer than 8 bytes
    assert pk.gpeps_probe_fill_lds(0, 1001, 1, None) == invalid_value  # not a multiple of 8
    assert pk.gpeps_probe_fill_lds(0, 1024, 0, None) == invalid_value  # no workgroup
