"""Kernels must not depend on LDS they did not write.

LDS keeps whatever the previous workgroup on a CU left there, so a kernel that read an LDS word
before writing it would see values from earlier kernels, or from earlier processes, and could
give wrong results only now and then (the register Jacobi once read the tracked norms of its
padding columns that way: finite leftovers were harmless, a NaN or a huge one froze a real
column).  Here every CU's LDS is filled with NaN, or with the largest finite double, before each
Trotter step and before the reverse sweep (testing aid of libgpeps_peaks.so, on the simulator's
stream), and the history and the gradient must be bit for bit those of a run without the fill.
"""

import ctypes
import json
import os
import sys

import numpy as np
import pytest

from heavyhex import make_workload

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")
PATTERNS = {"nan": 0x7FF8000000000000, "huge": 0x7FEFFFFFFFFFFFFF}
LDS_BYTES = 160 * 1024  # the whole LDS of a CU on gfx950
FILL_BLOCKS = 2048      # several workgroups per CU


def _say(msg):
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    path = os.path.join(ROOT, "paper_2309_15642_amd", "libgpeps_peaks.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: run __graft_entry__.build() first")
    pk = ctypes.CDLL(path)
    pk.gpeps_probe_fill_lds.argtypes = [ctypes.c_ulonglong, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    pk.gpeps_probe_fill_lds.restype = ctypes.c_int
    from paper_2309_15642_amd import simulator
    return simulator, pk


def _run(env, sim_args, steps, pattern, backward):
    """History (and gradient) of `steps` Trotter steps with the LDS filled before each step and
    before the reverse sweep (pattern None: no fill)."""
    sm, pk = env
    s = sm.Simulator(*sim_args[0], **sim_args[1])

    def fill():
        if pattern is not None:
            rc = pk.gpeps_probe_fill_lds(pattern, LDS_BYTES, FILL_BLOCKS, ctypes.c_void_p(s.stream.cuda_stream))
            assert rc == 0, f"LDS fill launch failed (hipError {rc})"

    for _ in range(steps):
        fill()
        s.step(1)
    (h,) = s.z_history()
    grad = None
    if backward:
        fill()
        dh, dj = s.backward([np.full(s.n_nodes_total, 1.0 / s.n_nodes_total)])
        grad = (float(dh[0]), float(dj[0]))
    s.close()
    return h, grad


def _check(env, label, sim_args, steps, backward):
    _say(f"{label}: clean run")
    h0, g0 = _run(env, sim_args, steps, None, backward)
    for name, pat in PATTERNS.items():
        _say(f"{label}: LDS filled with {name} before every step" + (" and the backward" if backward else ""))
        h, g = _run(env, sim_args, steps, pat, backward)
        assert np.array_equal(h, h0), f"history differs after an LDS fill ({name}): max {np.max(np.abs(h - h0)):.3e}"
        assert g == g0, f"gradient differs after an LDS fill ({name}): {g} against {g0}"
    return h0


@pytest.mark.parametrize("d", [16, 32])
def test_results_do_not_depend_on_lds_residue(env, d):
    """127 qubits, theta_h = 0.6, D = 16 or 32, 20 steps, complex64, adjoint context: forward
    history and gradient with every CU's LDS filled before each step equal the clean run bit for
    bit, and the loss matches the oracle."""
    gold = json.load(open(os.path.join(GOLDEN, f"oracle_grad_eagle127_d{d}.json")))
    w = make_workload(f"eagle127_grad_d{d}")
    args = (([w.graphs[0]], [0], [gold["theta_h"]], [gold["theta_j"]]),
            dict(d_max=w.d_max, precision=w.precision, trunc_rel=w.trunc_rel, max_steps=w.steps, adjoint=True))
    h0 = _check(env, f"eagle127_grad_d{d}", args, w.steps, True)
    assert abs(float(h0[-1].mean()) - gold["loss"]) < 1e-5


def test_big_bond_and_complex128_paths_do_not_depend_on_lds_residue(env):
    """The D = 64 kernel (127 qubits, theta_h = 0.7, 8 steps, complex64) and the complex128 path
    (127 qubits, theta_h = 0.6, D = 8, 6 steps): histories bit for bit equal with and without the
    LDS fill."""
    from heavyhex import eagle127
    w = make_workload("eagle127_d64_t20")
    i = w.instances[0]
    _check(env, "eagle127 D=64 8 steps",
           (([w.graphs[0]], [0], [i.theta_h], [i.theta_j]),
            dict(d_max=w.d_max, precision=w.precision, trunc_rel=w.trunc_rel, max_steps=8)), 8, False)
    _check(env, "eagle127 D=8 c128 6 steps",
           (([eagle127()], [0], [0.6], [i.theta_j]),
            dict(d_max=8, precision="c128", trunc_rel=1e-12, max_steps=6)), 6, False)


def test_stored_adjoint_and_bp_do_not_depend_on_lds_residue(env):
    """The stored-forward adjoint (cfg.adjoint = 2: the forward keeps every class's SVD data; 127
    qubits, theta_h = 0.6, D = 16, 20 steps) with the fill before each step and the reverse
    sweep, then belief propagation on the resulting state (30 iterations) with the fill before
    it: everything bit for bit equal to the clean run."""
    sm, pk = env
    gold = json.load(open(os.path.join(GOLDEN, "oracle_grad_eagle127_d16.json")))
    w = make_workload("eagle127_grad_d16")
    g = w.graphs[0]
    out = {}
    for name, pat in [("clean", None)] + list(PATTERNS.items()):
        _say(f"eagle127_grad_d16 stored adjoint + BP: {name}")
        s = sm.Simulator([g], [0], [gold["theta_h"]], [gold["theta_j"]], d_max=w.d_max, precision=w.precision,
                         trunc_rel=w.trunc_rel, max_steps=w.steps, adjoint=2)

        def fill():
            if pat is not None:
                rc = pk.gpeps_probe_fill_lds(pat, LDS_BYTES, FILL_BLOCKS, ctypes.c_void_p(s.stream.cuda_stream))
                assert rc == 0, f"LDS fill launch failed (hipError {rc})"

        for _ in range(w.steps):
            fill()
            s.step(1)
        (h,) = s.z_history()
        fill()
        dh, dj = s.backward([np.full(g.n_nodes, 1.0 / g.n_nodes)])
        fill()
        zb = np.asarray(s.bp_expect_z(30)[0]).copy()
        s.close()
        out[name] = (h, float(dh[0]), float(dj[0]), zb)
    h0, dh0, dj0, zb0 = out["clean"]
    for name in PATTERNS:
        h, dh, dj, zb = out[name]
        assert np.array_equal(h, h0) and dh == dh0 and dj == dj0, f"stored adjoint differs after an LDS fill ({name})"
        assert np.array_equal(zb, zb0), f"BP readout differs after an LDS fill ({name})"


@pytest.mark.parametrize("mode,svd_threads", [("batched", 64), ("plain", 256)])
def test_other_launch_shapes_do_not_depend_on_lds_residue(env, mode, svd_threads):
    """127 qubits, theta_h = 0.7, D = 16, 10 steps, complex64: the 64-thread SVD workgroups the
    autotuner may pick, and the plain (one launch per instance and class) mode, under the fill."""
    sm, pk = env
    w = make_workload("eagle127_d16")
    i = w.instances[0]
    out = {}
    for name, pat in [("clean", None)] + list(PATTERNS.items()):
        _say(f"eagle127_d16 {mode}, SVD {svd_threads} threads, 10 steps: {name}")
        s = sm.Simulator([w.graphs[0]], [0], [i.theta_h], [i.theta_j], d_max=w.d_max, precision=w.precision,
                         trunc_rel=w.trunc_rel, max_steps=10, mode=mode)
        s.set_tiles(8, 1, svd_threads)
        for _ in range(10):
            if pat is not None:
                rc = pk.gpeps_probe_fill_lds(pat, LDS_BYTES, FILL_BLOCKS, ctypes.c_void_p(s.stream.cuda_stream))
                assert rc == 0, f"LDS fill launch failed (hipError {rc})"
            s.step(1)
        (h,) = s.z_history()
        s.close()
        out[name] = h
    for name in PATTERNS:
        assert np.array_equal(out[name], out["clean"]), f"history differs after an LDS fill ({name})"
