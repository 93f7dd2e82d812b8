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


def _run(env, d, pattern):
    sm, pk = env
    gold = json.load(open(os.path.join(GOLDEN, f"oracle_grad_eagle127_d{d}.json")))
    w = make_workload(f"eagle127_grad_d{d}")
    g = w.graphs[0]
    s = sm.Simulator([g], [0], [gold["theta_h"]], [gold["theta_j"]], d_max=w.d_max, precision=w.precision,
                     trunc_rel=w.trunc_rel, max_steps=w.steps, adjoint=True)

    def fill():
        if pattern is not None:
            rc = pk.gpeps_probe_fill_lds(pattern, LDS_BYTES, FILL_BLOCKS, ctypes.c_void_p(s.stream.cuda_stream))
            assert rc == 0, f"LDS fill launch failed (hipError {rc})"

    for _ in range(w.steps):
        fill()
        s.step(1)
    (h,) = s.z_history()
    fill()
    dh, dj = s.backward([np.full(g.n_nodes, 1.0 / g.n_nodes)])
    s.close()
    return h, float(dh[0]), float(dj[0]), gold


@pytest.mark.parametrize("d", [16, 32])
def test_results_do_not_depend_on_lds_residue(env, d):
    """127 qubits, theta_h = 0.6, D = 16 or 32, 20 steps, complex64: forward history and
    gradient with every CU's LDS filled before each step equal the clean run bit for bit, and
    the loss matches the oracle."""
    _say(f"eagle127_grad_d{d}: clean run")
    h0, dh0, dj0, gold = _run(env, d, None)
    assert abs(float(h0[-1].mean()) - gold["loss"]) < 1e-5
    for name, pat in PATTERNS.items():
        _say(f"eagle127_grad_d{d}: LDS filled with {name} before every step and the backward")
        h, dh, dj, _ = _run(env, d, pat)
        assert np.array_equal(h, h0), f"history differs after an LDS fill ({name}): max {np.max(np.abs(h - h0)):.3e}"
        assert dh == dh0 and dj == dj0, f"gradient differs after an LDS fill ({name})"
