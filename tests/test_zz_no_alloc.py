"""gpeps_bp_expect_z_noalloc (BP messages in the library's device array, no allocation) against
gpeps_bp_expect_z (messages in the caller's workspace), through the C ABI: two calls in a row,
the second on a smaller input, each bit for bit equal to the workspace call; and the size limit."""

import ctypes
import math
import sys

import numpy as np
import pytest

from heavyhex import eagle127, ring

pytestmark = pytest.mark.gpu
TJ = -math.pi / 2


def _say(msg):
    print(f"[gpu case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sim_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2309_15642_amd import simulator
    return simulator


def _bp(sim, fn, iters):
    out = np.empty(sim.n_nodes_total, dtype=np.float64)
    res = ctypes.c_double(-1.0)
    st = fn(sim.ctx, int(iters), ctypes.c_void_p(out.ctypes.data), 0, ctypes.byref(res))
    return st, out, res.value


def _compare(sim_mod, graphs, goi, th, d, prec, steps, iters):
    s = sim_mod.Simulator(graphs, goi, th, [TJ] * len(th), d_max=d, precision=prec,
                          trunc_rel=1e-6 if prec == "c64" else 1e-12, max_steps=steps)
    s.step(steps)
    lib = s.lib
    st_a, za, ra = _bp(s, lib.gpeps_bp_expect_z_noalloc, iters)
    st_b, zb, rb = _bp(s, lib.gpeps_bp_expect_z, iters)
    s.close()
    assert st_a == 0 and st_b == 0
    print(f"max |z_noalloc - z_workspace| = {np.max(np.abs(za - zb)):.1e}, residuals {ra:.3e} {rb:.3e}")
    assert np.array_equal(za, zb) and ra == rb
    return za


def test_noalloc_equals_workspace_call_twice_shrinking(sim_mod):
    _say("bp noalloc: eagle127 x 2 D=16 c64 8 steps, 20 iterations; then ring12 D=4 c128 5 steps, 6 iterations")
    _compare(sim_mod, [eagle127()], [0, 0], [0.7, 1.1], 16, "c64", 8, 20)
    _compare(sim_mod, [ring(12)], [0], [0.5], 4, "c128", 5, 6)


def test_noalloc_rejects_oversized_input(sim_mod):
    """8 instances of the 127-qubit graph at D = 32 need 4 * 1152 * 32^2 * 16 B = 72 MiB of
    messages, more than the 64 MiB array: GPEPS_ERR_ARG, no device work."""
    _say("bp noalloc: eagle127 x 8 D=32 must be rejected")
    s = sim_mod.Simulator([eagle127()], [0] * 8, [0.5] * 8, [TJ] * 8, d_max=32, precision="c64",
                          trunc_rel=1e-6, max_steps=1)
    st, _, _ = _bp(s, s.lib.gpeps_bp_expect_z_noalloc, 1)
    msg = s.lib.gpeps_last_error(s.ctx).decode()
    s.close()
    assert st == -1 and "scratch" in msg
