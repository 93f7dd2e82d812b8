"""GPU adjoint (gpeps_backward through the C ABI) against the oracle gradient.

The loss is the mean <Z> after the last step; the reference is oracle/grad.py (its own
reverse sweep, pinned to finite differences in tests/test_oracle_grad.py).
"""

import json
import math
import os
import sys

import numpy as np
import pytest

from heavyhex import eagle127, make_workload, ring
from oracle import grad as G

pytestmark = pytest.mark.gpu
TJ = -math.pi / 2
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


def _gpu_grad(sim_mod, g, th, tj, d, prec, eps, steps):
    s = sim_mod.Simulator([g], [0], [th], [tj], d_max=d, precision=prec, trunc_rel=eps, max_steps=steps,
                          adjoint=True)
    s.step(steps)
    (h,) = s.z_history()
    # printed for the record of a failing case: where the forward left the expected trajectory
    print(f"forward: mean <Z> per step {np.round(h.mean(axis=1), 8).tolist()}; stats {s.stats()}", flush=True)
    dh, dj = s.backward([np.full(g.n_nodes, 1.0 / g.n_nodes)])
    s.close()
    return float(h[-1].mean()), float(dh[0]), float(dj[0])


def test_ring12_c128_gradient(sim_mod):
    _say("ring12 D=4 c128 5 steps gradient")
    g = ring(12)
    loss, dh, dj = _gpu_grad(sim_mod, g, 0.5, -1.2, 4, "c128", 1e-12, 5)
    r = G.loss_and_grad_graph(g, 0.5, -1.2, 4, 5, 1e-12)
    print(f"gpu {dh:.12f} {dj:.12f} oracle {r.dtheta_h:.12f} {r.dtheta_j:.12f}")
    assert abs(loss - r.loss) < 1e-12
    assert abs(dh - r.dtheta_h) < 1e-8 and abs(dj - r.dtheta_j) < 1e-8


@pytest.mark.parametrize("prec,tol", [("c128", 1e-8), ("c64", 2e-5)])
def test_eagle_d4_gradient(sim_mod, prec, tol):
    _say(f"eagle127 D=4 {prec} 5 steps gradient")
    g = eagle127()
    eps = 1e-12 if prec == "c128" else 1e-6
    loss, dh, dj = _gpu_grad(sim_mod, g, 0.6, TJ, 4, prec, eps, 5)
    r = G.loss_and_grad_graph(g, 0.6, TJ, 4, 5, eps)
    print(f"gpu {dh:.10f} {dj:.10f} oracle {r.dtheta_h:.10f} {r.dtheta_j:.10f}")
    assert abs(dh - r.dtheta_h) < tol and abs(dj - r.dtheta_j) < tol


@pytest.mark.parametrize("prec,tol", [("c128", 1e-8), ("c64", 2e-5)])
def test_ring12_d32_gradient(sim_mod, prec, tol):
    """D = 32: the row kernel of the edge adjoint takes more than 64 KB of dynamic LDS here.

    theta_h = 1.1, theta_J = -1.4, 7 steps: bonds reach the cap of 32 and every cut keeps a gap
    of at least 1.6e-3 s_0 (a near-degenerate cut would amplify rounding by 1 / gap).
    """
    _say(f"ring12 D=32 {prec} 7 steps gradient")
    g = ring(12)
    eps = 1e-12 if prec == "c128" else 1e-6
    loss, dh, dj = _gpu_grad(sim_mod, g, 1.1, -1.4, 32, prec, eps, 7)
    r = G.loss_and_grad_graph(g, 1.1, -1.4, 32, 7, eps)
    print(f"gpu {dh:.10f} {dj:.10f} oracle {r.dtheta_h:.10f} {r.dtheta_j:.10f}")
    assert abs(dh - r.dtheta_h) < tol and abs(dj - r.dtheta_j) < tol


def test_gradient_zeros_and_closed_form(sim_mod):
    g = eagle127()
    _say("eagle127 theta_h=0 gradient zeros")
    loss, dh, dj = _gpu_grad(sim_mod, g, 0.0, TJ, 8, "c64", 1e-6, 4)
    assert loss == 1.0 and np.isfinite(dh) and np.isfinite(dj)
    assert abs(dh) < 1e-12 and abs(dj) < 1e-12
    _say("eagle127 theta_J=0 closed form")
    loss, dh, dj = _gpu_grad(sim_mod, g, 0.37, 0.0, 4, "c128", 1e-12, 5)
    assert abs(dh + 5 * math.sin(5 * 0.37)) < 1e-10
    assert abs(dj) < 1e-10


def test_autograd_function(sim_mod):
    import torch
    from paper_2309_15642_amd.autograd import GpepsMeanZ
    _say("autograd.Function ring12 + eagle127 batch")
    gs = [ring(12), eagle127()]
    sim = sim_mod.Simulator(gs, [0, 1], [0.4, 0.8], [TJ, TJ], d_max=4, precision="c128", trunc_rel=1e-12,
                            max_steps=4, adjoint=True)
    th = torch.tensor([0.5, 0.6], dtype=torch.float64, requires_grad=True)
    tj = torch.tensor([-1.2, TJ], dtype=torch.float64, requires_grad=True)
    m = GpepsMeanZ.apply(th, tj, sim, 4)
    (m[0] + 2.0 * m[1]).backward()
    sim.close()
    for k, (g, w) in enumerate(zip(gs, (1.0, 2.0))):
        r = G.loss_and_grad_graph(g, float(th[k]), float(tj[k]), 4, 4, 1e-12)
        assert abs(float(m[k]) - r.loss) < 1e-12
        assert abs(float(th.grad[k]) - w * r.dtheta_h) < 1e-8
        assert abs(float(tj.grad[k]) - w * r.dtheta_j) < 1e-8


@pytest.mark.parametrize("d", [16, 32])
def test_grad_workload_full(sim_mod, d):
    """127 qubits, theta_h = 0.6, D = 16 or 32, 20 steps, complex64 + float64 QR/SVD: the adjoint
    workloads."""
    gold = json.load(open(os.path.join(GOLDEN, f"oracle_grad_eagle127_d{d}.json")))
    w = make_workload(f"eagle127_grad_d{d}")
    _say(f"eagle127_grad_d{d} full gradient")
    loss, dh, dj = _gpu_grad(sim_mod, w.graphs[0], gold["theta_h"], gold["theta_j"], w.d_max, w.precision,
                             w.trunc_rel, w.steps)
    print(f"gpu loss {loss:.10f} dh {dh:.8f} dj {dj:.8f}; oracle {gold['loss']:.10f} {gold['dtheta_h']:.8f} "
          f"{gold['dtheta_j']:.8f}; fd {gold['fd_dtheta_h']:.8f} {gold['fd_dtheta_j']:.8f}")
    assert abs(loss - gold["loss"]) < 1e-5
    # the complex64 state limits the forward to ~1e-6; the adjoint matches the oracle to ~1e-6
    # relative, independently of how the forward SVD resolved noise-level singular values
    assert abs(dh - gold["dtheta_h"]) < 2e-5 * max(1.0, abs(gold["dtheta_h"]))
    assert abs(dj - gold["dtheta_j"]) < 2e-5 * max(1.0, abs(gold["dtheta_j"]))


@pytest.mark.parametrize("name,prec,d,steps,mode", [("eagle127", "c128", 4, 4, "batched"),
                                                    ("ring12", "c128", 4, 6, "plain"),
                                                    ("eagle127", "c64", 16, 20, "batched")])
def test_stored_forward_adjoint_equals_recompute(sim_mod, name, prec, d, steps, mode):
    """cfg.adjoint = 2 (the forward keeps every class's state and SVD data) gives the same
    gradient as cfg.adjoint = 1 (the backward recomputes each step) bit for bit: the recompute
    follows the forward path, and every reduction of the reverse sweep runs in a fixed order.  A
    second backward of the same forward gives the same bits again.  The forward history is bit for
    bit that of a context without the adjoint."""
    from heavyhex import eagle127, ring
    g = eagle127() if name == "eagle127" else ring(12)
    th = 0.6
    dl = [np.full(g.n_nodes, 1.0 / g.n_nodes)]
    _say(f"{name} D={d} {prec} {steps} steps {mode}: adjoint 0 / 1 / 2")
    out = {}
    for adj in (0, 1, 2):
        s = sim_mod.Simulator([g], [0], [th], [TJ], d_max=d, precision=prec, trunc_rel=1e-6 if prec == "c64" else 1e-12,
                              max_steps=steps, mode=mode, adjoint=adj)
        s.step(steps)
        (h,) = s.z_history()
        grad = s.backward(dl) if adj else None
        again = s.backward(dl) if adj else None
        s.close()
        if adj:
            assert np.array_equal(grad[0], again[0]) and np.array_equal(grad[1], again[1])
        out[adj] = (h, grad)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][0], out[2][0])
    (h1, (gh1, gj1)), (h2, (gh2, gj2)) = out[1], out[2]
    print(f"d/dtheta_h {gh1[0]:.17e} {gh2[0]:.17e}  d/dtheta_J {gj1[0]:.17e} {gj2[0]:.17e}")
    assert gh1[0] == gh2[0] and gj1[0] == gj2[0]


def test_mean_z_and_its_backward_through_the_abi(sim_mod):
    """gpeps_mean_z is the mean of the last history row of every instance, and
    gpeps_backward_mean_z (seed formed on the device) equals gpeps_backward with dl_dz = w_k / n_k."""
    _say("ring12 + eagle127 D=4 c128 4 steps: gpeps_mean_z, gpeps_backward_mean_z")
    gs = [ring(12), eagle127()]
    s = sim_mod.Simulator(gs, [0, 1], [0.5, 0.7], [-1.1, TJ], d_max=4, precision="c128", trunc_rel=1e-12,
                          max_steps=4, adjoint=True)
    s.step(4)
    hist = s.z_history()
    m = s.mean_z()
    assert abs(m[0] - hist[0][-1].mean()) < 1e-15 and abs(m[1] - hist[1][-1].mean()) < 1e-15
    w = np.array([0.3, -1.7])
    dh1, dj1 = s.backward([np.full(g.n_nodes, w[k] / g.n_nodes) for k, g in enumerate(gs)])
    dh2, dj2 = s.backward_mean_z(w)
    s.close()
    assert np.allclose(dh1, dh2, rtol=1e-12, atol=1e-15) and np.allclose(dj1, dj2, rtol=1e-12, atol=1e-15)
    for k, g in enumerate(gs):
        r = G.loss_and_grad_graph(g, [0.5, 0.7][k], [-1.1, TJ][k], 4, 4, 1e-12)
        assert abs(dh2[k] - w[k] * r.dtheta_h) < 1e-8 and abs(dj2[k] - w[k] * r.dtheta_j) < 1e-8


def test_adjoint_context_rejects_unrecorded_changes(sim_mod):
    """With cfg.adjoint set, the single RX / RZZ layers (not checkpointed), and set_angles or
    set_tiles once a step is recorded, fail with GPEPS_ERR_STATE; after a reset they work."""
    from paper_2309_15642_amd._lib import GpepsError
    _say("eagle127 D=4 c128 adjoint context: layer, set_angles and set_tiles rejections")
    g = eagle127()
    s = sim_mod.Simulator([g], [0], [0.6], [TJ], d_max=4, precision="c128", trunc_rel=1e-12, max_steps=3,
                          adjoint=True)
    for call in (s.rx_layer, s.rzz_layer):
        with pytest.raises(GpepsError) as ei:
            call()
        assert ei.value.status == -5
    s.step(2)
    with pytest.raises(GpepsError) as ei:
        s.set_angles([0.7], [TJ])
    assert ei.value.status == -5 and "reset" in str(ei.value)
    with pytest.raises(GpepsError) as ei:
        s.set_tiles(16, 2, 256)
    assert ei.value.status == -5
    # the recorded evolution is untouched: its gradient is still the oracle's at theta_h = 0.6
    dh, dj = s.backward([np.full(g.n_nodes, 1.0 / g.n_nodes)])
    r = G.loss_and_grad_graph(g, 0.6, TJ, 4, 2, 1e-12)
    assert abs(dh[0] - r.dtheta_h) < 1e-8 and abs(dj[0] - r.dtheta_j) < 1e-8
    s.reset()
    s.set_angles([0.7], [TJ])
    s.set_tiles(16, 2, 256)
    s.step(1)
    s.close()


def test_autograd_refuses_a_stale_forward(sim_mod):
    """Two forwards on one simulator before backward: the first term's gradient is gone, so its
    backward raises instead of returning the gradient of the last forward."""
    import torch
    from paper_2309_15642_amd.autograd import GpepsMeanZ
    _say("autograd: two forwards on one simulator")
    g = ring(12)
    sim = sim_mod.Simulator([g], [0], [0.4], [TJ], d_max=4, precision="c128", trunc_rel=1e-12, max_steps=3,
                            adjoint=True)
    a = torch.tensor([0.5], dtype=torch.float64, requires_grad=True)
    b = torch.tensor([0.9], dtype=torch.float64, requires_grad=True)
    tj = torch.tensor([TJ], dtype=torch.float64)
    loss = GpepsMeanZ.apply(a, tj, sim, 3).sum() + GpepsMeanZ.apply(b, tj, sim, 3).sum()
    with pytest.raises(RuntimeError, match="changed after this forward"):
        loss.backward()
    sim.close()


def test_jacobi_cap_reports_numeric_error(sim_mod):
    """The device status word's failure path: with one Jacobi sweep allowed, SVDs of the
    20-step D = 16 workload stop unconverged; every kernel still exits normally, the next
    synchronising call returns GPEPS_ERR_NUMERIC naming Jacobi, and stats count the SVDs."""
    from paper_2309_15642_amd._lib import GpepsError
    w = make_workload("eagle127_d16")
    _say("eagle127_d16 with max_jacobi_sweeps = 1: GPEPS_ERR_NUMERIC expected")
    s = sim_mod.from_workload(w, max_jacobi_sweeps=1)
    s.step(w.steps)
    with pytest.raises(GpepsError) as ei:
        s.sync()
    assert ei.value.status == -4 and "jacobi" in str(ei.value).lower()
    st = s.stats()
    assert st["not_converged"] > 0 and st["max_sweeps"] == 1
    s.reset()
    s.close()
