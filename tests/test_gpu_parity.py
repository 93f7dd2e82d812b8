"""GPU path (libgpeps through its C ABI) against the FP64 oracle.

Tolerances (absolute, on every <Z_v> of every recorded step):
  complex128 path: 1e-10; complex64 storage with float64 QR/SVD: 1e-5.
Every test prints the case it is about to run, so a failing run names it.
"""

import math
import sys

import numpy as np
import pytest

import oracle.su as su
from exactref import lightcone_z
from heavyhex import eagle127, make_workload, ring

pytestmark = pytest.mark.gpu
TJ = -math.pi / 2
TOL = {"c128": 1e-10, "c64": 1e-5}


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


def _run(sim_mod, graphs, goi, ths, tjs, d, prec, eps, steps, mode="batched"):
    s = sim_mod.Simulator(graphs, goi, ths, tjs, d_max=d, precision=prec, trunc_rel=eps, max_steps=steps, mode=mode)
    s.step(steps)
    hist = s.z_history()
    dims = s.bond_dims()
    s.close()
    return hist, dims


def test_ring12_c128_config(sim_mod):
    w = make_workload("ring12_d4_c128")
    g = w.graphs[0]
    for mode in ("batched", "plain"):
        _say(f"ring12 D=4 c128 5 steps {mode}")
        (h,), _ = _run(sim_mod, [g], [0], [0.5], [TJ], 4, "c128", w.trunc_rel, 5, mode)
        ref = su.evolve_graph(g, 0.5, TJ, 4, 5, w.trunc_rel).z
        assert np.max(np.abs(h - ref)) < TOL["c128"]


def test_theta_h_zero_exact_one(sim_mod):
    g = eagle127()
    _say("eagle127 theta_h=0 D=16 c64 6 steps")
    (h,), (dims,) = _run(sim_mod, [g], [0], [0.0], [TJ], 16, "c64", 1e-6, 6)
    assert np.all(h == 1.0)
    assert np.all(dims == 1)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_eagle_d8_truncating(sim_mod, prec):
    g = eagle127()
    eps = 1e-12 if prec == "c128" else 1e-6
    _say(f"eagle127 D=8 {prec} 8 steps theta_h=0.7")
    (h,), (dims,) = _run(sim_mod, [g], [0], [0.7], [TJ], 8, prec, eps, 8)
    tr = su.evolve_graph(g, 0.7, TJ, 8, 8, eps)
    assert np.max(np.abs(h - tr.z)) < TOL[prec]
    if prec == "c128":
        assert np.array_equal(dims, tr.bond_dims[-1])


def test_eagle_d32_c64_truncating(sim_mod):
    """D = 32, complex64 storage: the 256-thread SVD path with QR preconditioning; truncation from t = 6."""
    g = eagle127()
    _say("eagle127 D=32 c64 7 steps theta_h=1.0")
    (h,), _ = _run(sim_mod, [g], [0], [1.0], [TJ], 32, "c64", 1e-6, 7)
    tr = su.evolve_graph(g, 1.0, TJ, 32, 7, 1e-6)
    assert np.max(np.abs(h - tr.z)) < TOL["c64"]


def test_lightcone_exact_t5_d32_c128(sim_mod):
    g = eagle127()
    _say("eagle127 D=32 c128 5 steps theta_h=0.9 vs light cone")
    (h,), _ = _run(sim_mod, [g], [0], [0.9], [TJ], 32, "c128", 1e-12, 5)
    for s in (62, 13, 58, 0):
        assert abs(h[4, s] - lightcone_z(g.n_nodes, g.edges, s, 0.9, TJ, 5)) < 1e-12


def test_batched_equals_plain_bitwise(sim_mod):
    g = eagle127()
    _say("eagle127 D=8 c64 4 steps batched vs plain")
    (hb,), _ = _run(sim_mod, [g], [0], [0.8], [TJ], 8, "c64", 1e-6, 4, "batched")
    (hp,), _ = _run(sim_mod, [g], [0], [0.8], [TJ], 8, "c64", 1e-6, 4, "plain")
    assert np.array_equal(hb, hp)


def test_mixed_batch_instances(sim_mod):
    """Graphs of different size and colour count in one batch; each instance matches its own oracle."""
    gs = [ring(12), eagle127()]
    goi = [1, 0, 1]
    ths = [0.3, 0.5, 1.2]
    _say("mixed batch ring12 + 2 x eagle127, D=8 c128 6 steps")
    hs, _ = _run(sim_mod, gs, goi, ths, [TJ] * 3, 8, "c128", 1e-12, 6)
    for h, gi, th in zip(hs, goi, ths):
        ref = su.evolve_graph(gs[gi], th, TJ, 8, 6, 1e-12).z
        assert np.max(np.abs(h - ref)) < TOL["c128"]


def test_eagle_d16_config_full(sim_mod):
    """127 qubits, theta_h = 0.7, D = 16, complex64 + float64 QR/SVD, 20 steps (the D=16 workload)."""
    w = make_workload("eagle127_d16")
    _say("eagle127_d16 full 20 steps batched")
    (h,), _ = _run(sim_mod, w.graphs, [0], [0.7], [TJ], 16, "c64", w.trunc_rel, 20)
    tr = su.evolve_graph(w.graphs[0], 0.7, TJ, 16, 20, w.trunc_rel)
    err = np.max(np.abs(h - tr.z), axis=1)
    print("max |dZ| per step:", " ".join(f"{x:.1e}" for x in err))
    assert err.max() < TOL["c64"]


@pytest.mark.parametrize("prec,mode", [("c128", "batched"), ("c64", "batched"), ("c64", "plain")])
def test_inverse_steps_undo_forward(sim_mod, prec, mode):
    """Three steps of U(0.9), then three of U(0.9)^dagger: every row matches the oracle and the
    state is back at |0...0> (nothing is truncated at bond dimension <= 8).

    On the way back the bonds shrink: singular values that are exactly zero come out at the
    storage rounding level, ~1e-7 of the largest in complex64, and the re-absorb divides by
    them.  The complex64 run therefore uses the 1e-6 relative cutoff of the complex64 workloads,
    which drops them; the complex128 run keeps the 1e-12 cutoff."""
    g = eagle127()
    eps = 1e-12 if prec == "c128" else 1e-6
    _say(f"eagle127 D=16 {prec} {mode}: 3 steps + 3 inverse steps at theta_h=0.9, cutoff {eps}")
    s = sim_mod.Simulator([g], [0], [0.9], [TJ], d_max=16, precision=prec, trunc_rel=eps, max_steps=6, mode=mode)
    s.step(3)
    s.step_inverse(3)
    (h,) = s.z_history()
    s.close()
    ref = su.evolve_graph(g, 0.9, TJ, 16, 3, eps, inverse_steps=3, theta_h_inverse=0.9).z
    assert np.max(np.abs(h - ref)) < TOL[prec]
    assert np.max(np.abs(h[-1] - 1.0)) < TOL[prec]


def test_weight_observable_lightcone_instance(sim_mod):
    """One instance of Appendix B at D = 32 in complex128: 5 steps at theta_h = 0.8, then
    5 steps of U(pi/2)^dagger, every row against the oracle; a second instance in the same
    batch with other angles checks that set_angles reaches both parameter arrays."""
    g = eagle127()
    _say("eagle127 D=32 c128: 5 steps at theta_h=0.8 / 0.3, set_angles(pi/2), 5 inverse steps")
    s = sim_mod.Simulator([g], [0, 0], [0.8, 0.3], [TJ, TJ], d_max=32, precision="c128", trunc_rel=1e-6,
                          max_steps=10)
    s.step(5)
    s.set_angles([math.pi / 2] * 2, [TJ] * 2)
    s.step_inverse(5)
    hs = s.z_history()
    s.close()
    for h, th in zip(hs, (0.8, 0.3)):
        tr = su.evolve_graph(g, th, TJ, 32, 5, 1e-6, inverse_steps=5)
        err = np.max(np.abs(h - tr.z), axis=1)
        print(f"theta_h={th} max |dZ| per row:", " ".join(f"{x:.1e}" for x in err),
              f"min cut gap {tr.min_cut_gap.min():.1e}")
        assert err.max() < 1e-10


def test_inverse_step_rejected_with_adjoint(sim_mod):
    """The adjoint covers forward steps only: an inverse step on an adjoint context is an error."""
    g = ring(12)
    _say("ring12 D=4 adjoint context: GPEPS_STEP_INVERSE must fail")
    s = sim_mod.Simulator([g], [0], [0.5], [TJ], d_max=4, precision="c128", trunc_rel=1e-12, max_steps=4,
                          adjoint=True)
    s.step(1)
    with pytest.raises(RuntimeError, match="adjoint"):
        s.step_inverse(1)
    s.close()


def test_cell10_batched_equals_plain_bitwise(sim_mod):
    """The periodic unit cell (wrapped links) through both launch configurations, forward and
    inverse steps: bit-identical histories."""
    from heavyhex import heavy_hex_cell10
    g = heavy_hex_cell10()
    hs = []
    for mode in ("batched", "plain"):
        _say(f"cell10 x 3 instances D=16 c64 {mode}: 6 steps + 2 inverse steps")
        s = sim_mod.Simulator([g], [0, 0, 0], [0.4, 0.9, 1.3], [TJ] * 3, d_max=16, precision="c64", trunc_rel=1e-6,
                              max_steps=8, mode=mode)
        s.step(6)
        s.set_angles([math.pi / 2] * 3, [TJ] * 3)
        s.step_inverse(2)
        hs.append(s.z_history())
        s.close()
    for a, b in zip(*hs):
        assert np.array_equal(a, b)


def test_inverse_graph_rebuilt_after_set_tiles(sim_mod):
    """Changing tile shapes drops both captured step graphs; inverse steps recorded before and
    after the change continue the same evolution as the oracle."""
    g = eagle127()
    _say("eagle127 D=8 c128: 3 steps, inverse, set_tiles, inverse")
    s = sim_mod.Simulator([g], [0], [0.7], [TJ], d_max=8, precision="c128", trunc_rel=1e-12, max_steps=5)
    s.step(3)
    s.set_angles([math.pi / 2], [TJ])
    s.step_inverse(1)
    s.set_tiles(8, 1, 64)
    s.step_inverse(1)
    (h,) = s.z_history()
    s.close()
    ref = su.evolve_graph(g, 0.7, TJ, 8, 3, 1e-12, inverse_steps=2).z
    assert np.max(np.abs(h - ref)) < TOL["c128"]
