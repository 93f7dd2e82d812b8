"""Full-size workloads against oracle trajectories written by tests/golden/make_oracle_golden.py.

The batched launch configuration is the one bench.py times (every instance and every edge of a
colour class in one launch per kernel, a captured hipGraph per Trotter step).
"""

import math
import os
import sys

import numpy as np
import pytest

from heavyhex import make_workload

pytestmark = pytest.mark.gpu
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


def _errors(sim_mod, name, fname, precision=None):
    w = make_workload(name)
    gold = np.load(os.path.join(GOLDEN, fname))
    _say(f"{name}: {len(w.instances)} instances, {w.steps} + {w.inverse_steps} inverse steps, batched, "
         f"{precision or w.precision}")
    if precision is None:
        s = sim_mod.from_workload(w, mode="batched")
    else:
        s = sim_mod.Simulator(w.graphs, [i.graph for i in w.instances], [i.theta_h for i in w.instances],
                              [i.theta_j for i in w.instances], d_max=w.d_max, precision=precision,
                              trunc_rel=w.trunc_rel, max_steps=w.rows, mode="batched")
    s.step(w.steps)
    if w.inverse_steps:
        s.set_angles([w.theta_h_inverse] * len(w.instances), [i.theta_j for i in w.instances])
        s.step_inverse(w.inverse_steps)
    hist = s.z_history()
    s.close()
    return w, hist, [np.max(np.abs(hist[k] - gold[f"z{k}"]), axis=1) for k in range(len(w.instances))]


def _storage_tolerance(name):
    """Per-instance complex64 parity bound: max(1e-5, 8 S_k).

    S_k (tests/golden/oracle_sens_<name>.npz, written by make_oracle_golden.py from oracle/ only) is
    the largest |<Z> - <Z>_oracle| over three re-runs of the oracle with a model of complex64 storage
    applied to every site tensor after each update (rounding to complex64; two seeded relative
    perturbations of size 2^-24).  It measures how far complex64 storage alone moves the trajectory.
    Where 8 S_k exceeds 1e-5 (near-Clifford theta_h: fast scrambling with cut gaps ~1e-3 amplifies
    the rounding), the fifth digit is decided by the storage precision, not by the algorithm, and
    the instance is held to 8 S_k; every other instance is held to 1e-5.  The factor covers the
    spread of one more complex64 trajectory (the GPU's, which also rounds its R factors and stops
    Jacobi at 1e-4 rotations) around three samples: measured GPU error / S_k <= 3.7 where S_k > 1.25e-6."""
    sens = np.load(os.path.join(GOLDEN, f"oracle_sens_{name}.npz"))["deviation"].max(axis=1)
    return np.maximum(1e-5, 8.0 * sens)


def test_sweep_d32_all_instances(sim_mod):
    """32 theta_h instances on [0, pi/2], D = 32, 20 steps, complex64 storage.

    theta_h = 0 stays exactly 1.  theta_h = pi/2 (Clifford point) is exactly 0 while the bonds
    are untruncated (t <= 5); from t = 6 its cut is exactly degenerate (gap 0 in the oracle),
    several truncations are correct, and it is compared for t <= 5 only.  Every other instance is
    held to max(1e-5, 8 S_k) (_storage_tolerance): 1e-5 except the near-Clifford theta_h = 1.47
    and 1.52 (and 1.32, 1.42 marginally), whose sensitivity to complex64 storage is 1e-5 and 5e-5.
    The complex128 run of the same batch below matches the oracle to 1e-10 on them.
    """
    w, hist, err = _errors(sim_mod, "eagle127_sweep_d32", "oracle_z_eagle127_sweep_d32.npz")
    tol = _storage_tolerance("eagle127_sweep_d32")
    for k, e in enumerate(err):
        print(f"instance {k:2d} theta_h={w.instances[k].theta_h:.4f} max|dZ|={e.max():.2e} tol {tol[k]:.1e}")
    assert np.all(hist[0] == 1.0)
    assert np.max(np.abs(hist[-1][:5])) < 1e-6
    for k in range(len(err) - 1):
        assert err[k].max() < tol[k], k
    assert err[-1][:5].max() < 1e-5


def test_sweep_d16_256_instances(sim_mod):
    """256 theta_h instances on [0, pi/2] of the 127-qubit graph at D = 16 in one batch (12,288
    items per colour-class launch), 20 steps, complex64 storage: every 17th instance against the
    oracle's trajectory, each within max(1e-5, 8 S_k) with S_k its complex64 storage sensitivity
    (as in _storage_tolerance; both stored with the sampled trajectories).  theta_h = 0 stays
    exactly 1.  theta_h = pi/2 has an exactly degenerate cut (oracle gap 0) from t = 5 at D = 16,
    where several truncations are correct: it is compared before that step, to 1e-5."""
    w = make_workload("eagle127_sweep_d16")
    gold = np.load(os.path.join(GOLDEN, "oracle_z_eagle127_sweep_d16_sample.npz"))
    _say(f"eagle127_sweep_d16: {len(w.instances)} instances, D=16, batched, c64")
    s = sim_mod.from_workload(w, mode="batched")
    s.step(w.steps)
    hist = s.z_history()
    s.close()
    tol = np.maximum(1e-5, 8.0 * gold["deviation"].max(axis=1))
    last = len(w.instances) - 1
    for i, k in enumerate(gold["sample"]):
        k = int(k)
        z = gold[f"z{k}"]
        if k == last:
            t0 = int(np.argmax(gold[f"gap{k}"] == 0.0))  # first exactly degenerate cut
            assert t0 == 4
            err = np.max(np.abs(hist[k][:t0] - z[:t0]))
        else:
            err = np.max(np.abs(hist[k] - z))
        print(f"instance {k:3d} theta_h={w.instances[k].theta_h:.4f} max|dZ|={err:.2e} tol {tol[i]:.1e}")
        assert err < (1e-5 if k == last else tol[i]), k
    assert np.all(hist[0] == 1.0)


def test_sweep_d32_complex128(sim_mod):
    """The same batch in complex128 (float64 everywhere, cutoff 1e-6 as the oracle): the algorithm
    matches the oracle to 1e-10 on every instance with a non-degenerate cut."""
    w, hist, err = _errors(sim_mod, "eagle127_sweep_d32", "oracle_z_eagle127_sweep_d32.npz", "c128")
    for k, e in enumerate(err):
        print(f"instance {k:2d} theta_h={w.instances[k].theta_h:.4f} max|dZ|={e.max():.2e}")
    assert np.all(hist[0] == 1.0)
    for k in range(31):
        assert err[k].max() < 1e-10, k
    assert err[-1][:5].max() < 1e-10


def test_mixed_batch_all_instances(sim_mod):
    """435 + 1123 + 8 x 127 qubits, cap D = 32, cutoff 1e-8, 40 steps."""
    if not os.path.exists(os.path.join(GOLDEN, "oracle_z_mixed_d32.npz")):
        pytest.skip("oracle trajectories of the mixed batch not generated")
    w, hist, err = _errors(sim_mod, "mixed_d32", "oracle_z_mixed_d32.npz")
    for k, e in enumerate(err):
        print(f"instance {k} ({w.graphs[w.instances[k].graph].n_nodes} q) max|dZ|={e.max():.2e}")
    for k, e in enumerate(err):
        assert e.max() < 1e-5, k


def _weight_report(w, hist, err, gold):
    for k, e in enumerate(err):
        print(f"instance {k:2d} theta_h={w.instances[k].theta_h:.4f} max|dZ|={e.max():.2e} "
              f"<Z_13>={hist[k][-1][13]:+.6f} <Z_58>={hist[k][-1][58]:+.6f} "
              f"min cut gap {gold[f'gap{k}'].min():.1e}")


def test_weight_observables_d32(sim_mod):
    """Appendix B on the 32-instance sweep: 5 steps at theta_h, then 5 steps of U(pi/2)^dagger;
    <Z_13> and <Z_58> of the last row are the weight-10 and weight-17 observables of Fig. 3."""
    w, hist, err = _errors(sim_mod, "eagle127_weight_d32", "oracle_z_eagle127_weight_d32.npz")
    gold = np.load(os.path.join(GOLDEN, "oracle_z_eagle127_weight_d32.npz"))
    _weight_report(w, hist, err, gold)
    # theta_h = 0: |0...0>, then five Clifford steps leave every <Z> at 0 (nothing truncated);
    # theta_h = pi/2: the inverse steps undo the forward ones, every <Z> is back at 1
    assert np.max(np.abs(hist[0][-1])) < 1e-6
    assert np.max(np.abs(hist[-1][-1] - 1.0)) < 1e-5
    for k, e in enumerate(err):
        assert e.max() < 1e-5, k


def test_weight_observables_d32_complex128(sim_mod):
    """The same batch in complex128: every instance matches the oracle to 1e-10."""
    w, hist, err = _errors(sim_mod, "eagle127_weight_d32", "oracle_z_eagle127_weight_d32.npz", "c128")
    gold = np.load(os.path.join(GOLDEN, "oracle_z_eagle127_weight_d32.npz"))
    _weight_report(w, hist, err, gold)
    for k, e in enumerate(err):
        assert e.max() < 1e-10, k


def test_infinite_lattice_d32(sim_mod):
    """Infinite heavy-hex lattice as the 10-qubit periodic cell: 256 theta_h instances on
    [0, pi/2] in one batch, D = 32, 20 steps, complex64 storage.  theta_h = pi/2 has exactly
    degenerate cuts from t = 6 (several truncations are correct) and is compared for t <= 5.
    Every other instance is held to max(1e-5, 8 S_k) (_storage_tolerance): 1e-5 below
    theta_h ~ 1.38, up to 5e-4 at the near-Clifford end, where complex64 storage alone moves the
    oracle's <Z> by up to 6e-5; the complex128 run below matches the oracle to 1e-10 on every 8th
    instance, these included."""
    w, hist, err = _errors(sim_mod, "heavyhex_inf_d32", "oracle_z_heavyhex_inf_d32.npz")
    tol = _storage_tolerance("heavyhex_inf_d32")
    for k, e in enumerate(err[:-1]):
        if e.max() > 1e-6:
            print(f"instance {k:3d} theta_h={w.instances[k].theta_h:.4f} max|dZ|={e.max():.2e} tol {tol[k]:.1e}")
    assert np.all(hist[0] == 1.0)
    for k in range(len(err) - 1):
        assert err[k].max() < tol[k], k
    assert err[-1][:5].max() < 1e-5


def test_infinite_lattice_d32_complex128(sim_mod):
    """Every 8th instance of the same batch in complex128: within 1e-10 of the oracle."""
    w = make_workload("heavyhex_inf_d32")
    sub = list(range(0, 255, 8))
    gold = np.load(os.path.join(GOLDEN, "oracle_z_heavyhex_inf_d32.npz"))
    _say(f"heavyhex_inf_d32 c128 on {len(sub)} instances")
    s = sim_mod.Simulator(w.graphs, [0] * len(sub), [w.instances[k].theta_h for k in sub], [w.instances[k].theta_j for k in sub],
                          d_max=w.d_max, precision="c128", trunc_rel=w.trunc_rel, max_steps=w.steps)
    s.step(w.steps)
    hist = s.z_history()
    s.close()
    errs = [float(np.max(np.abs(h - gold[f"z{k}"]))) for h, k in zip(hist, sub)]
    print("max|dZ| per instance:", " ".join(f"{e:.1e}" for e in errs))
    for e, k in zip(errs, sub):
        assert e < 1e-10, k


def test_infinite_lattice_weight_d32(sim_mod):
    """Table I on the infinite lattice: 5 steps, 5 steps of U(pi/2)^dagger, <Z_2> of the cell."""
    w, hist, err = _errors(sim_mod, "heavyhex_inf_weight_d32", "oracle_z_heavyhex_inf_weight_d32.npz")
    print("<Z_2>:", " ".join(f"{h[-1][2]:+.4f}" for h in hist))
    assert np.max(np.abs(hist[-1][-1] - 1.0)) < 1e-5
    for k, e in enumerate(err):
        assert e.max() < 1e-5, k


@pytest.mark.parametrize("d", [8, 16, 32])
def test_long_time_ladder(sim_mod, d):
    """Long-time evolution (Figs. 5-6): 127 + 435 + 1123 qubits in one batch, theta_h = 1.0,
    39 steps, one rung of the bond-dimension ladder, every row against the oracle."""
    fname = f"oracle_z_long_theta1_d{d}.npz"
    if not os.path.exists(os.path.join(GOLDEN, fname)):
        pytest.skip("oracle trajectories of the long-time workload not generated")
    w, hist, err = _errors(sim_mod, f"long_theta1_d{d}", fname)
    gold = np.load(os.path.join(GOLDEN, fname))
    for k, e in enumerate(err):
        print(f"{w.graphs[k].n_nodes} qubits D={d}: max|dZ|={e.max():.2e} min cut gap {gold[f'gap{k}'].min():.1e}")
    for k, e in enumerate(err):
        assert e.max() < 1e-5, k


def test_instance_order_does_not_change_results(sim_mod):
    """The class work lists put the instances in descending |sin theta_h| and the edge kernels
    dispatch the ends of degree-3 sites first; the items of a class touch disjoint sites, so every
    instance's history is bit for bit the same whatever the order the instances are given in
    (mixed graphs, a tie in |sin theta_h|, theta_h = 0 among them)."""
    from heavyhex import eagle127, heavy_hex
    graphs = [eagle127(), heavy_hex(13, 27, False)]
    th = [0.3, 1.2, 0.0, math.pi - 0.3, 0.9, 1.5]
    gi = [0, 1, 0, 0, 1, 0]
    tj = [-math.pi / 2] * len(th)
    orders = [list(range(len(th))), list(reversed(range(len(th)))), [3, 0, 5, 2, 4, 1]]
    hist = []
    for order in orders:
        _say(f"127 + 435 qubits, 6 instances in order {order}, D=16, 6 steps, batched")
        s = sim_mod.Simulator(graphs, [gi[k] for k in order], [th[k] for k in order], [tj[k] for k in order],
                              d_max=16, precision="c64", trunc_rel=1e-6, max_steps=6, mode="batched")
        s.step(6)
        h = s.z_history()
        s.close()
        hist.append({k: h[pos] for pos, k in enumerate(order)})
    for k in range(len(th)):
        for o in range(1, len(orders)):
            assert np.array_equal(hist[0][k], hist[o][k]), (k, orders[o])
    assert np.all(hist[0][2] == 1.0)
