"""Write the oracle-generated expected values used by the GPU tests (calls only oracle/ and heavyhex/).

    python tests/golden/make_oracle_golden.py [grad] [grad32] [sweep] [sweep16] [mixed] [weight] [inf] [infweight] [bp] [long]

grad  : oracle gradient + central differences for the 127-qubit D=16 20-step workload (theta_h=0.6)
grad32: the same at D=32
sweep16: <Z_v> per step, cut gaps and complex64 storage sensitivity of every 17th instance of the
        256-instance D=16 sweep
sweep : <Z_v> per step of the 32-instance D=32 sweep (20 steps)
mixed : <Z_v> per step of the 435 + 1123 + 8 x 127 mixed batch (cap D=32, 40 steps)
weight: <Z_v> per row of the 32-instance D=32 weight-observable workload (5 steps, 5 inverse steps)
inf   : <Z_v> per step of the 256-instance infinite-lattice (10-qubit cell) D=32 workload, 20 steps
infweight: the infinite-lattice weight-observable workload (5 steps, 5 inverse steps)
bp    : BP readout and residual after 30 iterations on the state of the D=16 workload (20 steps)
long  : <Z_v> per step of the long-time workloads (127 + 435 + 1123 qubits, theta_h=1.0, 39 steps,
        D = 8, 16, 32), all nine (size, D) evolutions in one process pool
d64   : <Z_v> per step of eagle127_d64 (2 instances, 8 steps), eagle127_d64_t20 (20 steps) and
        long_theta1_d64_127 (39 steps), D = 64
sens  : sensitivity of the D=32 sweep and of the infinite-lattice batch to complex64 storage: the
        oracle re-run with every site tensor rounded to complex64 after each update, and twice with
        every site tensor multiplied entrywise by 1 + 2^-24 (a + ib), a, b uniform in [-1, 1]
        (seeds 1, 2); per instance, the largest |<Z> - <Z>_oracle| over the three runs
"""

import json
import math
import multiprocessing as mp
import os
import sys

# one BLAS thread per worker process: the pool already fills the cores
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from heavyhex import make_workload  # noqa: E402
from oracle import bp as BP  # noqa: E402
from oracle import grad as G  # noqa: E402
from oracle import su  # noqa: E402


def grad_golden(name="eagle127_grad_d16", fname="oracle_grad_eagle127_d16.json"):
    w = make_workload(name)
    g, ins = w.graphs[0], w.instances[0]
    r = G.loss_and_grad_graph(g, ins.theta_h, ins.theta_j, w.d_max, w.steps, w.trunc_rel)
    out = {"workload": w.name, "theta_h": ins.theta_h, "theta_j": ins.theta_j, "d_max": w.d_max,
           "steps": w.steps, "trunc_rel": w.trunc_rel, "loss": r.loss, "dtheta_h": r.dtheta_h,
           "dtheta_j": r.dtheta_j,
           "source": "oracle/grad.py reverse sweep and central differences of oracle/su.py"}
    # central differences at h = 1e-5, and at h = 1e-4 (the step the differentiation workload names)
    def fd(h):
        return ((G.mean_z(g, ins.theta_h + h, ins.theta_j, w.d_max, w.steps, w.trunc_rel)
                 - G.mean_z(g, ins.theta_h - h, ins.theta_j, w.d_max, w.steps, w.trunc_rel)) / (2 * h),
                (G.mean_z(g, ins.theta_h, ins.theta_j + h, w.d_max, w.steps, w.trunc_rel)
                 - G.mean_z(g, ins.theta_h, ins.theta_j - h, w.d_max, w.steps, w.trunc_rel)) / (2 * h))
    out["fd_h"] = 1e-5
    out["fd_dtheta_h"], out["fd_dtheta_j"] = fd(1e-5)
    out["fd_h1e-4_dtheta_h"], out["fd_h1e-4_dtheta_j"] = fd(1e-4)
    with open(os.path.join(HERE, fname), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


def _traj(args):
    name, k = args
    w = make_workload(name)
    ins = w.instances[k]
    g = w.graphs[ins.graph]
    tr = su.evolve_graph(g, ins.theta_h, ins.theta_j, w.d_max, w.steps, w.trunc_rel,
                         inverse_steps=w.inverse_steps, theta_h_inverse=w.theta_h_inverse)
    return k, (tr.z, tr.min_cut_gap)


def traj_golden(name, fname, procs=8):
    w = make_workload(name)
    with mp.Pool(procs) as pool:
        res = dict(pool.map(_traj, [(name, k) for k in range(len(w.instances))]))
    arrs = {f"z{k}": res[k][0] for k in range(len(w.instances))}
    arrs.update({f"gap{k}": res[k][1] for k in range(len(w.instances))})
    np.savez_compressed(os.path.join(HERE, fname), **arrs,
                        theta_h=np.array([i.theta_h for i in w.instances]))
    print("wrote", fname)


U32 = 2.0 ** -24  # unit roundoff of float32, the storage precision of complex64 site tensors


def _storage_noise_evolve(g, ins, w, model):
    """oracle/su.py's evolution with a model of complex64 storage applied to every site tensor after
    each RX layer and each gate: model 0 rounds to complex64; model s > 0 multiplies every entry by
    1 + U32 (a + ib), a, b uniform in [-1, 1] from numpy.random.default_rng(s)."""
    rng = np.random.default_rng(model) if model else None

    def store(x):
        if rng is None:
            return x.astype(np.complex64).astype(np.complex128)
        a = rng.uniform(-1.0, 1.0, x.shape) + 1j * rng.uniform(-1.0, 1.0, x.shape)
        return x * (1.0 + U32 * a)

    real_edge, real_rx = su.simple_update_edge, su.apply_rx_layer

    def edge(peps, e, theta_j, d_max, eps):
        rec = real_edge(peps, e, theta_j, d_max, eps)
        for v in (int(peps.edges[e, 0]), int(peps.edges[e, 1])):
            peps.gammas[v] = store(peps.gammas[v])
        return rec

    def rx(peps, theta_h):
        real_rx(peps, theta_h)
        for v in range(peps.n_nodes):
            peps.gammas[v] = store(peps.gammas[v])
    su.simple_update_edge, su.apply_rx_layer = edge, rx
    try:
        return su.evolve_graph(g, ins.theta_h, ins.theta_j, w.d_max, w.steps, w.trunc_rel).z
    finally:
        su.simple_update_edge, su.apply_rx_layer = real_edge, real_rx


def _sens(args):
    name, k, model = args
    w = make_workload(name)
    ins = w.instances[k]
    return k, model, _storage_noise_evolve(w.graphs[ins.graph], ins, w, model)


def sens_golden(procs=8):
    for name, fname in (("eagle127_sweep_d32", "oracle_z_eagle127_sweep_d32.npz"),
                        ("heavyhex_inf_d32", "oracle_z_heavyhex_inf_d32.npz")):
        w = make_workload(name)
        gold = np.load(os.path.join(HERE, fname))
        jobs = [(name, k, m) for k in range(len(w.instances)) for m in (0, 1, 2)]
        with mp.Pool(procs) as pool:
            res = pool.map(_sens, jobs)
        dev = np.zeros((len(w.instances), 3))
        for k, m, z in res:
            dev[k, m] = np.max(np.abs(z - gold[f"z{k}"]))
        np.savez_compressed(os.path.join(HERE, f"oracle_sens_{name}.npz"), deviation=dev,
                            theta_h=np.array([i.theta_h for i in w.instances]))
        print("wrote sensitivity of", name, dev.max(axis=1))


SWEEP16_SAMPLE = list(range(0, 256, 17))  # 16 of the 256 instances, theta_h = 0 and pi/2 among them


def sweep16_golden(procs=8):
    """Trajectories, cut gaps and complex64 storage sensitivity of every 17th instance of the
    256-instance D = 16 sweep."""
    name = "eagle127_sweep_d16"
    w = make_workload(name)
    with mp.Pool(procs) as pool:
        res = dict(pool.map(_traj, [(name, k) for k in SWEEP16_SAMPLE]))
        sens = pool.map(_sens, [(name, k, m) for k in SWEEP16_SAMPLE for m in (0, 1, 2)])
    arrs = {f"z{k}": res[k][0] for k in SWEEP16_SAMPLE}
    arrs.update({f"gap{k}": res[k][1] for k in SWEEP16_SAMPLE})
    dev = np.zeros((len(SWEEP16_SAMPLE), 3))
    for k, m, z in sens:
        dev[SWEEP16_SAMPLE.index(k), m] = np.max(np.abs(z - res[k][0]))
    np.savez_compressed(os.path.join(HERE, "oracle_z_eagle127_sweep_d16_sample.npz"), **arrs,
                        sample=np.array(SWEEP16_SAMPLE), deviation=dev,
                        theta_h=np.array([w.instances[k].theta_h for k in SWEEP16_SAMPLE]))
    print("wrote oracle_z_eagle127_sweep_d16_sample.npz", dev.max(axis=1))


def long_golden(procs=8):
    names = ["long_theta1_d8", "long_theta1_d16", "long_theta1_d32"]
    jobs = [(n, k) for n in names for k in range(3)]
    with mp.Pool(procs) as pool:
        res = pool.map(_traj, jobs)
    for n in names:
        arrs = {}
        for (jn, k), (kk, (z, gap)) in zip(jobs, res):
            if jn == n:
                arrs[f"z{kk}"] = z
                arrs[f"gap{kk}"] = gap
        np.savez_compressed(os.path.join(HERE, f"oracle_z_{n}.npz"), **arrs)
        print("wrote", n)


def bp_golden(iters=30):
    w = make_workload("eagle127_d16")
    g, ins = w.graphs[0], w.instances[0]
    tr = su.evolve_graph(g, ins.theta_h, ins.theta_j, w.d_max, w.steps, w.trunc_rel, keep_state=True)
    r = BP.run(tr.peps, iters)
    out = {"workload": w.name, "iters": iters, "bp_z": r.z.tolist(), "residual": r.residual,
           "mean_field_z": tr.z[-1].tolist(),
           "source": "oracle/bp.py run() on the oracle/su.py state after the workload's steps"}
    with open(os.path.join(HERE, "oracle_bp_eagle127_d16.json"), "w") as f:
        json.dump(out, f)
    print("wrote oracle_bp_eagle127_d16.json", r.residual)


if __name__ == "__main__":
    what = sys.argv[1:] or ["grad"]
    if "grad" in what:
        grad_golden()
    if "grad32" in what:
        grad_golden("eagle127_grad_d32", "oracle_grad_eagle127_d32.json")
    if "sweep" in what:
        traj_golden("eagle127_sweep_d32", "oracle_z_eagle127_sweep_d32.npz")
    if "mixed" in what:
        traj_golden("mixed_d32", "oracle_z_mixed_d32.npz")
    if "weight" in what:
        traj_golden("eagle127_weight_d32", "oracle_z_eagle127_weight_d32.npz")
    if "inf" in what:
        traj_golden("heavyhex_inf_d32", "oracle_z_heavyhex_inf_d32.npz")
    if "bp" in what:
        bp_golden()
    if "long" in what:
        long_golden()
    if "sens" in what:
        sens_golden()
    if "sweep16" in what:
        sweep16_golden()
    if "d64" in what:
        for name in ("eagle127_d64", "eagle127_d64_t20", "long_theta1_d64_127"):
            traj_golden(name, f"oracle_z_{name}.npz", procs=3)
    if "infweight" in what:
        traj_golden("heavyhex_inf_weight_d32", "oracle_z_heavyhex_inf_weight_d32.npz")
