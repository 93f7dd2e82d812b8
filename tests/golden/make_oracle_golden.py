"""Write the oracle-generated expected values used by the GPU tests (calls only oracle/ and heavyhex/).

    python tests/golden/make_oracle_golden.py [grad] [sweep] [mixed] [weight] [inf] [infweight] [bp] [long]

grad  : oracle gradient + central differences for the 127-qubit D=16 20-step workload (theta_h=0.6)
sweep : <Z_v> per step of the 32-instance D=32 sweep (20 steps)
mixed : <Z_v> per step of the 435 + 1123 + 8 x 127 mixed batch (cap D=32, 40 steps)
weight: <Z_v> per row of the 32-instance D=32 weight-observable workload (5 steps, 5 inverse steps)
inf   : <Z_v> per step of the 256-instance infinite-lattice (10-qubit cell) D=32 workload, 20 steps
infweight: the infinite-lattice weight-observable workload (5 steps, 5 inverse steps)
bp    : BP readout and residual after 30 iterations on the state of the D=16 workload (20 steps)
long  : <Z_v> per step of the long-time workloads (127 + 435 + 1123 qubits, theta_h=1.0, 39 steps,
        D = 8, 16, 32), all nine (size, D) evolutions in one process pool
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


def grad_golden():
    w = make_workload("eagle127_grad_d16")
    g, ins = w.graphs[0], w.instances[0]
    r = G.loss_and_grad_graph(g, ins.theta_h, ins.theta_j, w.d_max, w.steps, w.trunc_rel)
    h = 1e-5
    fd_h = (G.mean_z(g, ins.theta_h + h, ins.theta_j, w.d_max, w.steps, w.trunc_rel)
            - G.mean_z(g, ins.theta_h - h, ins.theta_j, w.d_max, w.steps, w.trunc_rel)) / (2 * h)
    fd_j = (G.mean_z(g, ins.theta_h, ins.theta_j + h, w.d_max, w.steps, w.trunc_rel)
            - G.mean_z(g, ins.theta_h, ins.theta_j - h, w.d_max, w.steps, w.trunc_rel)) / (2 * h)
    out = {"workload": w.name, "theta_h": ins.theta_h, "theta_j": ins.theta_j, "d_max": w.d_max,
           "steps": w.steps, "trunc_rel": w.trunc_rel, "loss": r.loss, "dtheta_h": r.dtheta_h,
           "dtheta_j": r.dtheta_j, "fd_h": 1e-5, "fd_dtheta_h": fd_h, "fd_dtheta_j": fd_j,
           "source": "oracle/grad.py reverse sweep and central differences of oracle/su.py"}
    with open(os.path.join(HERE, "oracle_grad_eagle127_d16.json"), "w") as f:
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
    if w.inverse_steps or name.startswith("heavyhex_inf"):
        arrs.update({f"gap{k}": res[k][1] for k in range(len(w.instances))})
    np.savez_compressed(os.path.join(HERE, fname), **arrs,
                        theta_h=np.array([i.theta_h for i in w.instances]))
    print("wrote", fname)


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
    if "infweight" in what:
        traj_golden("heavyhex_inf_weight_d32", "oracle_z_heavyhex_inf_weight_d32.npz")
