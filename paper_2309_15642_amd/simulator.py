"""Python front end of libgpeps: marshals arguments, owns the torch workspace.

Every step of the simple update runs in the HIP kernels of libgpeps.  PyTorch
provides the device workspace (one uint8 tensor) and the HIP stream; nothing
here computes on the state.
"""

from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _lib

PRECISIONS = {"c64": _lib.GPEPS_C64_F64SVD, "c128": _lib.GPEPS_C128}
MODES = {"batched": _lib.GPEPS_MODE_BATCHED, "plain": _lib.GPEPS_MODE_PLAIN}


def _graph_struct(n_nodes: int, edges: np.ndarray, colour: Optional[np.ndarray], keep: list) -> _lib.gpeps_graph:
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    keep.append(e)
    g = _lib.gpeps_graph()
    g.n_nodes = int(n_nodes)
    g.n_edges = int(e.shape[0])
    g.edges = e.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    if colour is not None:
        c = np.ascontiguousarray(np.asarray(colour, dtype=np.int32))
        keep.append(c)
        g.colour = c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    else:
        g.colour = None
    return g


class Simulator:
    """A batch of kicked-Ising gPEPS evolutions on one GPU.

    graphs: objects with n_nodes, edges [E, 2] and colour [E] (colour may be
    None for library colouring); graph_of_instance: graph index per instance;
    theta_h, theta_j: angles per instance (radians).
    """

    def __init__(self, graphs: Sequence, graph_of_instance: Sequence[int], theta_h: Sequence[float],
                 theta_j: Sequence[float], d_max: int, precision: str = "c64", trunc_rel: float = 1e-6,
                 max_steps: int = 64, mode: str = "batched", max_jacobi_sweeps: int = 40,
                 device: str = "cuda:0", stream=None, adjoint: int = 0):
        import torch

        self._torch = torch
        self.lib = _lib.load()
        self._keep: List[np.ndarray] = []
        n_g = len(graphs)
        garr = (_lib.gpeps_graph * n_g)()
        for k, g in enumerate(graphs):
            garr[k] = _graph_struct(g.n_nodes, g.edges, getattr(g, "colour", None), self._keep)
        self.graphs = list(graphs)
        goi = np.ascontiguousarray(np.asarray(graph_of_instance, dtype=np.int32))
        th = np.ascontiguousarray(np.asarray(theta_h, dtype=np.float64))
        tj = np.ascontiguousarray(np.asarray(theta_j, dtype=np.float64))
        if not (len(goi) == len(th) == len(tj)):
            raise ValueError("graph_of_instance, theta_h and theta_j must have one entry per instance")
        self.graph_of_instance = goi
        self.n_instances = len(goi)
        self.nodes_per_instance = [int(graphs[g].n_nodes) for g in goi]
        self.edges_per_instance = [int(np.asarray(graphs[g].edges).shape[0]) for g in goi]
        cfg = _lib.gpeps_config()
        cfg.d_max = int(d_max)
        cfg.precision = PRECISIONS[precision]
        cfg.trunc_rel = float(trunc_rel)
        cfg.max_jacobi_sweeps = int(max_jacobi_sweeps)
        cfg.max_steps = int(max_steps)
        cfg.mode = MODES[mode]
        cfg.adjoint = int(adjoint)  # False/0, True/1 (recompute), 2 (forward keeps every class's data)
        self.cfg = cfg
        P = ctypes.POINTER
        nbytes = ctypes.c_size_t(0)
        _lib.check(self.lib, self.lib.gpeps_workspace_size(garr, n_g, goi.ctypes.data_as(P(ctypes.c_int32)),
                                                           len(goi), ctypes.byref(cfg), ctypes.byref(nbytes)))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        ctx = ctypes.c_void_p(0)
        _lib.check(self.lib, self.lib.gpeps_init(
            ctypes.byref(ctx), garr, n_g, goi.ctypes.data_as(P(ctypes.c_int32)), len(goi),
            th.ctypes.data_as(P(ctypes.c_double)), tj.ctypes.data_as(P(ctypes.c_double)), ctypes.byref(cfg),
            ctypes.c_void_p(self.workspace.data_ptr()), ctypes.c_size_t(int(nbytes.value)),
            ctypes.c_void_p(self.stream.cuda_stream)))
        self.ctx = ctx
        self.generation = 0  # bumped by every call that changes the state, the angles or the tiles
        self.n_nodes_total = int(sum(self.nodes_per_instance))
        self.n_edges_total = int(sum(self.edges_per_instance))
        self.max_steps = int(max_steps)

    # ---------------------------------------------------------------- calls
    def _check(self, status: int) -> None:
        _lib.check(self.lib, status, self.ctx)

    def reset(self) -> None:
        self.generation += 1
        self._check(self.lib.gpeps_reset(self.ctx))

    def step(self, n: int = 1) -> None:
        self.generation += 1
        self._check(self.lib.gpeps_apply_layer(self.ctx, _lib.GPEPS_STEP, int(n)))

    def step_inverse(self, n: int = 1) -> None:
        """n applications of U(theta_h)^dagger with the current angles, each recorded in the history."""
        self.generation += 1
        self._check(self.lib.gpeps_apply_layer(self.ctx, _lib.GPEPS_STEP_INVERSE, int(n)))

    def regauge(self, n: int = 1) -> None:
        """n BP-gauging sweeps (identity-gate simple update on every edge); the state is unchanged."""
        self.generation += 1
        self._check(self.lib.gpeps_apply_layer(self.ctx, _lib.GPEPS_LAYER_REGAUGE, int(n)))

    def rx_layer(self) -> None:
        self.generation += 1
        self._check(self.lib.gpeps_apply_layer(self.ctx, _lib.GPEPS_LAYER_RX, 1))

    def rzz_layer(self) -> None:
        self.generation += 1
        self._check(self.lib.gpeps_apply_layer(self.ctx, _lib.GPEPS_LAYER_RZZ, 1))

    def sync(self) -> None:
        self._check(self.lib.gpeps_sync(self.ctx))

    def expect_z(self) -> List[np.ndarray]:
        """<Z_v> per instance (list of float64 arrays)."""
        out = np.empty(self.n_nodes_total, dtype=np.float64)
        self._check(self.lib.gpeps_expect_z(self.ctx, ctypes.c_void_p(out.ctypes.data), 0))
        return self._split(out)

    def bp_expect_z(self, iters: int):
        """Belief propagation on the current state: (BP <Z_v> per instance, residual of the last iteration)."""
        out = np.empty(self.n_nodes_total, dtype=np.float64)
        res = ctypes.c_double(0.0)
        self._check(self.lib.gpeps_bp_expect_z(self.ctx, int(iters), ctypes.c_void_p(out.ctypes.data), 0,
                                               ctypes.byref(res)))
        return self._split(out), res.value

    def z_history(self) -> List[np.ndarray]:
        """Per-step <Z_v> per instance: list of [steps, n_nodes] arrays."""
        n = ctypes.c_int32(0)
        self._check(self.lib.gpeps_z_history(self.ctx, None, 0, ctypes.byref(n)))
        out = np.empty((n.value, self.n_nodes_total), dtype=np.float64)
        if n.value:
            self._check(self.lib.gpeps_z_history(self.ctx, ctypes.c_void_p(out.ctypes.data), 0, ctypes.byref(n)))
        res, off = [], 0
        for m in self.nodes_per_instance:
            res.append(out[:, off:off + m].copy())
            off += m
        return res

    def bond_dims(self) -> List[np.ndarray]:
        out = np.empty(self.n_edges_total, dtype=np.int32)
        self._check(self.lib.gpeps_bond_dims(self.ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        res, off = [], 0
        for m in self.edges_per_instance:
            res.append(out[off:off + m].copy())
            off += m
        return res

    def set_angles(self, theta_h: Sequence[float], theta_j: Sequence[float]) -> None:
        th = np.ascontiguousarray(np.asarray(theta_h, dtype=np.float64))
        tj = np.ascontiguousarray(np.asarray(theta_j, dtype=np.float64))
        if th.shape != (self.n_instances,) or tj.shape != (self.n_instances,):
            raise ValueError("one theta_h and one theta_j per instance")
        P = ctypes.POINTER(ctypes.c_double)
        self.generation += 1
        self._check(self.lib.gpeps_set_angles(self.ctx, th.ctypes.data_as(P), tj.ctypes.data_as(P)))

    def backward(self, dl_dz: Sequence[np.ndarray]):
        """Reverse sweep for L = sum_v dl_dz[v] <Z_v> after the last step.

        dl_dz: one float64 array per instance (its qubits).  Returns (dL/dtheta_h, dL/dtheta_J),
        one value per instance."""
        flat = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.float64) for x in dl_dz]))
        if flat.shape != (self.n_nodes_total,):
            raise ValueError("dl_dz must cover every qubit of every instance")
        dh = np.zeros(self.n_instances)
        dj = np.zeros(self.n_instances)
        P = ctypes.POINTER(ctypes.c_double)
        self._check(self.lib.gpeps_backward(self.ctx, ctypes.c_void_p(flat.ctypes.data), 0,
                                            dh.ctypes.data_as(P), dj.ctypes.data_as(P)))
        return dh, dj

    def mean_z(self) -> np.ndarray:
        """Magnetisation of every instance: mean <Z> of its qubits after the last recorded step."""
        out = np.empty(self.n_instances, dtype=np.float64)
        self._check(self.lib.gpeps_mean_z(self.ctx, ctypes.c_void_p(out.ctypes.data), 0))
        return out

    def backward_mean_z(self, dl_dm: Sequence[float]):
        """Reverse sweep for L = sum_k dl_dm[k] * magnetisation_k; returns (dL/dtheta_h, dL/dtheta_J)."""
        g = np.ascontiguousarray(np.asarray(dl_dm, dtype=np.float64))
        if g.shape != (self.n_instances,):
            raise ValueError("one dL/dm per instance")
        dh = np.zeros(self.n_instances)
        dj = np.zeros(self.n_instances)
        P = ctypes.POINTER(ctypes.c_double)
        self._check(self.lib.gpeps_backward_mean_z(self.ctx, g.ctypes.data_as(P), dh.ctypes.data_as(P),
                                                   dj.ctypes.data_as(P)))
        return dh, dj

    def stats(self) -> Dict[str, int]:
        """Jacobi SVD statistics since the last reset."""
        out = (ctypes.c_int64 * 4)()
        self._check(self.lib.gpeps_stats(self.ctx, out, 4))
        return {"jacobi_sweeps": int(out[0]), "svds": int(out[1]), "max_sweeps": int(out[2]),
                "not_converged": int(out[3])}

    def autotune(self, steps: int) -> Dict[str, int]:
        """Time every candidate tile pair over `steps` steps, keep the fastest, reset the state."""
        out = (ctypes.c_int32 * 3)()
        self.generation += 1
        self._check(self.lib.gpeps_autotune(self.ctx, int(steps), out))
        return {"qr_rows_per_lane": int(out[0]), "reabsorb_tiles_per_wave": int(out[1]),
                "svd_threads": int(out[2])}

    def set_tiles(self, qr_rows_per_lane: int, reabsorb_tiles_per_wave: int, svd_threads: int = 256) -> None:
        """Force the tiles (8|16, 1|2|4|8, 64|256)."""
        t = (ctypes.c_int32 * 3)(int(qr_rows_per_lane), int(reabsorb_tiles_per_wave), int(svd_threads))
        self.generation += 1
        self._check(self.lib.gpeps_set_tiles(self.ctx, t))

    def time_kernels(self, steps: int) -> Dict[str, Dict[str, float]]:
        """Run `steps` steps with a hipEvent pair around every kernel launch."""
        n = 5
        avg = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        names = (ctypes.c_char_p * n)()
        self.generation += 1
        self._check(self.lib.gpeps_time_kernels(self.ctx, int(steps), n, avg, cnt, names))
        return {names[k].decode(): {"avg_ms": float(avg[k]), "launches": int(cnt[k])} for k in range(n)}

    def time_backward(self, dl_dz: Sequence[np.ndarray]):
        """gpeps_backward with a hipEvent pair around every launch of the reverse sweep: returns
        ((dL/dtheta_h, dL/dtheta_J), {kind: {"avg_ms", "launches"}})."""
        flat = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.float64) for x in dl_dz]))
        if flat.shape != (self.n_nodes_total,):
            raise ValueError("dl_dz must cover every qubit of every instance")
        n = 9
        dh = np.zeros(self.n_instances)
        dj = np.zeros(self.n_instances)
        avg = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        names = (ctypes.c_char_p * n)()
        P = ctypes.POINTER(ctypes.c_double)
        self._check(self.lib.gpeps_time_backward(self.ctx, flat.ctypes.data_as(P), dh.ctypes.data_as(P),
                                                 dj.ctypes.data_as(P), n, avg, cnt, names))
        return (dh, dj), {names[k].decode(): {"avg_ms": float(avg[k]), "launches": int(cnt[k])} for k in range(n)}

    def _split(self, flat: np.ndarray) -> List[np.ndarray]:
        res, off = [], 0
        for m in self.nodes_per_instance:
            res.append(flat[off:off + m].copy())
            off += m
        return res

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            st = self.lib.gpeps_destroy(self.ctx)
            self.ctx = ctypes.c_void_p(0)
            _lib.check(self.lib, st)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def from_workload(w, mode: str = "batched", max_steps: Optional[int] = None, **kw) -> Simulator:
    """A Simulator for a heavyhex workload recipe (graphs, angles, D, precision, cutoff)."""
    return Simulator(w.graphs, [i.graph for i in w.instances], [i.theta_h for i in w.instances],
                     [i.theta_j for i in w.instances], d_max=w.d_max, precision=w.precision,
                     trunc_rel=w.trunc_rel, max_steps=max_steps or w.rows, mode=mode, **kw)
