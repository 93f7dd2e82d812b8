"""torch.autograd.Function over the simple-update evolution and its hand-written adjoint.

GpepsMeanZ.apply(theta_h, theta_j, sim, steps) returns, per instance, the mean <Z> after
`steps` Trotter steps from |0...0> (the average magnetisation of Fig. 2a).  The forward
runs libgpeps with per-step checkpoints; backward runs its reverse sweep.  Angles are
float64 tensors with one entry per instance; the result is a float64 tensor.
"""

from __future__ import annotations

import numpy as np
import torch


class GpepsMeanZ(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta_h: torch.Tensor, theta_j: torch.Tensor, sim, steps: int):
        th = theta_h.detach().to("cpu", torch.float64).numpy()
        tj = theta_j.detach().to("cpu", torch.float64).numpy()
        sim.set_angles(th, tj)
        sim.reset()
        sim.step(int(steps))
        hist = sim.z_history()
        ctx.sim = sim
        ctx.n_nodes = [h.shape[1] for h in hist]
        means = np.array([h[-1].mean() for h in hist], dtype=np.float64)
        return torch.from_numpy(means).to(theta_h.device)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        g = grad_out.detach().to("cpu", torch.float64).numpy()
        dl_dz = [np.full(n, g[k] / n) for k, n in enumerate(ctx.n_nodes)]
        dh, dj = ctx.sim.backward(dl_dz)
        dev = grad_out.device
        return torch.from_numpy(dh).to(dev), torch.from_numpy(dj).to(dev), None, None
