"""torch.autograd.Function over the simple-update evolution and its hand-written adjoint.

GpepsMeanZ.apply(theta_h, theta_j, sim, steps) returns, per instance, the mean <Z> after
`steps` Trotter steps from |0...0> (the average magnetisation of Fig. 2a).  The forward
runs libgpeps with per-step checkpoints and reads the magnetisation through gpeps_mean_z;
backward runs its reverse sweep through gpeps_backward_mean_z, which seeds the loss on the
device.  Angles are float64 tensors with one entry per instance; the result is a float64
tensor.

The reverse sweep differentiates the evolution the simulator holds when backward runs, so
backward refuses to run once anything has changed the simulator's state, angles or tiles
since this forward (for instance a second forward on the same simulator): run backward
before reusing the simulator, or give each forward its own simulator.
"""

from __future__ import annotations

import torch


class GpepsMeanZ(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta_h: torch.Tensor, theta_j: torch.Tensor, sim, steps: int):
        th = theta_h.detach().to("cpu", torch.float64).numpy()
        tj = theta_j.detach().to("cpu", torch.float64).numpy()
        sim.reset()
        sim.set_angles(th, tj)
        sim.step(int(steps))
        means = sim.mean_z()
        ctx.sim = sim
        ctx.generation = sim.generation
        return torch.from_numpy(means).to(theta_h.device)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        if ctx.sim.generation != ctx.generation:
            raise RuntimeError("GpepsMeanZ.backward: the simulator changed after this forward (another "
                               "forward, step, reset, set_angles or set_tiles); the recorded evolution "
                               "is gone, so its gradient cannot be computed")
        g = grad_out.detach().to("cpu", torch.float64).numpy()
        dh, dj = ctx.sim.backward_mean_z(g)
        dev = grad_out.device
        return torch.from_numpy(dh).to(dev), torch.from_numpy(dj).to(dev), None, None
