"""Host logic of GpepsMeanZ: a backward whose forward is no longer the simulator's recorded
evolution raises instead of returning another forward's gradient (a stand-in simulator that
counts generations like the real one; no device work)."""

import numpy as np
import pytest
import torch

from paper_2309_15642_amd.autograd import GpepsMeanZ


class _CountingSim:
    """Mimics Simulator's generation counter and the two calls the Function makes."""

    def __init__(self):
        self.generation = 0
        self.angles = None

    def reset(self):
        self.generation += 1

    def set_angles(self, th, tj):
        self.generation += 1
        self.angles = (np.array(th), np.array(tj))

    def step(self, n):
        self.generation += 1

    def mean_z(self):
        return np.cos(self.angles[0])

    def backward_mean_z(self, g):
        return -np.sin(self.angles[0]) * g, np.zeros_like(g)


def test_single_forward_backward_passes():
    sim = _CountingSim()
    th = torch.tensor([0.3, 0.8], dtype=torch.float64, requires_grad=True)
    m = GpepsMeanZ.apply(th, torch.zeros(2, dtype=torch.float64), sim, 2)
    m.sum().backward()
    assert torch.allclose(th.grad, -torch.sin(th.detach()))


def test_second_forward_invalidates_the_first():
    sim = _CountingSim()
    a = torch.tensor([0.3], dtype=torch.float64, requires_grad=True)
    b = torch.tensor([0.8], dtype=torch.float64, requires_grad=True)
    z = torch.zeros(1, dtype=torch.float64)
    loss = GpepsMeanZ.apply(a, z, sim, 2).sum() + GpepsMeanZ.apply(b, z, sim, 2).sum()
    with pytest.raises(RuntimeError, match="changed after this forward"):
        loss.backward()


def test_step_after_forward_invalidates():
    sim = _CountingSim()
    a = torch.tensor([0.3], dtype=torch.float64, requires_grad=True)
    m = GpepsMeanZ.apply(a, torch.zeros(1, dtype=torch.float64), sim, 2)
    sim.step(1)
    with pytest.raises(RuntimeError):
        m.sum().backward()
