"""The oracle gradient pinned to finite differences, closed forms and symmetry zeros.

  * central differences of the simple-update oracle (h = 1e-5) on truncating cases;
  * theta_J = 0: <Z_v>_T = cos(T theta_h), so dL/dtheta_h = -T sin(T theta_h) (Eq. 2);
  * dL/dtheta_J = 0 at theta_J = 0 (L is even in theta_J) and dL/dtheta_h = 0 at theta_h = 0
    (L is even in theta_h): exact zeros of Eq. 2's symmetries, reached at rank-one bonds
    where the SVD backward must stay finite;
  * L(theta_h, -theta_J) = L(theta_h, theta_J), so dL/dtheta_J is odd in theta_J.
"""

import math

import numpy as np
import pytest

from heavyhex import eagle127, path, ring
from oracle import grad as G

TJ = -math.pi / 2


def _fd(g, th, tj, d, t, eps, h=1e-5):
    fh = (G.mean_z(g, th + h, tj, d, t, eps) - G.mean_z(g, th - h, tj, d, t, eps)) / (2 * h)
    fj = (G.mean_z(g, th, tj + h, d, t, eps) - G.mean_z(g, th, tj - h, d, t, eps)) / (2 * h)
    return fh, fj


@pytest.mark.parametrize("case", ["ring_d4", "chain_d4", "eagle_d4"])
def test_gradient_matches_finite_differences(case):
    g, d, t, th, tj, eps = {
        "ring_d4": (ring(12), 4, 5, 0.5, -1.2, 1e-12),
        "chain_d4": (path(8), 4, 6, 0.8, TJ, 1e-12),
        "eagle_d4": (eagle127(), 4, 4, 0.6, TJ, 1e-6),
    }[case]
    r = G.loss_and_grad_graph(g, th, tj, d, t, eps)
    fh, fj = _fd(g, th, tj, d, t, eps)
    assert abs(r.loss - G.mean_z(g, th, tj, d, t, eps)) < 1e-12
    assert abs(r.dtheta_h - fh) < 1e-7 * max(1.0, abs(fh))
    assert abs(r.dtheta_j - fj) < 1e-7 * max(1.0, abs(fj))


def test_free_precession_closed_form():
    g = eagle127()
    th, t = 0.37, 5
    r = G.loss_and_grad_graph(g, th, 0.0, 4, t, 1e-12)
    assert abs(r.loss - math.cos(t * th)) < 1e-13
    assert abs(r.dtheta_h + t * math.sin(t * th)) < 1e-10
    assert abs(r.dtheta_j) < 1e-12


def test_symmetry_zeros_at_rank_one_bonds():
    g = eagle127()
    r = G.loss_and_grad_graph(g, 0.0, TJ, 4, 4, 1e-6)
    assert r.loss == 1.0
    assert np.isfinite(r.dtheta_h) and np.isfinite(r.dtheta_j)
    assert abs(r.dtheta_h) < 1e-12 and abs(r.dtheta_j) < 1e-12


def test_theta_j_derivative_is_odd():
    g = ring(12)
    a = G.loss_and_grad_graph(g, 0.7, -1.1, 4, 5, 1e-12)
    b = G.loss_and_grad_graph(g, 0.7, 1.1, 4, 5, 1e-12)
    assert abs(a.loss - b.loss) < 1e-12
    assert abs(a.dtheta_j + b.dtheta_j) < 1e-10
    assert abs(a.dtheta_h - b.dtheta_h) < 1e-10


def test_broadening_on_squares_is_biased():
    """The SVD-backward Lorentzian on the difference of singular values agrees with central
    differences; the same Lorentzian written on squared differences (eps_F = 1e-12, s in units of
    s_0) visibly misses them, because it also suppresses well-separated pairs of small kept values
    (|s_l^2 - s_k^2| ~ 1e-6 while |s_l - s_k| ~ 1e-3)."""
    g = eagle127()
    a = G.loss_and_grad_graph(g, 0.6, TJ, 8, 6, 1e-6, eps_f=1e-12)
    b = G.loss_and_grad_graph(g, 0.6, TJ, 8, 6, 1e-6, eps_f=1e-12, broaden="squares")
    assert a.loss == b.loss
    fh, fj = _fd(g, 0.6, TJ, 8, 6, 1e-6)
    assert abs(a.dtheta_h - fh) < 1e-7 and abs(a.dtheta_j - fj) < 1e-7
    # measured: 8.1e-7 and 1.18e-5 on the squares, 6e-10 and 1.1e-9 on the difference
    assert abs(b.dtheta_j - fj) > 5e-6
    assert abs(b.dtheta_h - fh) > 2e-7
