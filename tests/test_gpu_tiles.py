"""Tile shapes of the batched launches: every candidate the autotuner may pick is parity-green.

  * each (QR rows per lane, re-absorb tiles per wave, SVD threads) choice against the oracle at
    D = 16 and 32, in complex64 and complex128, and the adjoint with the one-wave SVD;
  * the complex64 re-absorb on the matrix cores gives the same bits for every tile choice;
  * gpeps_autotune returns a candidate pair, leaves the initial state (history cleared) and the
    evolution that follows matches the oracle.
"""

import math
import sys

import numpy as np
import pytest

from heavyhex import eagle127
from oracle import su

pytestmark = pytest.mark.gpu
TJ = -math.pi / 2


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


@pytest.fixture(scope="module")
def ref16():
    return su.evolve_graph(eagle127(), 0.7, TJ, 16, 8, 1e-6).z


@pytest.mark.parametrize("qr,rb,sv", [(16, 1, 256), (8, 2, 64), (16, 4, 64), (8, 4, 256)])
def test_tile_pairs_d16(sim_mod, ref16, qr, rb, sv):
    _say(f"eagle127 D=16 c64 8 steps tiles qr={qr} rb={rb} svd={sv}")
    s = sim_mod.Simulator([eagle127()], [0], [0.7], [TJ], d_max=16, precision="c64", trunc_rel=1e-6, max_steps=8)
    s.set_tiles(qr, rb, sv)
    s.step(8)
    (h,) = s.z_history()
    s.close()
    assert np.max(np.abs(h - ref16)) < 1e-5


def test_reabsorb_tiles_bitwise_d32(sim_mod):
    g = eagle127()
    hs = []
    for rb in (1, 2, 4, 8):
        _say(f"eagle127 D=32 c64 6 steps re-absorb tiles {rb}")
        s = sim_mod.Simulator([g], [0], [1.0], [TJ], d_max=32, precision="c64", trunc_rel=1e-6, max_steps=6)
        s.set_tiles(16, rb, 256)
        s.step(6)
        hs.append(s.z_history()[0])
        s.close()
    assert all(np.array_equal(hs[0], h) for h in hs[1:])
    ref = su.evolve_graph(g, 1.0, TJ, 32, 6, 1e-6).z
    assert np.max(np.abs(hs[0] - ref)) < 1e-5


def test_qr_rows_d32(sim_mod):
    g = eagle127()
    _say("eagle127 D=32 c64 6 steps QR rows 8")
    s = sim_mod.Simulator([g], [0], [1.0], [TJ], d_max=32, precision="c64", trunc_rel=1e-6, max_steps=6)
    s.set_tiles(8, 2)
    s.step(6)
    (h,) = s.z_history()
    s.close()
    ref = su.evolve_graph(g, 1.0, TJ, 32, 6, 1e-6).z
    assert np.max(np.abs(h - ref)) < 1e-5


def test_one_wave_svd_complex128(sim_mod):
    """The 64-thread SVD on the complex128 path (accumulated rotations) against the oracle."""
    g = eagle127()
    _say("eagle127 D=8 c128 8 steps, 64-thread SVD")
    s = sim_mod.Simulator([g], [0], [0.7], [TJ], d_max=8, precision="c128", trunc_rel=1e-12, max_steps=8)
    s.set_tiles(16, 2, 64)
    s.step(8)
    (h,) = s.z_history()
    (dims,) = s.bond_dims()
    s.close()
    tr = su.evolve_graph(g, 0.7, TJ, 8, 8, 1e-12)
    assert np.max(np.abs(h - tr.z)) < 1e-10
    assert np.array_equal(dims, tr.bond_dims[-1])


@pytest.mark.parametrize("prec,tol", [("c128", 1e-8), ("c64", 2e-5)])
def test_one_wave_svd_gradient(sim_mod, prec, tol):
    """The reverse sweep recomputes with the forward's SVD workgroup size (same gauge)."""
    from oracle import grad as G
    g = eagle127()
    eps = 1e-12 if prec == "c128" else 1e-6
    _say(f"eagle127 D=4 {prec} 5 steps gradient, 64-thread SVD")
    s = sim_mod.Simulator([g], [0], [0.6], [TJ], d_max=4, precision=prec, trunc_rel=eps, max_steps=5, adjoint=True)
    s.set_tiles(16, 2, 64)
    s.step(5)
    dh, dj = s.backward([np.full(g.n_nodes, 1.0 / g.n_nodes)])
    s.close()
    r = G.loss_and_grad_graph(g, 0.6, TJ, 4, 5, eps)
    assert abs(float(dh[0]) - r.dtheta_h) < tol and abs(float(dj[0]) - r.dtheta_j) < tol


def test_autotune_then_evolve(sim_mod, ref16):
    _say("eagle127 D=16 c64 autotune over 4 steps, then 8 steps")
    s = sim_mod.Simulator([eagle127()], [0], [0.7], [TJ], d_max=16, precision="c64", trunc_rel=1e-6, max_steps=8)
    t = s.autotune(4)
    assert t["qr_rows_per_lane"] in (8, 16) and t["reabsorb_tiles_per_wave"] in (1, 2, 4, 8)
    assert t["svd_threads"] in (64, 256)
    assert np.all(s.bond_dims()[0] == 1)
    s.step(8)
    (h,) = s.z_history()
    s.close()
    assert h.shape[0] == 8
    assert np.max(np.abs(h - ref16)) < 1e-5


def test_set_tiles_rejects_bad_values(sim_mod):
    s = sim_mod.Simulator([eagle127()], [0], [0.7], [TJ], d_max=8, precision="c64", trunc_rel=1e-6, max_steps=2)
    with pytest.raises(RuntimeError):
        s.set_tiles(12, 2)
    with pytest.raises(RuntimeError):
        s.set_tiles(16, 3)
    with pytest.raises(RuntimeError):
        s.set_tiles(16, 2, 128)
    s.close()
