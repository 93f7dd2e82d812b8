"""Degenerate and ragged inputs through the C ABI: a graph with no edges, an isolated qubit,
a single edge, bond dimension 1, and one batch that mixes them with loopy graphs (instances
whose colour classes are empty next to instances with three classes).  Every result against
a closed form, a state vector, or the oracle on the same instance."""

import math
import sys

import numpy as np
import pytest

import oracle.bp as bp
import oracle.su as su
from exactref import statevector_z
from heavyhex import eagle127, path, ring
from heavyhex.graphs import _make

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


NONE3 = _make("none3", 3, [])
ISO3 = _make("iso3", 3, [(0, 1)])


@pytest.mark.parametrize("prec,tol", [("c128", 1e-12), ("c64", 1e-6)])
def test_no_edges_free_precession(sim_mod, prec, tol):
    """No two-qubit gates: <Z>_t = cos(t theta_h) on every qubit (Eq. 2 with no couplings)."""
    _say(f"3 qubits, no edges, {prec}, 5 steps, batched and plain")
    for mode in ("batched", "plain"):
        s = sim_mod.Simulator([NONE3], [0], [0.7], [TJ], d_max=4, precision=prec, trunc_rel=1e-12, max_steps=5,
                              mode=mode)
        s.step(5)
        (h,) = s.z_history()
        (zb,), res = s.bp_expect_z(3)
        s.close()
        assert np.max(np.abs(h - np.cos(0.7 * np.arange(1, 6))[:, None])) < tol
        assert np.max(np.abs(zb - h[-1])) < tol and res == 0.0


def test_isolated_qubit_and_single_edge(sim_mod):
    """One edge plus an isolated qubit, and a two-qubit chain: trees, so exact at D = 2."""
    _say("iso3 and path2, D=2 c128, 5 steps, one batch")
    s = sim_mod.Simulator([ISO3, path(2)], [0, 1], [0.7, 0.8], [TJ, TJ], d_max=2, precision="c128",
                          trunc_rel=1e-12, max_steps=5)
    s.step(5)
    ha, hb = s.z_history()
    (za, zb), _ = s.bp_expect_z(2)
    s.close()
    sva = statevector_z(3, [(0, 1)], 0.7, TJ, 5)
    svb = statevector_z(2, [(0, 1)], 0.8, TJ, 5)
    assert np.max(np.abs(ha - sva)) < 1e-12 and np.max(np.abs(hb - svb)) < 1e-12
    assert np.max(np.abs(za - sva[-1])) < 1e-12 and np.max(np.abs(zb - svb[-1])) < 1e-12
    assert abs(ha[-1][2] - math.cos(5 * 0.7)) < 1e-12


@pytest.mark.parametrize("prec,tol", [("c128", 1e-10), ("c64", 1e-5)])
def test_bond_dimension_one(sim_mod, prec, tol):
    """D = 1 (every bond truncated to one value: a product-state evolution) against the oracle."""
    g = eagle127()
    _say(f"eagle127 D=1 {prec} 5 steps")
    s = sim_mod.Simulator([g], [0], [0.9], [TJ], d_max=1, precision=prec, trunc_rel=1e-12, max_steps=5)
    s.step(5)
    (h,) = s.z_history()
    (dims,) = s.bond_dims()
    s.close()
    ref = su.evolve_graph(g, 0.9, TJ, 1, 5, 1e-12).z
    assert np.all(dims == 1)
    assert np.max(np.abs(h - ref)) < tol


def test_ragged_batch_with_empty_classes(sim_mod):
    """One batch of five graphs of 2 to 127 qubits, one of them without edges (its instance has
    no work in any colour class), D = 4 complex128, 4 steps: every instance against its oracle,
    and the BP readout against the BP oracle."""
    gs = [NONE3, ISO3, path(2), ring(12), eagle127()]
    ths = [0.5, 0.7, 0.8, 0.6, 0.6]
    _say("ragged batch none3 + iso3 + path2 + ring12 + eagle127, D=4 c128, 4 steps")
    s = sim_mod.Simulator(gs, list(range(5)), ths, [TJ] * 5, d_max=4, precision="c128", trunc_rel=1e-12,
                          max_steps=4)
    s.step(4)
    hs = s.z_history()
    zbs, _ = s.bp_expect_z(6)
    s.close()
    for g, th, h, zb in zip(gs, ths, hs, zbs):
        tr = su.evolve_graph(g, th, TJ, 4, 4, 1e-12, keep_state=True)
        assert np.max(np.abs(h - tr.z)) < 1e-10, g.name
        assert np.max(np.abs(zb - bp.run(tr.peps, 6).z)) < 1e-10, g.name
