"""Edge cases of the GPU path: an empty circuit (no gates, no parameters), the
smallest chain with excitations, and the largest supported bond dimension
(d_max = 256: the widest site buffers and the 4-column Jacobi blocks) on a
problem whose bonds stay small, all against the CPU oracle or closed forms."""
import numpy as np
import pytest

from vqe_inputs import configs
from gpu_util import Prefix, golden, rel
from test_oracle_exact import hf_energy_closed_form

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_07983_amd import Context
    c = Context(0)
    yield c
    c.close()


def make_plan(ctx, p, g, d_max=None, **kw):
    from paper_2211_07983_amd import Plan
    return Plan(ctx, p.occ, g, p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0,
                p.bond_dim if d_max is None else d_max, p.eps, **kw)


def grad_ok(g, ref, tol=1e-8):
    return np.abs(g - ref).max() <= tol * max(1.0, np.abs(ref).max())


def test_empty_circuit_is_the_hartree_fock_state(ctx):
    p, g = configs.load("c1")
    empty = Prefix(g, 0)
    plan = make_plan(ctx, p, empty)
    assert plan.n_theta == 0
    ref = hf_energy_closed_form(p)
    e, grad, st = plan.energy_grad(np.zeros(0))
    assert abs(e - ref) <= 1e-12 * abs(ref) and grad.shape == (0,)
    assert st["n_gates_applied"] == 0
    eb, gb, _ = plan.energy_grad_batched(np.zeros((3, 0)))
    assert np.all(np.abs(eb - ref) <= 1e-12 * abs(ref)) and gb.shape == (3, 0)
    ep, gp, gg, _ = plan.energy_grad_psr(np.zeros(0))
    assert abs(ep - ref) <= 1e-12 * abs(ref) and gp.shape == (0,) and gg.shape == (0,)
    plan.free()


def test_smallest_chain_energy_grad_matches_oracle(ctx):
    """4 qubits, 2 electrons: one occupied and one virtual spatial orbital."""
    from oracle import mps
    p, g = configs.small(4, 2, 4, seed=2, theta_sigma=0.3)
    assert g.n_gates > 0
    E, grad, _ = mps.energy_grad(p, g, p.theta)
    plan = make_plan(ctx, p, g)
    e, gg, _ = plan.energy_grad(p.theta)
    assert rel(e, E) <= 1e-10
    assert grad_ok(gg, grad)
    eb, gb, _ = plan.energy_grad_batched(np.stack([p.theta, p.theta]))
    assert np.all(np.abs(eb - e) <= 1e-13 * abs(e)) and np.array_equal(gb[1], gb[0])
    plan.free()


def test_largest_bond_capacity_matches_oracle(ctx):
    """d_max = 256 (capacity 256: 512-column SVD buffers, 4-column Jacobi
    blocks, 64 work-groups per SVD) on the 8-qubit problem, whose bonds never
    exceed 16: no truncation, so E and the gradient equal the oracle's."""
    p, g = configs.load("c1")
    gold = golden()["c1"]
    plan = make_plan(ctx, p, g, d_max=256)
    e, gg, st = plan.energy_grad(p.theta)
    assert st["max_bond"] == 16 and st["gates_truncated"] == 0
    assert rel(e, gold["E"]) <= 1e-10
    assert grad_ok(gg, np.array(gold["grad"]))
    assert plan.lanes_per_launch() >= 1
    eb, gb, _ = plan.energy_grad_batched(np.stack([p.theta] * 3))
    assert np.all(np.abs(eb - e) <= 1e-13 * abs(e))
    assert np.abs(gb[2] - gg).max() <= 1e-12 * np.abs(gg).max()
    plan.free()
