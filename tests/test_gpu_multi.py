"""Several instances of the batched set in one call (mps_energy_grad_multi):
instances of one size class (12 qubits at D = 64: one compiled circuit, each
instance with its own seeded Hamiltonian and theta) run as lanes of the same
gate-chain launches.  Each result must equal that instance's own evaluation
(same kernels, same arithmetic per lane) and, for the instance with a stored
oracle value, the oracle's.  Plans that cannot share launches are refused."""
import numpy as np
import pytest

from vqe_inputs import configs
from gpu_util import Prefix, golden, rel

pytestmark = pytest.mark.gpu

CLASS = [4, 5, 10]          # 12 qubits, D = 64 (no truncation at 12 qubits)


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_07983_amd import Context
    c = Context(0)
    yield c
    c.close()


def instance(i):
    from vqe_inputs.compile import compile_problem
    from vqe_inputs.problem import make_problem
    n, ne, D, s1, s2 = configs.batched_instances()[i]
    p = make_problem(f"c4_{i}", n, ne, D, configs.PARITY_EPS, s1, s2, 0.05)
    return p, compile_problem(p)


def plan_of(ctx, p, g):
    from paper_2211_07983_amd import Plan
    return Plan(ctx, p.occ, g, p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, p.bond_dim, p.eps)


def test_same_class_instances_in_one_call(ctx):
    from paper_2211_07983_amd import energy_grad_multi
    inst = [instance(i) for i in CLASS]
    assert len({(p.n_qubits, p.bond_dim) for p, _ in inst}) == 1
    plans = [plan_of(ctx, p, g) for p, g in inst]
    thetas = np.stack([p.theta for p, _ in inst])
    e, gr, st = energy_grad_multi(plans, thetas)
    print(f"{len(plans)} instances in one call: E {e}, max bond {st['max_bond']}")
    for k in (0, 2):
        e1, g1, _ = plans[k].energy_grad(inst[k][0].theta)
        assert abs(e[k] - e1) <= 1e-13 * abs(e1)
        assert np.abs(gr[k] - g1).max() <= 1e-12 * np.abs(g1).max()
    gold = golden()["c4_4"]
    assert rel(e[0], gold["E"]) <= 1e-10
    ref = np.array(gold["grad"])
    assert np.abs(gr[0] - ref).max() <= 1e-8 * max(1.0, np.abs(ref).max())
    # the Hamiltonians differ, so the energies must too
    assert len(set(np.round(e, 6))) == len(e)
    for pl in plans:
        pl.free()


def test_incompatible_plans_are_refused(ctx):
    from paper_2211_07983_amd import MPSError, energy_grad_multi
    p4, g4 = instance(4)
    p3, g3 = instance(3)          # 12 qubits, D = 32
    a = plan_of(ctx, p4, g4)
    b = plan_of(ctx, p3, g3)
    other = Prefix(g4, len(g4.bond))       # the same gates, one angle coefficient changed
    other.coeff = np.array(other.coeff, dtype=np.float64)
    k = int(np.nonzero(np.asarray(g4.kind) == 1)[0][0])
    other.coeff[k] *= 2.0
    c = plan_of(ctx, p4, other)
    assert c.n_theta == a.n_theta
    with pytest.raises(MPSError, match="truncation"):
        energy_grad_multi([a, b], np.stack([p4.theta, p3.theta]))
    with pytest.raises(MPSError, match="circuit"):
        energy_grad_multi([a, c], np.stack([p4.theta, p4.theta]))
    with pytest.raises(ValueError):
        energy_grad_multi([a, a], p4.theta[None, :])
    for pl in (a, b, c):
        pl.free()
