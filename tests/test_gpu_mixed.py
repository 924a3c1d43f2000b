"""Instances of different sizes in shared launches (mps_energy_grad_plans):
each plan its own circuit, qubit count, capacity (and so Jacobi block width
and work-group count), truncation, precision and checkpoint interval, all
lanes of the same gate-chain launches.  Every result is checked against the
same plan evaluated alone and against the oracle:

* 6 qubits, D = 8 (exact, 243 gates);
* 8 qubits, D = 16 (exact, 1415 gates) in precision 1 (FP32 matrix-core
  sweeps), held to the reduced-precision tolerances;
* 12 qubits, D = 64, eps = 1e-6 (batched-set instance 5, truncating by eps);
* 12 qubits, D = 128, eps = 1e-6 (instance 8) with the broadened SVD adjoint.

That is Jacobi widths 32, 16 and 8 (1, 4 and 16 work-groups per lane) in one
launch."""
import numpy as np
import pytest

from vqe_inputs import configs
from gpu_util import golden, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_07983_amd import Context
    c = Context(0)
    yield c
    c.close()


def _instance(i):
    from vqe_inputs.compile import compile_problem
    from vqe_inputs.problem import make_problem
    n, ne, D, s1, s2 = configs.batched_instances()[i]
    p = make_problem(f"c4_{i}", n, ne, D, configs.PAPER_EPS, s1, s2, 0.05)
    return p, compile_problem(p)


def test_mixed_sizes_in_shared_launches(ctx):
    from oracle import sector
    from paper_2211_07983_amd import Plan, energy_grad_plans
    gold = golden()
    cases = []
    p6, g6 = configs.small(6, 2, 8, seed=1)
    cases.append(dict(p=p6, g=g6, kw={}, E=sector.UCCSD(p6).energy(p6.theta),
                      grad=sector.UCCSD(p6).gradient(p6.theta), etol=1e-10, gtol=1e-8))
    p8, g8 = configs.load("c1")
    cases.append(dict(p=p8, g=g8, kw={"precision": 1, "ckpt_gates": 300}, E=gold["c1"]["E"],
                      grad=np.array(gold["c1"]["grad"]), etol=None, gtol=1e-5))
    p5, g5 = _instance(5)
    cases.append(dict(p=p5, g=g5, kw={"ckpt_gates": 1024}, E=gold["c4p_5"]["E"], grad=np.array(gold["c4p_5"]["grad"]),
                      etol=1e-10, gtol=1e-8))
    p8b, g8b = _instance(8)
    cases.append(dict(p=p8b, g=g8b, kw={"broaden": gold["c4p_8_b"]["broaden"]}, E=gold["c4p_8_b"]["E"],
                      grad=np.array(gold["c4p_8_b"]["grad"]), etol=1e-10, gtol=1e-8))
    plans = [Plan(ctx, c["p"].occ, c["g"], c["p"].n_qubits, c["p"].ham_x, c["p"].ham_z, c["p"].ham_c, c["p"].c0,
                  c["p"].bond_dim, c["p"].eps, **c["kw"]) for c in cases]
    e, grads, st = energy_grad_plans(plans, [c["p"].theta for c in cases])
    print(f"mixed: {len(plans)} instances in {st['t_backward_ms'] / 1e3:.1f} s, max bond {st['max_bond']}")
    for k, (c, pl) in enumerate(zip(cases, plans)):
        e1, g1, _ = pl.energy_grad(c["p"].theta)
        gerr = np.abs(grads[k] - c["grad"]).max() / max(1.0, np.abs(c["grad"]).max())
        print(f"  {c['p'].n_qubits} q, D={c['p'].bond_dim}: E error {abs(e[k] - c['E']):.2e}, grad error {gerr:.2e}, "
              f"vs alone {abs(e[k] - e1):.1e} / {np.abs(grads[k] - g1).max():.1e}")
        assert abs(e[k] - e1) <= 1e-12 * abs(e1)
        assert np.abs(grads[k] - g1).max() <= 1e-10 * max(1.0, np.abs(g1).max())
        if c["etol"] is None:
            assert abs(e[k] - c["E"]) <= 1e-6
        else:
            assert rel(e[k], c["E"]) <= c["etol"]
        assert gerr <= c["gtol"]
    for pl in plans:
        pl.free()


def test_mixed_call_refuses_bad_arguments(ctx):
    from paper_2211_07983_amd import Context, MPSError, Plan, energy_grad_plans
    p, g = configs.small(6, 2, 8, seed=1)
    a = Plan(ctx, p.occ, g, p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, 8, p.eps)
    with pytest.raises(MPSError, match="MPS_EINVAL"):
        energy_grad_plans([a, a], [p.theta, p.theta])
    bad = np.array(p.theta)
    bad[0] = np.nan
    with pytest.raises(MPSError, match="MPS_EINVAL"):
        energy_grad_plans([a], [bad])
    other = Context(0)
    b = Plan(other, p.occ, g, p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, 8, p.eps)
    with pytest.raises(MPSError, match="MPS_EINVAL"):
        energy_grad_plans([a, b], [p.theta, p.theta])
    b.free()
    other.close()
    a.free()
