"""Parameter-shift gradient (Sec. 4, Eq. psr) on the GPU: 2M + 1 shifted
forward evaluations as lanes of the gate-chain kernel, against the oracle's
back-propagated per-gate derivatives and gradient (no truncation at the
8-qubit workload's D = 16, so both are exact up to rounding)."""
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


def make_plan(ctx, p, g, **kw):
    from paper_2211_07983_amd import Plan
    return Plan(ctx, p.occ, g, p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, p.bond_dim, p.eps, **kw)


def test_psr_matches_oracle_gate_derivatives(ctx):
    from oracle import mps
    p, g = configs.load("c1")
    gold = golden()["c1"]
    _, _, info = mps.energy_grad(p, g, p.theta)
    gphi_ref = np.asarray(info["gphi"])
    plan = make_plan(ctx, p, g)
    e, grad, gg, st = plan.energy_grad_psr(p.theta)
    kind = np.asarray(g.kind)
    assert rel(e, gold["E"]) <= 1e-10
    assert st["n_gates_applied"] == (2 * int((kind == 1).sum()) + 1) * g.n_gates
    assert np.all(gg[kind == 0] == 0.0)
    scale = np.abs(gphi_ref).max()
    assert np.abs(gg - gphi_ref).max() <= 1e-9 * scale
    ref = np.array(gold["grad"])
    assert np.abs(grad - ref).max() <= 1e-9 * np.abs(ref).max()
    plan.free()


def test_psr_equals_backprop_on_gpu(ctx):
    p, g = configs.load("c1")
    plan = make_plan(ctx, p, g)
    rng = np.random.default_rng(5)
    theta = p.theta + 0.3 * rng.normal(size=p.theta.shape)
    e_bp, g_bp, _ = plan.energy_grad(theta)
    e_ps, g_ps, _, _ = plan.energy_grad_psr(theta)
    assert abs(e_ps - e_bp) <= 1e-12 * abs(e_bp)
    assert np.abs(g_ps - g_bp).max() <= 1e-9 * np.abs(g_bp).max()
    plan.free()


def test_psr_validation(ctx):
    from paper_2211_07983_amd import MPSError
    p, g = configs.load("c1")
    plan = make_plan(ctx, p, g)
    with pytest.raises(MPSError):
        plan.energy_grad_psr(p.theta[:-1])
    bad = p.theta.copy()
    bad[0] = np.nan
    with pytest.raises(MPSError):
        plan.energy_grad_psr(bad)
    plan.free()
