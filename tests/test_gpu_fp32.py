"""Precision mode 1: the Pauli sweep's transfers as complex FP32 products on
the matrix cores (three real products, FP32 accumulation), against the FP64
oracle and the FP64 GPU path on the same circuit.

Error bound used below: every transfer GEMM sums at most 2D products of
FP32-rounded operands, and a term's environment crosses at most n_qubits
sites, so a normalised term value is off by at most about
n_qubits * 2D * u32 (u32 = 2^-24, worst-case accumulation) times the
environment norms (<= 1 for the canonical sites here) times a small constant
for the three-product complex form (its re+im sums), taken as 4.  The energy
error is bounded by that times sum_k |c_k|.  The measured errors are far
below these bounds; the tests print them.
"""
import math

import numpy as np
import pytest

from vqe_inputs import configs
from gpu_util import golden, gpu_energy, rel

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def term_bound(p):
    return 4.0 * p.n_qubits * 2 * p.bond_dim * U32


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_07983_amd import Context
    c = Context(0)
    yield c
    c.close()


def fp32_energy(ctx, p, g, theta):
    from paper_2211_07983_amd import State
    st = State.product(ctx, p.occ, p.bond_dim, p.eps, precision=1)
    st.apply_circuit(g, theta)
    e, tv, s = st.expect(p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, terms=True)
    st.free()
    return e, tv, s


def test_fp32_terms_match_oracle_c1(ctx):
    """Every normalised term value of the 8-qubit workload against the oracle's."""
    from oracle import mps
    p, g = configs.load("c1")
    m = mps.forward(p, g, p.theta)
    e_ref, _, _, vals = m.energy(p.ham_x, p.ham_z, p.ham_c, p.c0)
    e, tv, s = fp32_energy(ctx, p, g, p.theta)
    err = np.abs(np.asarray(tv) - vals.real).max()
    print(f"c1 fp32: max term error {err:.2e} (bound {term_bound(p):.2e}), E error {abs(e - e_ref):.2e} Ha")
    assert err <= term_bound(p)
    assert abs(e - e_ref) <= term_bound(p) * np.abs(p.ham_c).sum()
    assert abs(s["norm"] - 1.0) <= term_bound(p)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_fp32_energy_against_oracle_and_fp64_path(ctx, name):
    p, g = configs.load(name)
    gold = golden()[name]
    e32, tv32, _ = fp32_energy(ctx, p, g, p.theta)
    e64, tv64, _, _, st = gpu_energy(ctx, p, g, p.theta, terms=True)
    st.free()
    dt = np.abs(np.asarray(tv32) - np.asarray(tv64)).max()
    print(f"{name} fp32: E error {abs(e32 - gold['E']):.2e} Ha vs oracle, max term diff vs FP64 path {dt:.2e}")
    assert dt <= term_bound(p)
    assert abs(e32 - gold["E"]) <= term_bound(p) * np.abs(p.ham_c).sum()
    assert rel(e64, gold["E"]) <= 1e-10


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_fp32_plan_energy_grad(ctx, name):
    """A plan in precision 1: E from the FP32 sweep, the site cotangents from
    the FP32 adjoint sweep (FP64 accumulation), the gate chain in FP64; E and
    the gradient against the oracle, single and batched.  The gradient bound:
    the cotangent of a site is a sum of term transfers with the same per-term
    error as the energy's, so relative to the largest entry it is within
    term_bound * sum_k |c_k| / max |g|; 1e-5 is above that for both sizes."""
    from paper_2211_07983_amd import Plan
    p, g = configs.load(name)
    gold = golden()[name]
    plan = Plan(ctx, p.occ, g, p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, p.bond_dim, p.eps, precision=1)
    e, grad, _ = plan.energy_grad(p.theta)
    ref = np.array(gold["grad"])
    gerr = np.abs(grad - ref).max() / np.abs(ref).max()
    print(f"{name} fp32 plan: E error {abs(e - gold['E']):.2e} Ha, gradient error {gerr:.2e} (relative to max)")
    assert abs(e - gold["E"]) <= term_bound(p) * np.abs(p.ham_c).sum()
    assert gerr <= 1e-5
    eb, gb, _ = plan.energy_grad_batched(np.stack([p.theta, p.theta]))
    assert abs(eb[1] - e) <= 1e-12 * abs(e)
    assert np.abs(gb[1] - grad).max() <= 1e-9 * np.abs(grad).max()
    plan.free()


def test_fp32_gradient_first_in_a_fresh_context():
    """A context whose first and only work is a precision-1 gradient: every
    buffer of the FP32 sweep and of the FP64 environments that the gradient
    takes must be set up by that call itself (regression: the FP64 identity
    scratch was only allocated by an FP64 energy sweep)."""
    from paper_2211_07983_amd import Context, Plan
    p, g = configs.load("c1")
    gold = golden()["c1"]
    c = Context(0)
    plan = Plan(c, p.occ, g, p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, p.bond_dim, p.eps, precision=1)
    e, grad, _ = plan.energy_grad(p.theta)
    ref = np.array(gold["grad"])
    assert abs(e - gold["E"]) <= term_bound(p) * np.abs(p.ham_c).sum()
    assert np.abs(grad - ref).max() <= 1e-5 * np.abs(ref).max()
    plan.free()
    c.close()


def test_fp32_full_size_24_qubits(ctx):
    """Full-size case of the matrix-core sweep: the 24-qubit, D = 128 state after
    its first 3000 gates (middle bonds 128), all 29736 terms, against the FP64
    path on the same circuit: every term value within the FP32 bound."""
    from gpu_util import Prefix
    p, g = configs.load("c3")
    pre = Prefix(g, 3000)
    e32, tv32, _ = fp32_energy(ctx, p, pre, p.theta)
    e64, tv64, _, _, st = gpu_energy(ctx, p, pre, p.theta, terms=True)
    st.free()
    dt = np.abs(np.asarray(tv32) - np.asarray(tv64)).max()
    print(f"c3 prefix fp32: E difference {abs(e32 - e64):.2e} Ha, max term diff {dt:.2e}")
    assert dt <= term_bound(p)
    assert abs(e32 - e64) <= 1e-6


def test_precision_validation(ctx):
    from paper_2211_07983_amd import MPSError, State
    p, _ = configs.load("c1")
    with pytest.raises(MPSError):
        State.product(ctx, p.occ, p.bond_dim, p.eps, precision=2)
