"""GPU forward path (S1-S6) against the CPU oracle, through the C ABI."""
import numpy as np
import pytest

from vqe_inputs import configs
from test_oracle_exact import hf_energy_closed_form
from gpu_util import Prefix, golden, gpu_energy, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_07983_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_product_state_energy_is_hf_closed_form(ctx, name):
    from paper_2211_07983_amd import State
    p, _ = configs.load(name)
    st = State.product(ctx, p.occ, p.bond_dim, p.eps)
    e, tv, s = st.expect(p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, terms=True)
    ref = hf_energy_closed_form(p)
    assert abs(e - ref) <= 1e-12 * max(1.0, abs(ref))
    assert abs(s["norm"] - 1.0) < 1e-15 and abs(s["imag_E"]) < 1e-14
    occ_mask = sum(1 << q for q in range(p.n_qubits) if p.occ[q])
    for x, z, v in zip(p.ham_x[:500], p.ham_z[:500], tv[:500]):
        want = 0.0 if int(x) else (-1.0 if bin(int(z) & occ_mask).count("1") % 2 else 1.0)
        assert v == want


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_forward_energy_matches_oracle(ctx, name):
    p, g = configs.load(name)
    gold = golden()[name]
    e, _, s1, s2, st = gpu_energy(ctx, p, g, p.theta)
    assert rel(e, gold["E"]) <= 1e-10
    assert rel(e, gold["E_exact"]) <= 1e-10
    assert abs(s2["norm"] - 1.0) <= 1e-12
    assert abs(s2["imag_E"]) <= 1e-12 * abs(e)
    dims, B, lam = st.export()
    assert list(dims[1:-1]) == gold["bonds"]
    for k in range(1, p.n_qubits):
        ref = np.array(gold["lam"][k])
        assert np.abs(lam[k] - ref).max() <= 1e-10


def test_forward_paper_threshold_matches_oracle(ctx):
    """Energy-only forward (Jacobi on C~^H without V) at eps = 1e-6, where the
    threshold truncates thousands of gates: E and final bonds against the oracle."""
    p, g = configs.load("c2", eps=configs.PAPER_EPS)
    gold = golden()["c2_paper"]
    e, _, s1, s2, st = gpu_energy(ctx, p, g, p.theta)
    assert s1["gates_truncated"] > 1000
    assert rel(e, gold["E"]) <= 1e-10
    dims, _, _ = st.export()
    assert list(dims[1:-1]) == gold["bonds"]


def test_forward_term_values_match_oracle_c1(ctx):
    from oracle import mps
    p, g = configs.load("c1")
    e, tv, _, _, _ = gpu_energy(ctx, p, g, p.theta, terms=True)
    _, info = mps.energy(p, g, p.theta)
    vals = info["mps"].term_values(p.ham_x, p.ham_z) / info["Z"]
    assert np.abs(tv - vals.real).max() <= 1e-11


def test_c3_prefix_full_size_matches_oracle(ctx):
    """First 3000 gates of the 24-qubit D=128 workload (bonds already at D)."""
    p, g = configs.load("c3")
    gold = golden()["c3_prefix"]
    pre = Prefix(g, gold["gates"])
    e, _, s1, s2, st = gpu_energy(ctx, p, pre, p.theta)
    dims, B, lam = st.export()
    assert list(dims[1:-1]) == gold["bonds"]
    assert rel(e, gold["E"]) <= 1e-10
    assert np.abs(lam[12] - np.array(gold["lam_mid"])).max() <= 1e-10
    assert s1["max_bond"] == 128


def test_repeat_is_bitwise_deterministic(ctx):
    p, g = configs.load("c1")
    a = gpu_energy(ctx, p, g, p.theta)[0]
    b = gpu_energy(ctx, p, g, p.theta)[0]
    assert a == b


def test_invalid_inputs_are_rejected(ctx):
    from paper_2211_07983_amd import MPSError, State
    p, g = configs.load("c1")
    st = State.product(ctx, p.occ, p.bond_dim, p.eps)
    bad = p.theta.copy()
    bad[3] = np.nan
    with pytest.raises(MPSError) as ei:
        st.apply_circuit(g, bad)
    assert ei.value.code == -1
    pre = Prefix(g, 5)
    pre.bond = pre.bond.copy()
    pre.bond[2] = p.n_qubits - 1
    with pytest.raises(MPSError) as ei:
        st.apply_circuit(pre, p.theta)
    assert ei.value.code == -1
    # the state is unchanged by the rejected calls
    e, _, s = st.expect(p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0)
    assert abs(e - hf_energy_closed_form(p)) < 1e-12
