"""The Pauli sweep alone (Sec. 3, Eq. paulistringexp; Sec. 2, Eq.
expect-val) on states built by the oracle and imported through
mps_state_import: every term's normalised <P_k> and the compensated energy
against the oracle's on

* the 8-qubit workload's state after the whole circuit at a random theta
  (oracle forward pass, right-canonical with Schmidt values);
* a random MPS that is neither canonical nor normalised, so the sweep's
  division by Z = <psi|psi> and its explicit identity environments carry the
  result;

and the import's round trip and argument checks."""
import numpy as np
import pytest

from vqe_inputs import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_07983_amd import Context
    c = Context(0)
    yield c
    c.close()


def oracle_terms(m, p):
    e, _, Z, vals = m.energy(p.ham_x, p.ham_z, p.ham_c, p.c0)
    return e, vals, Z


@pytest.mark.parametrize("seed", [0, 1])
def test_imported_oracle_state_terms_match(ctx, seed):
    from oracle import mps
    from paper_2211_07983_amd import State
    p, g = configs.load("c1")
    th = np.random.default_rng(100 + seed).normal(0.0, 0.3, p.n_theta)
    m = mps.forward(p, g, th)
    e_ref, vals, _ = oracle_terms(m, p)
    st = State.from_tensors(ctx, m.B, m.lam, p.bond_dim, p.eps)
    e, tv, s = st.expect(p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, terms=True)
    dims, B, lam = st.export()
    st.free()
    assert list(dims[1:-1]) == m.bond_dims()
    for n in range(p.n_qubits):
        assert np.array_equal(B[n], m.B[n])
    print(f"seed {seed}: max term error {np.abs(tv - vals.real).max():.2e}, E error {abs(e - e_ref):.2e}")
    assert np.abs(tv - vals.real).max() <= 1e-10
    assert abs(e - e_ref) <= 1e-10 * abs(e_ref)
    assert abs(s["norm"] - 1.0) <= 1e-12


def test_random_noncanonical_state_terms_match(ctx):
    from oracle import mps
    from paper_2211_07983_amd import State
    p, _ = configs.load("c1")
    rng = np.random.default_rng(7)
    N = p.n_qubits
    dims = [1, 2, 3, 5, 7, 5, 3, 2, 1]
    m = mps.MPS(p.occ)
    for n in range(N):
        m.B[n] = rng.normal(size=(dims[n], 2, dims[n + 1])) + 1j * rng.normal(size=(dims[n], 2, dims[n + 1]))
    m.lam = [np.abs(rng.normal(size=d)) + 0.1 for d in dims]
    e_ref, vals, Z = oracle_terms(m, p)
    assert abs(Z - 1.0) > 1.0          # really unnormalised
    st = State.from_tensors(ctx, m.B, m.lam, 8, p.eps)
    e, tv, s = st.expect(p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, terms=True)
    _, _, lam = st.export()
    st.free()
    assert all(np.array_equal(a, b) for a, b in zip(lam, m.lam))
    assert abs(s["norm"] - Z.real) <= 1e-12 * abs(Z)
    assert np.abs(tv - vals.real).max() <= 1e-10
    assert abs(e - e_ref) <= 1e-10 * abs(e_ref)


@pytest.mark.parametrize("precision", [0, 1])
def test_random_strings_on_a_random_complex_state(ctx, precision):
    """Strings of every kind, odd numbers of Y included, on a random complex,
    non-canonical MPS.  A real Hamiltonian holds only even-Y strings and the
    UCCSD states are real up to a phase, so on them a conjugated Y phase, a
    transposed environment or the bra and ket sides swapped in a transfer
    would go unseen; here the odd-Y values are of order one.  Precision 1 (the
    FP32 matrix-core transfers) is held to 1e-4 of the normalised values, FP64
    to 1e-11."""
    from oracle import mps
    from paper_2211_07983_amd import State
    n = 8
    dims = [1, 2, 4, 6, 8, 6, 4, 2, 1]
    rng = np.random.default_rng(13)
    m = mps.MPS([0] * n)
    for q in range(n):
        m.B[q] = rng.normal(size=(dims[q], 2, dims[q + 1])) + 1j * rng.normal(size=(dims[q], 2, dims[q + 1]))
    m.lam = [np.abs(rng.normal(size=d)) + 0.1 for d in dims]
    xs = rng.integers(0, 2 ** n, 400).astype(np.uint64)
    zs = rng.integers(0, 2 ** n, 400).astype(np.uint64)
    coeff = rng.normal(size=400)
    odd_y = np.array([bin(int(x) & int(z)).count("1") % 2 == 1 for x, z in zip(xs, zs)])
    e_ref, _, Z, vals = m.energy(xs, zs, coeff, 0.25)
    assert odd_y.sum() > 50 and np.abs(vals.real[odd_y]).max() > 1e-2
    st = State.from_tensors(ctx, m.B, m.lam, 8, 1e-12, precision)
    e, tv, s = st.expect(n, xs, zs, coeff, 0.25, terms=True)
    st.free()
    tol = 1e-11 if precision == 0 else 1e-4
    err = np.abs(tv - vals.real).max()
    print(f"precision {precision}: max term error {err:.2e} (odd-Y terms {odd_y.sum()}), "
          f"E error {abs(e - e_ref):.2e}")
    assert err <= tol
    assert abs(e - e_ref) <= tol * np.abs(coeff).sum()
    assert abs(s["norm"] - Z.real) <= (1e-12 if precision == 0 else 1e-5) * abs(Z)


def test_import_rejects_bad_arguments(ctx):
    from paper_2211_07983_amd import MPSError, State
    good = [np.ones((1, 2, 2)) / 2, np.ones((2, 2, 1)) / 2]
    lams = [np.ones(1), np.ones(2), np.ones(1)]
    State.from_tensors(ctx, good, lams, 2, 1e-12).free()
    with pytest.raises(MPSError, match="MPS_EINVAL"):       # bond above d_max
        State.from_tensors(ctx, good, lams, 1, 1e-12)
    bad = [good[0].copy(), good[1]]
    bad[0][0, 0, 0] = np.nan
    with pytest.raises(MPSError, match="MPS_EINVAL"):
        State.from_tensors(ctx, bad, lams, 2, 1e-12)
    with pytest.raises(MPSError, match="MPS_EINVAL"):       # negative Schmidt value
        State.from_tensors(ctx, good, [np.ones(1), -np.ones(2), np.ones(1)], 2, 1e-12)


def test_pauli_sum_rejects_identity_and_out_of_range_strings(ctx):
    """The identity string belongs in c0; masks beyond n_qubits and
    non-finite coefficients are refused before any work."""
    from paper_2211_07983_amd import MPSError, State
    st = State.product(ctx, [1, 0, 1, 0], 4, 1e-12)
    try:
        e, _, _ = st.expect(4, [0b0011], [0b0001], [0.5], 0.25)
        assert abs(e - 0.25) <= 1e-15          # Y0 X1 flips two bits of |1010>: <P> = 0
        with pytest.raises(MPSError, match="MPS_EINVAL"):
            st.expect(4, [0b0011, 0], [0b0001, 0], [0.5, 1.0], 0.25)
        with pytest.raises(MPSError, match="MPS_EINVAL"):
            st.expect(4, [0b10000], [0], [1.0], 0.0)
        with pytest.raises(MPSError, match="MPS_EINVAL"):
            st.expect(4, [0b0001], [0], [np.inf], 0.0)
        e, _, _ = st.expect(4, [0], [0b0101], [2.0], 0.0)
        assert abs(e - 2.0) <= 1e-15          # Z0 Z2 on |1010>: (-1)(-1) = 1
    finally:
        st.free()
