"""Pins of the seeded input generator (integrals, JW Hamiltonian, UCCSD, compiler)."""
import numpy as np
import pytest

from vqe_inputs import configs
from vqe_inputs.compile import compile_rotations
from vqe_inputs.pauli import support
from vqe_inputs.problem import integrals, uccsd_excitations
from oracle import sector as sec
from oracle import statevector as sv


def test_integral_symmetry_and_seed():
    h, g = integrals(4, 11)
    h2, g2 = integrals(4, 11)
    assert np.array_equal(h, h2) and np.array_equal(g, g2)
    assert np.array_equal(h, h.T)
    for perm in ("qprs", "pqsr", "rspq", "srqp", "qpsr"):
        assert np.array_equal(g, np.einsum("pqrs->" + perm, g))
    assert np.count_nonzero(g) > 0


def _dense_ops(n):
    dim = 2 ** n
    Nop = np.zeros(dim)
    Sz = np.zeros(dim)
    for idx in range(dim):
        for q in range(n):
            b = (idx >> (n - 1 - q)) & 1
            Nop[idx] += b
            Sz[idx] += b * (0.5 if q % 2 == 0 else -0.5)
    return np.diag(Nop), np.diag(Sz)


def test_hamiltonian_hermitian_and_symmetries():
    p, _ = configs.load("c1")
    H = sv.dense_hamiltonian(p.ham_x, p.ham_z, p.ham_c, p.c0, p.n_qubits)
    assert np.abs(H - H.conj().T).max() < 1e-12
    Nop, Sz = _dense_ops(p.n_qubits)
    assert np.abs(H @ Nop - Nop @ H).max() < 1e-12
    assert np.abs(H @ Sz - Sz @ H).max() < 1e-12


@pytest.mark.parametrize("nq,ne", [(8, 4), (10, 6)])
def test_jw_matches_fermionic_sector_elements(nq, ne):
    """Every sector matrix element of the JW Pauli sum equals the Slater-Condon one."""
    if nq == 8:
        p, _ = configs.load("c1")
    else:
        p, _ = configs.small(nq, ne, 16, seed=1)
    u = sec.UCCSD(p)
    Hs = u.H.toarray()
    ap = sv.PauliApplier(p.n_qubits)
    dets = u.sec.dets
    for j in range(len(dets)):
        e = np.zeros(len(dets))
        e[j] = 1.0
        col = sv.apply_h(ap, u.sec.to_dense(e), p.ham_x, p.ham_z, p.ham_c, p.c0)
        ref = u.sec.to_dense(Hs[:, j])
        assert np.abs(col - ref).max() < 1e-12


def test_uccsd_counts():
    # singles i->a same spin, doubles S_z-conserving, 2 and 8 strings each
    expect = {"c1": (26, 160), "c2": (140, 1000), "c3": (1818, 14112)}
    for name, (nt, M) in expect.items():
        cfg = configs.CONFIGS[name]
        exc = uccsd_excitations(cfg["n_qubits"], cfg["n_elec"])
        assert len(exc) == nt
    p, _ = configs.load("c1")
    assert len(p.rot_c) == 160
    ns = sum(1 for e in p.excitations if len(e) == 2)
    nd = len(p.excitations) - ns
    assert len(p.rot_c) == 2 * ns + 8 * nd
    assert np.allclose(np.abs(p.rot_c[: 2 * ns]), 1.0)
    assert np.allclose(np.abs(p.rot_c[2 * ns:]), 0.25)


def test_compiled_gate_list_structure():
    p, gl = configs.load("c1")
    a, b = support(p.rot_x, p.rot_z)
    assert gl.n_rot_gates == int(np.sum(2 * (b - a + 1) - 3))
    assert gl.n_gates <= gl.n_rot_gates
    th = p.theta
    for g in range(gl.n_gates):
        U = gl.matrix(g, th)
        assert np.abs(U.conj().T @ U - np.eye(4)).max() < 1e-12
        assert 0 <= gl.bond[g] < p.n_qubits - 1
    assert np.count_nonzero(gl.kind == 1) == len(p.rot_c)


@pytest.mark.parametrize("fuse", [False, True])
def test_compiled_circuit_equals_rotations(fuse):
    p, _ = configs.load("c1")
    gl = compile_rotations(p.rot_x, p.rot_z, p.rot_c, p.rot_p, p.n_qubits, fuse=fuse)
    rng = np.random.default_rng(5)
    th = rng.normal(0, 0.7, p.n_theta)
    a = sv.run_rotations(p, th)
    b = sv.run_gates(gl, p.occ, th)
    assert np.abs(a - b).max() < 1e-12


def test_counts_recorded_for_large_configs():
    p, gl = configs.load("c3")
    assert p.n_qubits == 24 and p.n_theta == 1818 and len(p.rot_c) == 14112
    assert 2.0e4 <= p.n_terms <= 4.0e4
    assert 3.5e5 <= gl.n_gates <= 5.0e5
