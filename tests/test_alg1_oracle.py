"""Pins of the Algorithm 1 oracle (Sec. 4, memory-efficient back-propagation
with Hamiltonian splitting) against what the mathematics fixes: the dense sum
its compression must reproduce, the exact gradient of the exact sector
simulator for every grouping when nothing is truncated (also at theta = 0,
where the local gradient of the truncated evolution vanishes), and the
reverse walk returning to the Hartree-Fock state.  In the truncating regime
the reference is a brute-force dense emulation on 6 qubits: every MPS
truncation (a gate update, a sweep of the compression) keeps the leading
Schmidt components of the state across one cut, which a dense SVD of the
2^N vector reproduces, renormalised for Psi and as a plain projection for
phi."""
import numpy as np
import pytest

from oracle import alg1, mps
from oracle import sector as sec
from oracle import statevector as sv
from vqe_inputs import configs
from dense_emulation import dense, schmidt_cut


@pytest.fixture(scope="module")
def six():
    p, g = configs.small(6, 2, 8, seed=1)      # 6 qubits: D = 8 never truncates
    return p, g, sec.UCCSD(p)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_compression_reproduces_the_dense_sum(six):
    p, g, _ = six
    psi = mps.forward(p, g, p.theta)
    ks = [3, 10, 11, 40, 77]
    terms = [(p.ham_c[k], alg1.pauli_apply(psi, p.ham_x[k], p.ham_z[k])) for k in ks]
    phi, eta = alg1.compress(terms, D=64, eps=1e-14)
    ap = sv.PauliApplier(p.n_qubits)
    v = dense(psi)
    ref = sum(p.ham_c[k] * ap.apply(v, p.ham_x[k], p.ham_z[k]) for k in ks)
    assert np.abs(eta * dense(phi) - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(eta - np.linalg.norm(ref)) <= 1e-12 * eta
    # right-canonical sites and exact Schmidt values, as the gate update needs
    for n in range(1, p.n_qubits):
        B = phi.B[n]
        a = B.shape[0]
        M = B.reshape(a, -1)
        assert np.abs(M @ M.conj().T - np.eye(a)).max() <= 1e-12
        s = sv.schmidt_values(dense(phi), p.n_qubits, n - 1)
        assert np.abs(s[:len(phi.lam[n])] - phi.lam[n]).max() <= 1e-12
    # one string twice is the same state with twice the weight
    one = alg1.pauli_apply(psi, p.ham_x[3], p.ham_z[3])
    two, eta2 = alg1.compress([(1.0, one), (1.0, one)], D=8, eps=1e-14)
    assert abs(eta2 - 2.0) <= 1e-12
    assert abs(abs(np.vdot(dense(two), dense(one))) - 1.0) <= 1e-12


@pytest.mark.parametrize("per_group", [1, 4, 117])
def test_exact_gradient_for_every_grouping(six, per_group):
    """Sec. 4: the split of H into groups never changes the gradient when
    nothing is truncated; 117 strings in one group is m = 1."""
    p, g, u = six
    assert len(p.ham_c) == 117
    grad, info = alg1.energy_grad(p, g, p.theta, per_group=per_group)
    ref = u.gradient(p.theta)
    assert rel(grad, ref) <= 1e-9
    assert len(info["eta"]) == -(-117 // per_group)


def test_exact_at_theta_zero_where_the_local_gradient_vanishes(six):
    p, g, u = six
    th = np.zeros(p.n_theta)
    ref = u.gradient(th)
    assert np.linalg.norm(ref) > 0.1
    grad, _ = alg1.energy_grad(p, g, th, per_group=4)
    assert rel(grad, ref) <= 1e-9
    _, local, _ = mps.energy_grad(p, g, th)
    assert np.abs(local).max() <= 1e-12


def test_reverse_walk_returns_to_the_initial_state(six):
    p, g, _ = six
    _, info = alg1.gate_gradient(p, g, p.theta, [[0]])
    hf = sv.basis_state(p.occ)
    assert abs(abs(np.vdot(hf, dense(info["psi_start"]))) - 1.0) <= 1e-12


def test_exact_gradient_on_8_qubits():
    """The 8-qubit problem at its exact D = 16, 16 strings per group."""
    p, g = configs.load("c1")
    u = sec.UCCSD(p)
    grad, _ = alg1.energy_grad(p, g, p.theta, per_group=16)
    assert rel(grad, u.gradient(p.theta)) <= 1e-9


def dense_algorithm1(p, g, theta, groups, D, eps):
    """Algorithm 1 on 2^N vectors with the MPS truncations emulated by
    Schmidt truncations; returns (dE/dphi per gate, smallest cut gap)."""
    from vqe_inputs.compile import rzz
    N = p.n_qubits
    zz = np.diag([1.0, -1.0, -1.0, 1.0])
    gap = 1.0
    psi = sv.basis_state(p.occ)
    for k in range(g.n_gates):
        psi = sv.apply_gate(psi, g.matrix(k, theta), int(g.bond[k]), N)
        psi, _, gp = schmidt_cut(psi, N, int(g.bond[k]), D, eps, True)
        gap = min(gap, gp)
    ap = sv.PauliApplier(N)
    gphi = np.zeros(g.n_gates)
    for grp in groups:
        phi = sum(2.0 * p.ham_c[k] * ap.apply(psi, p.ham_x[k], p.ham_z[k]) for k in grp)
        for cut in range(N - 2, -1, -1):          # compression: right-to-left sweep
            phi, _, gp = schmidt_cut(phi, N, cut, D, eps, False)
            gap = min(gap, gp)
        w = psi.copy()
        for k in range(g.n_gates - 1, -1, -1):
            Q = g.matrix(k, theta)
            n = int(g.bond[k])
            w, _, gp = schmidt_cut(sv.apply_gate(w, Q.conj().T, n, N), N, n, D, eps, True)
            gap = min(gap, gp)
            if g.kind[k] == 1:
                dQ = g.post[k] @ (-0.5j * zz @ rzz(g.coeff[k] * theta[g.param[k]])) @ g.pre[k]
                gphi[k] += np.vdot(phi, sv.apply_gate(w, dQ, n, N)).real
            phi, _, gp = schmidt_cut(sv.apply_gate(phi, Q.conj().T, n, N), N, n, D, eps, False)
            gap = min(gap, gp)
    return gphi, gap


@pytest.mark.parametrize("D", [2, 4])
def test_truncating_regime_against_dense_emulation(six, D):
    p, g, _ = six
    groups = alg1.split(len(p.ham_c), 4)[:6]
    gphi, _ = alg1.gate_gradient(p, g, p.theta, groups, D=D, eps=1e-12)
    ref, gap = dense_algorithm1(p, g, p.theta, groups, D, 1e-12)
    print(f"D={D}: max |dE/dphi| {np.abs(ref).max():.3e}, difference {np.abs(gphi - ref).max():.2e}, "
          f"smallest Schmidt gap at a cut {gap:.1e}")
    assert gap > 1e-8          # no cut inside a degenerate pair: the truncation is unique
    assert np.abs(gphi - ref).max() <= 1e-9 * np.abs(ref).max()


def test_truncating_regime_is_reported(six, capsys):
    p, g, u = six
    ref = u.gradient(p.theta)
    out = []
    for D in (2, 4, 8):
        grad, _ = alg1.energy_grad(p, g, p.theta, per_group=4, D=D, eps=1e-12)
        out.append((D, rel(grad, ref)))
    print("Algorithm 1, 6 q, N_h/m = 4: relative gradient error per D " +
          ", ".join(f"D={D}: {r:.2e}" for D, r in out))
    assert out[-1][1] <= 1e-9


def test_exact_gradient_on_a_random_complex_circuit():
    """Random complex gates and random strings of every kind
    (tests/random_circuit.py): the state is genuinely complex and odd-Y
    strings count, which the molecular workload never exercises (its strings
    hold even numbers of Y's, whose phases cancel in pairs).  With four strings
    per group and no truncation (D = 16 on 8 qubits) the gradient equals the
    Richardson central differences of the statevector energy."""
    import random_circuit as rc
    gl, th = rc.circuit(8, 120, 10, 5)
    p = rc.problem(8, 300, 16, 1e-12, 6)
    ap = sv.PauliApplier(8)

    def e_sv(t):
        return sv.energy(ap, sv.run_gates(gl, p.occ, t), p.ham_x, p.ham_z, p.ham_c, p.c0).real

    def d(k, h):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        return (e_sv(tp) - e_sv(tm)) / (2 * h)
    fd = np.array([(4 * d(k, 1e-4) - d(k, 2e-4)) / 3 for k in range(len(th))])
    grad, _ = alg1.energy_grad(p, gl, th, per_group=4)
    assert rel(grad, fd) <= 1e-9
