"""T3 (FP64 MPS oracle) against T1/T2, invariants and finite differences."""
import numpy as np
import pytest

from vqe_inputs import configs
from oracle import mps
from oracle import sector as sec
from oracle import statevector as sv


def test_product_state_terms_closed_form():
    """On a computational basis state <P> is 0 if P flips a bit, else +-1."""
    p, _ = configs.load("c1")
    m = mps.MPS(p.occ)
    vals = m.term_values(p.ham_x, p.ham_z)
    occ_mask = sum(1 << q for q in range(p.n_qubits) if p.occ[q])
    for x, z, v in zip(p.ham_x, p.ham_z, vals):
        if int(x) != 0:
            assert v == 0
        else:
            par = bin(int(z) & occ_mask).count("1") % 2
            assert v == (-1.0 if par else 1.0)


def test_c1_exact_energy_and_gradient_vs_sector():
    p, g = configs.load("c1")
    u = sec.UCCSD(p)
    E, grad, info = mps.energy_grad(p, g, p.theta)
    e1 = u.energy(p.theta)
    g1 = u.gradient(p.theta)
    assert abs(E - e1) <= 1e-11 * abs(e1)
    assert np.linalg.norm(grad - g1) / np.linalg.norm(g1) <= 1e-9
    assert max(info["discarded"]) < 1e-20


def test_c1_schmidt_values_and_invariants():
    p, g = configs.load("c1")
    E, info = mps.energy(p, g, p.theta)
    m = info["mps"]
    assert abs(info["Z"] - 1) <= 1e-12
    assert abs(info["imag"]) <= 1e-12 * abs(E)
    psi = sv.run_rotations(p, p.theta)
    for cut in range(p.n_qubits - 1):
        s = sv.schmidt_values(psi, p.n_qubits, cut)
        lam = m.lam[cut + 1]
        k = len(lam)
        assert np.abs(lam - s[:k]).max() < 1e-10
        assert np.all(s[k:] < 1e-11)
    # right-canonical condition sum_{i,beta} B B^dagger = 1 on every site but the first
    for n in range(1, p.n_qubits):
        B = m.B[n]
        Bm = B.reshape(B.shape[0], -1)
        assert np.abs(Bm @ Bm.conj().T - np.eye(B.shape[0])).max() < 1e-12


def test_exact_d_small_problem_gradient_vs_sector():
    p, g = configs.small(10, 6, 64, seed=2)
    u = sec.UCCSD(p)
    E, grad, _ = mps.energy_grad(p, g, p.theta, ckpt=50)
    g1 = u.gradient(p.theta)
    assert abs(E - u.energy(p.theta)) <= 1e-11 * abs(E)
    assert np.linalg.norm(grad - g1) / np.linalg.norm(g1) <= 1e-9


def test_checkpoint_interval_does_not_change_gradient():
    p, g = configs.load("c1")
    _, ga, _ = mps.energy_grad(p, g, p.theta, ckpt=7)
    _, gb, _ = mps.energy_grad(p, g, p.theta, ckpt=1000)
    assert np.abs(ga - gb).max() < 1e-13 * np.abs(ga).max()


@pytest.mark.parametrize("seed", [1, 3])
def test_truncating_gradient_directional_fd(seed):
    """Truncating D: g_D . v against central FD of E_D with the truncation frozen.

    Cases whose cut falls inside a (near-)degenerate cluster have no well-defined
    fixed-rank derivative; these two seeds truncate ~4% of the weight with clean gaps.
    """
    p, g = configs.small(8, 4, 6, seed=seed, theta_sigma=0.3)
    E, grad, info = mps.energy_grad(p, g, p.theta)
    assert max(info["discarded"]) > 1e-3          # the case really truncates
    e_info = mps.energy(p, g, p.theta)[1]
    assert e_info["degenerate_cuts"] == 0
    ranks = e_info["ranks"]
    rng = np.random.default_rng(0)
    u = sec.UCCSD(p)
    assert E >= u.ground_energy() - 1e-10
    for _ in range(8):
        v = rng.normal(size=p.n_theta)
        v /= np.linalg.norm(v)

        def d(h):
            ep = mps.energy(p, g, p.theta + h * v, ranks=ranks)[0]
            em = mps.energy(p, g, p.theta - h * v, ranks=ranks)[0]
            return (ep - em) / (2 * h)
        fd = (4 * d(5e-4) - d(1e-3)) / 3
        assert abs(fd - grad @ v) <= 1e-7 * max(1.0, np.linalg.norm(grad))


@pytest.mark.parametrize("seed", [1, 3])
def test_broadened_svd_adjoint_limits(seed):
    """The Lorentzian d/(d^2 + eta^2) replaces 1/d in the SVD adjoint: eta = 0
    is the plain derivative bit for bit; for eta far below every squared gap
    that carries a cotangent the change is -eta^2 sum c/d^3 + O(eta^4), so it
    falls by 4 when eta halves and vanishes with eta (the plain derivative is
    the one the directional finite differences above pin)."""
    p, g = configs.small(8, 4, 6, seed=seed, theta_sigma=0.3)
    _, g0, _ = mps.energy_grad(p, g, p.theta)
    _, gz, _ = mps.energy_grad(p, g, p.theta, broaden=0.0)
    assert np.array_equal(g0, gz)
    dev = []
    for eta in (4e-10, 2e-10, 1e-10):
        _, ge, _ = mps.energy_grad(p, g, p.theta, broaden=eta)
        dev.append(np.abs(ge - g0).max() / np.abs(g0).max())
    assert 0 < dev[2] < 1e-7
    for a, b in zip(dev, dev[1:]):
        assert 3.9 <= a / b <= 4.1
    # and it is a real change at larger eta: pairs with squared gaps near 1e-8
    _, ge, _ = mps.energy_grad(p, g, p.theta, broaden=1e-8)
    assert np.abs(ge - g0).max() > 1e-6 * np.abs(g0).max()


def test_degenerate_cut_raises_unless_broadened():
    """A truncation through an exactly degenerate pair that carries a cotangent
    has no fixed-rank derivative: the plain adjoint raises; the broadened one
    drops the pair (the Lorentzian is zero at d = 0) and stays finite."""
    import degenerate_case as dc
    p, g = dc.problem()
    _, info = mps.energy(p, g, p.theta)
    assert info["degenerate_cuts"] == 1 and abs(info["discarded"][0] - 0.5) < 1e-12
    with pytest.raises(mps.SVDDegenerate):
        mps.energy_grad(p, g, p.theta)
    _, gb, _ = mps.energy_grad(p, g, p.theta, broaden=1e-6)
    assert np.all(np.isfinite(gb))
    # away from the degeneracy the same circuit has a derivative again
    mps.energy_grad(p, g, p.theta + 0.3)


@pytest.mark.parametrize("D,eps", [(2, 1e-12), (4, 1e-12), (64, 1e-2)])
def test_one_truncating_gate_is_the_schmidt_truncation_at_its_cut(D, eps):
    """Sec. 3, two-qubit gate update: on a canonical MPS the singular values of
    lambda_{n-1} C are the state's Schmidt values across the gate's cut, so one
    truncating gate must leave exactly the state's leading r = min(D,
    #{s > eps}) Schmidt components, renormalised, with lambda_n their values
    and the discarded weight the rest.  The reference is a dense SVD of the
    2^N vector after the gate (the gate matrix from the compiled gate list, not
    the oracle's).  The state before each checked gate is the untruncated
    evolution, which stays canonical.  Over a long truncating run the two part:
    after a cut the left site is no longer exactly canonical, so later
    truncations are near-optimal, not optimal -- the method's own
    approximation, which this pin leaves alone.  D = 2, 4 cut by the bond
    limit; eps = 1e-2 cuts by the threshold."""
    from dense_emulation import dense, schmidt_cut
    p, g = configs.small(8, 4, 64, seed=3, theta_sigma=0.3)
    N = p.n_qubits
    m = mps.MPS(p.occ)
    checked = 0
    for k in range(400):
        n = int(g.bond[k])
        after = sv.apply_gate(dense(m), g.matrix(k, p.theta), n, N)
        _, r_full, _ = schmidt_cut(after, N, n, 10 ** 9, 1e-14, True)
        ref, r, gap = schmidt_cut(after, N, n, D, eps, True)
        Q, _ = mps.gate_mats(g, k, p.theta)
        if r < r_full and gap > 1e-3:
            t = m.copy()
            t.apply_gate(n, Q, D, eps)
            assert t.ranks == [r]
            assert np.abs(dense(t) - ref).max() <= 1e-12
            s = np.linalg.svd(after.reshape(2 ** (n + 1), -1), compute_uv=False)
            assert np.abs(t.lam[n + 1] - s[:r] / np.linalg.norm(s[:r])).max() <= 1e-12
            assert abs(t.discarded[0] - np.sum(s[r:] ** 2) / np.sum(s ** 2)) <= 1e-13
            assert t.degenerate_cuts == 0
            checked += 1
        m.apply_gate(n, Q, 64, 1e-14)
    assert checked >= 20


_PAULI = {(0, 0): np.eye(2), (1, 0): np.array([[0, 1], [1, 0]]),
          (1, 1): np.array([[0, -1j], [1j, 0]]), (0, 1): np.diag([1.0, -1.0])}


def _kron_pauli(x, z, n):
    """The textbook operator: one 2x2 Pauli matrix per qubit (x, z bits of
    qubit q: I = 00, X = 10, Y = 11, Z = 01), qubit 0 the leftmost factor."""
    P = np.ones((1, 1))
    for q in range(n):
        P = np.kron(P, _PAULI[((int(x) >> q) & 1, (int(z) >> q) & 1)])
    return P


@pytest.mark.parametrize("D", [16, 4])
def test_every_term_value_equals_the_kronecker_expectation(D):
    """Sec. 3, Eq. paulistringexp: every <P_k> of the sweep, divided by Z,
    against <psi|P_k|psi>/<psi|psi> with P_k a Kronecker product of the Pauli
    matrices applied to the MPS's own 2^N amplitudes.  D = 16 is exact on
    8 qubits (canonical state); D = 4 truncates, leaving a non-canonical
    state, so the environments cannot lean on canonical form."""
    from dense_emulation import dense
    p, g = configs.small(8, 4, 64, seed=3, theta_sigma=0.3)
    E, info = mps.energy(p, g, p.theta, D=D, eps=1e-12)
    m = info["mps"]
    if D == 4:
        assert max(info["discarded"]) > 1e-3
    v = dense(m)
    Z = np.vdot(v, v).real
    assert abs(Z - info["Z"]) <= 1e-12 * Z
    got = m.term_values(p.ham_x, p.ham_z) / info["Z"]
    ref = np.array([np.vdot(v, _kron_pauli(x, z, p.n_qubits) @ v) / Z for x, z in zip(p.ham_x, p.ham_z)])
    assert np.abs(ref.imag).max() <= 1e-13
    assert np.abs(got - ref).max() <= 1e-12
    assert abs(E - (p.c0 + np.dot(p.ham_c, ref.real))) <= 1e-12 * abs(E)


def test_random_strings_on_a_random_complex_mps():
    """The same against random strings of every kind on a random complex,
    non-canonical MPS.  A real Hamiltonian's strings hold an even number of
    Y's and the UCCSD state is real up to a phase, which would hide a
    conjugated Y; here the odd-Y expectations do not vanish."""
    from dense_emulation import dense
    n = 7
    rng = np.random.default_rng(11)
    m = mps.MPS([0] * n)
    bonds = [1, 2, 4, 6, 6, 4, 2, 1]
    m.B = [rng.normal(size=(bonds[q], 2, bonds[q + 1])) + 1j * rng.normal(size=(bonds[q], 2, bonds[q + 1]))
           for q in range(n)]
    v = dense(m)
    Z = np.vdot(v, v).real
    L, _ = m.identity_envs()
    assert abs(L[n][0, 0] - Z) <= 1e-12 * Z
    xs = rng.integers(0, 2 ** n, 300)
    zs = rng.integers(0, 2 ** n, 300)
    odd_y = np.array([bin(int(x) & int(z)).count("1") % 2 == 1 for x, z in zip(xs, zs)])
    got = m.term_values(xs, zs) / Z
    ref = np.array([np.vdot(v, _kron_pauli(x, z, n) @ v) / Z for x, z in zip(xs, zs)])
    assert odd_y.sum() > 50 and np.abs(ref.real[odd_y]).max() > 1e-2
    assert np.abs(ref.imag).max() <= 1e-13
    assert np.abs(got - ref).max() <= 1e-12


def _random_complex_case():
    import random_circuit as rc
    gl, th = rc.circuit(8, 120, 10, 5)
    return rc.problem(8, 300, 16, 1e-12, 6), gl, th


def test_random_complex_circuit_exact_energy_and_gradient():
    """Beyond the molecular workload: random complex two-qubit gates and a Pauli
    sum of random strings of every kind, so the state is genuinely complex and
    odd-Y terms count.  At exact D (16 on 8 qubits) E equals the statevector
    energy and every gradient entry the Richardson central difference of it."""
    p, gl, th = _random_complex_case()
    ap = sv.PauliApplier(8)

    def e_sv(t):
        return sv.energy(ap, sv.run_gates(gl, p.occ, t), p.ham_x, p.ham_z, p.ham_c, p.c0).real

    E, grad, info = mps.energy_grad(p, gl, th, ckpt=32)
    assert max(info["discarded"]) < 1e-20
    assert abs(E - e_sv(th)) <= 1e-12 * max(1.0, abs(E))

    def d(k, h):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        return (e_sv(tp) - e_sv(tm)) / (2 * h)
    fd = np.array([(4 * d(k, 1e-4) - d(k, 2e-4)) / 3 for k in range(len(th))])
    assert np.abs(grad - fd).max() <= 1e-8 * np.abs(fd).max()


def test_random_complex_circuit_truncating_directional_fd():
    """The same circuit at D = 4 (41 truncating gates, up to 12 % of the weight
    discarded, every cut at least 2.7e-2 s_1 from the next value): g_D . v
    against central differences of E_D with the truncation pattern frozen."""
    p, gl, th = _random_complex_case()
    E, grad, info = mps.energy_grad(p, gl, th, D=4)
    e_info = mps.energy(p, gl, th, D=4)[1]
    assert max(info["discarded"]) > 0.1 and e_info["degenerate_cuts"] == 0
    ranks = e_info["ranks"]
    rng = np.random.default_rng(1)
    for _ in range(6):
        v = rng.normal(size=len(th))
        v /= np.linalg.norm(v)

        def d(h):
            ep = mps.energy(p, gl, th + h * v, D=4, ranks=ranks)[0]
            em = mps.energy(p, gl, th - h * v, D=4, ranks=ranks)[0]
            return (ep - em) / (2 * h)
        # angles spread over [-pi, pi] and a 12 % truncation curve E_D strongly:
        # the Richardson error falls as h^4, to ~1e-9 at these steps
        fd = (4 * d(5e-5) - d(1e-4)) / 3
        assert abs(fd - grad @ v) <= 1e-7 * max(1.0, np.linalg.norm(grad))
