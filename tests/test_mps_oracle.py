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
