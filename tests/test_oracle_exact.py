"""T1 (sector) and T2 (statevector) against closed forms and each other."""
from itertools import combinations

import numpy as np
import pytest

from vqe_inputs import configs
from oracle import sector as sec
from oracle import statevector as sv
from oracle import mps


def _spin(q):
    return q % 2


def hf_energy_closed_form(p):
    """E_HF = sum_i h_ii + 1/2 sum_ij [(ii|jj) - delta_{s_i s_j} (ij|ji)] (Slater-Condon)."""
    occ = [q for q in range(p.n_qubits) if p.occ[q]]
    e = 0.0
    for i in occ:
        e += p.h[i // 2, i // 2]
    for i in occ:
        for j in occ:
            e += 0.5 * p.g[i // 2, i // 2, j // 2, j // 2]
            if _spin(i) == _spin(j):
                e -= 0.5 * p.g[i // 2, j // 2, j // 2, i // 2]
    return e


def grad_theta0_closed_form(p):
    """dE/dtheta_k at theta = 0: 2 f_ai for singles, 2 <ij||ab> for doubles."""
    occ = [q for q in range(p.n_qubits) if p.occ[q]]
    g = p.g
    out = []
    for exc in p.excitations:
        if len(exc) == 2:
            i, a = exc
            f = p.h[a // 2, i // 2]
            for j in occ:
                f += g[a // 2, i // 2, j // 2, j // 2]
                if _spin(a) == _spin(j):
                    f -= g[a // 2, j // 2, j // 2, i // 2]
            out.append(2.0 * f)
        else:
            i, j, a, b = exc
            v = 0.0
            if _spin(i) == _spin(a) and _spin(j) == _spin(b):
                v += g[i // 2, a // 2, j // 2, b // 2]
            if _spin(i) == _spin(b) and _spin(j) == _spin(a):
                v -= g[i // 2, b // 2, j // 2, a // 2]
            out.append(2.0 * v)
    return np.array(out)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_hf_energy_closed_form(name):
    p, _ = configs.load(name)
    ref = hf_energy_closed_form(p)
    ap = sv.PauliApplier(p.n_qubits)
    psi = sv.basis_state(p.occ)
    e2 = sv.energy(ap, psi, p.ham_x, p.ham_z, p.ham_c, p.c0).real
    u = sec.UCCSD(p)
    e1 = u.energy(np.zeros(p.n_theta))
    assert abs(e2 - ref) <= 1e-12 * max(1.0, abs(ref))
    assert abs(e1 - ref) <= 1e-12 * max(1.0, abs(ref))


def test_hf_energy_closed_form_c3_via_mps_oracle():
    p, _ = configs.load("c3")
    m = mps.MPS(p.occ)
    E, Eim, Z, _ = m.energy(p.ham_x, p.ham_z, p.ham_c, p.c0)
    ref = hf_energy_closed_form(p)
    assert abs(E - ref) <= 1e-12 * max(1.0, abs(ref))
    assert abs(Eim) < 1e-14 and abs(Z - 1) < 1e-15


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_theta0_gradient_closed_form(name):
    p, _ = configs.load(name)
    ref = grad_theta0_closed_form(p)
    u = sec.UCCSD(p)
    g1 = u.gradient(np.zeros(p.n_theta))
    assert np.abs(g1 - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_theta0_gradient_psr_c1():
    p, _ = configs.load("c1")
    ref = grad_theta0_closed_form(p)
    g2 = sv.chain_rule(p, sv.psr_gate_gradient(p, np.zeros(p.n_theta)))
    assert np.abs(g2 - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_sector_state_equals_rotation_circuit():
    p, _ = configs.load("c1")
    rng = np.random.default_rng(3)
    th = rng.normal(0, 0.5, p.n_theta)
    u = sec.UCCSD(p)
    a = u.sec.to_dense(u.state(th))
    b = sv.run_rotations(p, th)
    assert np.abs(a - b).max() < 1e-12
    assert abs(np.linalg.norm(a) - 1) < 1e-13


def test_generator_square_is_minus_projector():
    p, _ = configs.load("c1")
    u = sec.UCCSD(p)
    for G in u.G:
        G2 = (G @ G).toarray()
        d = np.diag(G2)
        assert np.all((np.abs(d) < 1e-14) | (np.abs(d + 1) < 1e-14))
        assert np.abs(G2 - np.diag(d)).max() < 1e-14


def test_gradients_adjoint_psr_fd_agree():
    p, _ = configs.load("c1")
    th = p.theta
    u = sec.UCCSD(p)
    g_adj = u.gradient(th)
    g_psr = sv.chain_rule(p, sv.psr_gate_gradient(p, th))
    g_adj2 = sv.chain_rule(p, sv.adjoint_gate_gradient(p, th))
    # central differences with one Richardson step
    fd = np.zeros(p.n_theta)
    for k in range(p.n_theta):
        def d(h):
            e = np.zeros(p.n_theta)
            e[k] = h
            return (u.energy(th + e) - u.energy(th - e)) / (2 * h)
        h = 1e-3
        fd[k] = (4 * d(h / 2) - d(h)) / 3
    scale = np.abs(g_adj).max()
    assert np.abs(g_adj - g_psr).max() < 1e-12 * scale
    assert np.abs(g_adj - g_adj2).max() < 1e-12 * scale
    assert np.abs(g_adj - fd).max() < 1e-9 * scale


def sector_rank_bound(n, n_alpha, n_beta, cut):
    """sum over (left alpha, left beta) blocks of min(dim_left, dim_right)."""
    from math import comb
    nl = cut + 1
    la = (nl + 1) // 2
    lb = nl // 2
    ra = (n + 1) // 2 - la
    rb = n // 2 - lb
    tot = 0
    for a in range(n_alpha + 1):
        for b in range(n_beta + 1):
            dl = comb(la, a) * comb(lb, b)
            dr = comb(ra, n_alpha - a) * comb(rb, n_beta - b)
            tot += min(dl, dr)
    return tot


def test_sector_rank_bounds_table():
    def worst(n, ne):
        return max(sector_rank_bound(n, ne // 2, ne // 2, c) for c in range(n - 1))
    assert worst(8, 4) == 16
    assert worst(14, 10) == 37
    assert worst(24, 12) == 4096
    assert worst(40, 4) == 232
    assert worst(12, 6) == 64


def test_exact_state_schmidt_ranks_within_bound():
    p, _ = configs.load("c1")
    psi = sv.run_rotations(p, p.theta)
    for cut in range(p.n_qubits - 1):
        s = sv.schmidt_values(psi, p.n_qubits, cut)
        rank = int(np.count_nonzero(s > 1e-12))
        assert rank <= sector_rank_bound(p.n_qubits, 2, 2, cut)
