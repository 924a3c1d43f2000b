"""T2: dense 2^N statevector oracle (test infrastructure only).

Only tests, the smoke entry point and the benchmark's CPU-baseline leg may
import this module; the HIP path never does.

Conventions: qubit q is axis q of the (2,)*N array (qubit 0 = leftmost ket
bit), |1> = occupied.  A Pauli string (x, z) is i^{|x&z|} X^x Z^z (so a
(1,1) qubit is Y).  Pauli rotations are exp(-i phi/2 P) (the gates of the
UCCSD circuit, Sec. 2) and the energy is E = c0 + sum_k c_k <psi|P_k|psi>
(Sec. 2, Eq. expect-val).  Gradients come from the parameter-shift rule per
rotation angle (Sec. 4, Eq. psr) and, independently, from the adjoint
identity dE/dtheta_j = <psi_j|dU_j|Psi_{j-1}> + h.c. (Sec. 4, Eq.
derivative2) evaluated on exact vectors.
"""
from __future__ import annotations

import numpy as np


def _flat_mask(mask, n):
    out = 0
    m = int(mask)
    for q in range(n):
        if (m >> q) & 1:
            out |= 1 << (n - 1 - q)
    return out


def basis_state(bits):
    n = len(bits)
    psi = np.zeros(2 ** n, dtype=np.complex128)
    idx = 0
    for q, b in enumerate(bits):
        idx |= int(b) << (n - 1 - q)
    psi[idx] = 1.0
    return psi


class PauliApplier:
    """Applies P(x,z) to flat statevectors of N qubits."""

    def __init__(self, n):
        self.n = n
        self.idx = np.arange(2 ** n, dtype=np.int64)

    def apply(self, psi, x, z):
        n = self.n
        xm = _flat_mask(x, n)
        zm = _flat_mask(z, n)
        src = self.idx ^ xm
        par = np.bitwise_count((src & zm).astype(np.uint64)) & 1
        sign = 1.0 - 2.0 * par
        ph = (1j) ** (bin(int(x) & int(z)).count("1") % 4)
        return ph * sign * psi[src]

    def expect(self, psi, x, z):
        return np.vdot(psi, self.apply(psi, x, z))


def rotate(ap, psi, x, z, phi):
    """exp(-i phi/2 P) psi."""
    return np.cos(0.5 * phi) * psi - 1j * np.sin(0.5 * phi) * ap.apply(psi, x, z)


def apply_gate(psi, U, bond, n):
    """4x4 gate on qubits (bond, bond+1); row = 2 i'_bond + i'_{bond+1}."""
    v = psi.reshape(2 ** bond, 4, 2 ** (n - bond - 2))
    return np.einsum("ab,xbz->xaz", U, v).reshape(-1)


def energy(ap, psi, hx, hz, hc, c0):
    e = c0 * np.vdot(psi, psi)
    for x, z, c in zip(hx, hz, hc):
        e = e + c * ap.expect(psi, x, z)
    return e / np.vdot(psi, psi)


def apply_h(ap, psi, hx, hz, hc, c0):
    out = c0 * psi
    for x, z, c in zip(hx, hz, hc):
        out = out + c * ap.apply(psi, x, z)
    return out


def dense_hamiltonian(hx, hz, hc, c0, n):
    """Dense 2^N x 2^N matrix of the Pauli sum (small N only)."""
    ap = PauliApplier(n)
    dim = 2 ** n
    H = np.zeros((dim, dim), dtype=np.complex128)
    eye = np.eye(dim, dtype=np.complex128)
    for j in range(dim):
        H[:, j] = apply_h(ap, eye[:, j], hx, hz, hc, c0)
    return H


def run_rotations(prob, theta, phi_shift=None):
    """Final state of the rotation circuit; phi_shift = (g, delta) shifts one angle."""
    n = prob.n_qubits
    ap = PauliApplier(n)
    psi = basis_state(prob.occ)
    for g, (x, z, c, p) in enumerate(zip(prob.rot_x, prob.rot_z, prob.rot_c, prob.rot_p)):
        phi = c * theta[p]
        if phi_shift is not None and phi_shift[0] == g:
            phi = phi + phi_shift[1]
        psi = rotate(ap, psi, x, z, phi)
    return psi


def run_gates(gates, occ, theta):
    n = gates.n_qubits
    psi = basis_state(occ)
    for g in range(gates.n_gates):
        psi = apply_gate(psi, gates.matrix(g, theta), int(gates.bond[g]), n)
    return psi


def energy_rotations(prob, theta, phi_shift=None):
    ap = PauliApplier(prob.n_qubits)
    psi = run_rotations(prob, theta, phi_shift)
    return energy(ap, psi, prob.ham_x, prob.ham_z, prob.ham_c, prob.c0).real


def psr_gate_gradient(prob, theta):
    """Parameter-shift rule per rotation angle phi_g (shift +-pi/2), Eq. psr."""
    M = len(prob.rot_c)
    gphi = np.zeros(M)
    for g in range(M):
        ep = energy_rotations(prob, theta, (g, 0.5 * np.pi))
        em = energy_rotations(prob, theta, (g, -0.5 * np.pi))
        gphi[g] = 0.5 * (ep - em)
    return gphi


def chain_rule(prob, gphi):
    """dE/dtheta_p = sum_{g: p_g = p} c_g dE/dphi_g."""
    out = np.zeros(len(prob.excitations))
    np.add.at(out, prob.rot_p, prob.rot_c * gphi)
    return out


def adjoint_gate_gradient(prob, theta):
    """dE/dphi_g = 2 Re <lambda_g| (-i/2) P_g |psi_g> on exact vectors (Eq. derivative2)."""
    n = prob.n_qubits
    ap = PauliApplier(n)
    psi = run_rotations(prob, theta)
    lam = apply_h(ap, psi, prob.ham_x, prob.ham_z, prob.ham_c, prob.c0)
    M = len(prob.rot_c)
    gphi = np.zeros(M)
    for g in range(M - 1, -1, -1):
        x, z, c, p = prob.rot_x[g], prob.rot_z[g], prob.rot_c[g], prob.rot_p[g]
        gphi[g] = 2.0 * np.vdot(lam, -0.5j * ap.apply(psi, x, z)).real
        phi = c * theta[p]
        psi = rotate(ap, psi, x, z, -phi)
        lam = rotate(ap, lam, x, z, -phi)
    return gphi


def schmidt_values(psi, n, cut):
    """Singular values of psi across the cut after qubit `cut` (bond index)."""
    m = psi.reshape(2 ** (cut + 1), 2 ** (n - cut - 1))
    return np.linalg.svd(m, compute_uv=False)
