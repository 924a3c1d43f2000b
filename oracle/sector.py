"""T1: exact fixed-(N_alpha, N_beta) sector simulator (test infrastructure only).

Only tests, the smoke entry point and the benchmark's CPU-baseline leg may
import this module; the HIP path never does.

Works in the determinant basis of one particle-number/S_z sector and never
uses Pauli strings or the Jordan-Wigner map: fermionic operators act on
occupation bit patterns with the sign (-1)^{#occupied modes below j}, which
is the ordering |x> = (a+_0)^{x_0} (a+_1)^{x_1} ... |0>.

* H is the second-quantised Hamiltonian of Sec. 2 (Eq. ham-pbc) built from
  the integrals, with chemists' (pq|rs) and interleaved spin orbitals.
* U_k = exp(theta_k G_k), G_k = T_k - T_k^dagger (Sec. 2, Eq. uccansatz).
  On the pairs of determinants G_k connects, G_k^2 = -1, and it is 0
  elsewhere, so exp(theta G) = 1 + sin(theta) G + (1 - cos(theta)) G^2.
* The gradient uses the adjoint identity of Sec. 4 (Eqs. derivative and
  derivative2): dE/dtheta_k = 2 Re <lambda_k|G_k|psi_k> with
  psi_k = U_k...U_1 Phi and lambda_k = U_{k+1}^dagger...U_M^dagger H psi,
  swept backwards with two vectors as in Algorithm 1.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.sparse as sp


def sector_basis(n_qubits, n_alpha, n_beta):
    even = list(range(0, n_qubits, 2))
    odd = list(range(1, n_qubits, 2))
    dets = []
    for A in combinations(even, n_alpha):
        for B in combinations(odd, n_beta):
            m = 0
            for q in A + B:
                m |= 1 << q
            dets.append(m)
    return np.array(sorted(dets), dtype=np.int64)


def _apply_ops(dets, ops):
    """Apply prod(ops) (rightmost acts first) to basis dets.

    ops: list of (mode, dagger).  Returns (new_dets, sign, valid).
    """
    cur = dets.copy()
    sign = np.ones(len(dets))
    valid = np.ones(len(dets), dtype=bool)
    for mode, dag in reversed(ops):
        bit = np.int64(1) << np.int64(mode)
        occ = (cur & bit) != 0
        ok = ~occ if dag else occ
        valid &= ok
        below = cur & (bit - 1)
        par = np.bitwise_count(below.astype(np.uint64)) & 1
        sign *= 1.0 - 2.0 * par
        cur = cur ^ bit
    return cur, sign, valid


class Sector:
    def __init__(self, n_qubits, n_elec_alpha, n_elec_beta):
        self.n = n_qubits
        self.dets = sector_basis(n_qubits, n_elec_alpha, n_elec_beta)
        self.dim = len(self.dets)
        self.index = {int(d): i for i, d in enumerate(self.dets)}

    def operator(self, terms):
        """Sparse matrix of sum_t c_t prod(ops_t) restricted to the sector."""
        rows, cols, vals = [], [], []
        for c, ops in terms:
            new, sign, valid = _apply_ops(self.dets, ops)
            src = np.nonzero(valid)[0]
            if len(src) == 0:
                continue
            dst = np.array([self.index.get(int(d), -1) for d in new[src]])
            keep = dst >= 0
            rows.append(dst[keep])
            cols.append(src[keep])
            vals.append(c * sign[src][keep])
        if not rows:
            return sp.csr_matrix((self.dim, self.dim))
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.dim, self.dim))

    def hamiltonian(self, h, g):
        n_orb = h.shape[0]
        terms = []
        for p in range(n_orb):
            for q in range(n_orb):
                if h[p, q] != 0.0:
                    for s in (0, 1):
                        terms.append((h[p, q], [(2 * p + s, True), (2 * q + s, False)]))
        for p in range(n_orb):
            for q in range(n_orb):
                for r in range(n_orb):
                    for s_ in range(n_orb):
                        v = g[p, q, r, s_]
                        if v == 0.0:
                            continue
                        for s in (0, 1):
                            for t in (0, 1):
                                P, Q, R, S = 2 * p + s, 2 * q + s, 2 * r + t, 2 * s_ + t
                                if P == R or Q == S:
                                    continue
                                terms.append((0.5 * v, [(P, True), (R, True), (S, False), (Q, False)]))
        return self.operator(terms)

    def generator(self, exc):
        """G = T - T^dagger of one excitation."""
        if len(exc) == 2:
            i, a = exc
            T = [(a, True), (i, False)]
            Td = [(i, True), (a, False)]
        else:
            i, j, a, b = exc
            T = [(a, True), (b, True), (j, False), (i, False)]
            Td = [(i, True), (j, True), (b, False), (a, False)]
        return self.operator([(1.0, T), (-1.0, Td)])

    def state(self, occ_bits):
        m = 0
        for q, b in enumerate(occ_bits):
            if b:
                m |= 1 << q
        v = np.zeros(self.dim)
        v[self.index[m]] = 1.0
        return v

    def to_dense(self, v):
        """Embed a sector vector into the 2^N statevector (qubit 0 leftmost)."""
        out = np.zeros(2 ** self.n, dtype=np.complex128)
        for i, d in enumerate(self.dets):
            idx = 0
            for q in range(self.n):
                if (int(d) >> q) & 1:
                    idx |= 1 << (self.n - 1 - q)
            out[idx] = v[i]
        return out


class UCCSD:
    def __init__(self, prob):
        n_a = sum(1 for q in range(prob.n_elec) if q % 2 == 0)
        n_b = prob.n_elec - n_a
        self.sec = Sector(prob.n_qubits, n_a, n_b)
        self.H = self.sec.hamiltonian(prob.h, prob.g)
        self.G = [self.sec.generator(e) for e in prob.excitations]
        self.phi0 = self.sec.state(prob.occ)

    @staticmethod
    def _apply_u(G, theta, v):
        Gv = G @ v
        return v + np.sin(theta) * Gv + (1.0 - np.cos(theta)) * (G @ Gv)

    def state(self, theta):
        v = self.phi0.copy()
        for G, t in zip(self.G, theta):
            v = self._apply_u(G, t, v)
        return v

    def energy(self, theta):
        v = self.state(theta)
        return float(v @ (self.H @ v)) / float(v @ v)

    def gradient(self, theta):
        psi = self.state(theta)
        lam = self.H @ psi
        g = np.zeros(len(theta))
        for k in range(len(theta) - 1, -1, -1):
            G = self.G[k]
            g[k] = 2.0 * float(lam @ (G @ psi))
            psi = self._apply_u(G, -theta[k], psi)
            lam = self._apply_u(G, -theta[k], lam)
        return g

    def ground_energy(self):
        from scipy.sparse.linalg import eigsh
        if self.sec.dim <= 2:
            return float(np.linalg.eigvalsh(self.H.toarray())[0])
        return float(eigsh(self.H, k=1, which="SA")[0][0])
