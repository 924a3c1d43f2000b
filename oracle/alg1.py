"""T3b: the paper's memory-efficient back-propagation (Sec. 4, Algorithm 1)
with Hamiltonian splitting, on plain FP64 MPS -- TEST INFRASTRUCTURE.

Only tests, the smoke entry point and the benchmark's CPU-baseline leg may
import this module; the HIP path never does.

What it computes (Sec. 4): the gradient is the adjoint of the circuit
evolution applied to the adjoint of the expectation, with the outer scalar
z = 1.  The adjoint of E(psi) = <psi|H|psi> is the state 2 H|psi> (Eq.
expecgrad).  Algorithm 1 then walks the circuit backwards with two states:
Psi, which starts at the final state Psi_M, and phi, which starts at 2 H Psi_M.
For each gate, last to first: Psi <- U^dagger Psi, then the gate's derivative
Re <phi| dU/dphi |Psi> is recorded, then phi <- U^dagger phi.  In the MPS
simulator H Psi_M is a sum of many MPS, so H is split into m groups H_j; each
group's phi_j = 2 H_j Psi_M is compressed to bond dimension D, runs its own
reverse walk, and the gradients of the groups add up (Sec. 4; the Psi walk
is the same for every group).

Readings (the paper does not spell these out):
* phi_j is built as the direct sum of the MPS c_k P_k Psi_M over the group's
  strings, then compressed by the standard two sweeps (Schollwoeck 2011,
  Sec. 4.5.1): QR from the left, then truncated SVDs from the right with the
  forward pass's rule r = min(D, #{s_i / |s| > eps}) >= 1.  A second,
  lossless pair of sweeps puts the result in the right-canonical form with
  exact Schmidt values that the two-site gate update needs.
* Both states use the forward pass's gate update (Hastings form, truncation
  to D, eps).  That update renormalises its output; Psi is a state and stays
  normalised, while phi is a cotangent whose norm matters, so phi is carried
  as eta * phi^ with phi^ normalised and every truncation multiplies eta by
  the kept norm nu (a projection, not a renormalisation).
* Gate level: U_g = post RZZ(phi_g) pre with phi_g = c_g theta_{p_g}; the
  derivative of U_g with respect to phi_g is post (-i ZZ / 2) RZZ(phi_g) pre,
  and dE/dtheta_p sums c_g dE/dphi_g over the gates of parameter p (Sec. 5
  counting).  A Pauli string P(x, z) = i^{|x & z|} X^x Z^z, as everywhere.

Without truncation (D at least the largest Schmidt rank met) the result is
the exact gradient, for any grouping, at every theta -- also at theta = 0,
where the state is a product state and the local gradient of the truncated
evolution (mps.energy_grad) is zero.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .mps import MPS, forward, gate_mats, site_phases


def pauli_apply(m, x, z):
    """P(x, z) |m>: a unitary on every site's physical index, so the
    right-canonical form and the Schmidt values are unchanged."""
    out = m.copy()
    for n in range(m.N):
        xb, o = site_phases(x, z, n)
        B = m.B[n]
        Bn = np.empty_like(B)
        for i in (0, 1):
            Bn[:, i ^ xb, :] = o[i] * B[:, i, :]
        out.B[n] = Bn
    return out


def _direct_sum(terms):
    """Site tensors of sum_k c_k |m_k> (block-diagonal bonds; the first site
    concatenated along its right bond and weighted by c_k, the last stacked
    along its left bond)."""
    N = terms[0][1].N
    sites = []
    for n in range(N):
        blocks = [m.B[n] for _, m in terms]
        if n == 0:
            A = np.concatenate([c * b for (c, _), b in zip(terms, blocks)], axis=2)
        elif n == N - 1:
            A = np.concatenate(blocks, axis=0)
        else:
            a = sum(b.shape[0] for b in blocks)
            bb = sum(b.shape[2] for b in blocks)
            A = np.zeros((a, 2, bb), dtype=np.complex128)
            r0 = c0 = 0
            for b in blocks:
                A[r0:r0 + b.shape[0], :, c0:c0 + b.shape[2]] = b
                r0 += b.shape[0]
                c0 += b.shape[2]
        sites.append(A)
    if N == 1:
        sites[0] = sum(c * m.B[0] for c, m in terms)
    return sites


def _left_qr(sites):
    for n in range(len(sites) - 1):
        a, _, b = sites[n].shape
        Q, R = np.linalg.qr(sites[n].reshape(2 * a, b))
        sites[n] = Q.reshape(a, 2, Q.shape[1])
        sites[n + 1] = np.einsum("kb,bic->kic", R, sites[n + 1])


def _right_svd(sites, D, eps):
    """Right-to-left SVDs; returns the normalised Schmidt values per bond
    (index n = bond between sites n-1 and n).  D = None keeps every nonzero."""
    N = len(sites)
    lam = [np.ones(1) for _ in range(N + 1)]
    for n in range(N - 1, 0, -1):
        a, _, b = sites[n].shape
        U, s, Vh = sla.svd(sites[n].reshape(a, 2 * b), full_matrices=False, lapack_driver="gesvd")
        tot = float(np.sqrt(np.sum(s ** 2)))
        sh = s / tot if tot > 0 else s
        if D is None:
            r = max(1, int(np.count_nonzero(sh > 1e-15)))
        else:
            r = max(1, min(D, int(np.count_nonzero(sh > eps))))
        sites[n] = Vh[:r].reshape(r, 2, b)
        sites[n - 1] = np.einsum("aib,bk->aik", sites[n - 1], U[:, :r] * s[:r])
        kept = s[:r]
        lam[n] = kept / np.sqrt(np.sum(kept ** 2))
    return lam


def compress(terms, D, eps):
    """sum_k c_k |m_k> as eta * phi^ with phi^ a normalised MPS of bond <= D
    in right-canonical form with its Schmidt values; returns (phi^, eta)."""
    sites = _direct_sum(terms)
    _left_qr(sites)
    _right_svd(sites, D, eps)
    # lossless re-canonicalisation: exact Schmidt values of the compressed state
    _left_qr(sites)
    lam = _right_svd(sites, None, 0.0)
    eta = float(np.linalg.norm(sites[0]))
    out = MPS.__new__(MPS)
    out.N = len(sites)
    out.B = [s.copy() for s in sites]
    out.B[0] = out.B[0] / eta
    out.lam = lam
    out.discarded = []
    out.ranks = []
    out.degenerate_cuts = 0
    return out, eta


def overlap_op(phi, op, n, psi):
    """<phi| O_{n,n+1} |psi> for a 4x4 operator O on sites (n, n+1); rows and
    columns of O are 2 i_n + i_{n+1}."""
    L = np.ones((1, 1), dtype=np.complex128)
    for k in range(n):
        L = sum(phi.B[k][:, i, :].conj().T @ L @ psi.B[k][:, i, :] for i in (0, 1))
    R = np.ones((1, 1), dtype=np.complex128)
    for k in range(psi.N - 1, n + 1, -1):
        R = sum(phi.B[k][:, i, :].conj() @ R @ psi.B[k][:, i, :].T for i in (0, 1))
    tp = np.einsum("aim,mjb->aijb", psi.B[n], psi.B[n + 1])
    tf = np.einsum("aim,mjb->aijb", phi.B[n], phi.B[n + 1])
    tp = np.einsum("xyij,aijb->axyb", op.reshape(2, 2, 2, 2), tp)
    return complex(np.einsum("ac,axyb,cxyd,bd->", L, tf.conj(), tp, R))


def _apply_kept_norm(m, n, Q, D, eps):
    """The forward pass's gate update on a normalised MPS; returns the kept
    norm nu of the truncation (1 when nothing is cut)."""
    m.apply_gate(n, Q, D, eps)
    return float(np.sqrt(max(0.0, 1.0 - m.discarded[-1])))


def gate_gradient(prob, gates, theta, groups, D=None, eps=None, psi_final=None):
    """dE/dphi_g for every gate by Algorithm 1 with the given groups (lists of
    term indices that together cover the Hamiltonian's strings).  Returns
    (gphi, info) with info["eta"] the norms of the groups' phi_j."""
    D = prob.bond_dim if D is None else D
    eps = prob.eps if eps is None else eps
    psi_M = forward(prob, gates, theta, D, eps) if psi_final is None else psi_final
    G = gates.n_gates
    mats = [gate_mats(gates, g, theta) for g in range(G)]
    gphi = np.zeros(G)
    etas = []
    for grp in groups:
        terms = [(2.0 * prob.ham_c[k], pauli_apply(psi_M, prob.ham_x[k], prob.ham_z[k])) for k in grp]
        phi, eta = compress(terms, D, eps)
        etas.append(eta)
        psi = psi_M.copy()
        for g in range(G - 1, -1, -1):
            Q, dQ = mats[g]
            n = int(gates.bond[g])
            Qh = Q.conj().T
            psi.apply_gate(n, Qh, D, eps)
            if dQ is not None:
                gphi[g] += eta * overlap_op(phi, dQ, n, psi).real
            eta *= _apply_kept_norm(phi, n, Qh, D, eps)
    return gphi, dict(eta=etas, psi_start=psi)


def chain_rule(gates, gphi, n_theta):
    """dE/dtheta_p = sum over the PARAM gates g of p of c_g dE/dphi_g."""
    out = np.zeros(n_theta)
    for g in range(gates.n_gates):
        if gates.kind[g] == 1:
            out[gates.param[g]] += gates.coeff[g] * gphi[g]
    return out


def split(n_terms, per_group):
    """Consecutive groups of per_group term indices (the last may be shorter)."""
    return [list(range(i, min(n_terms, i + per_group))) for i in range(0, n_terms, per_group)]


def energy_grad(prob, gates, theta, per_group=4, D=None, eps=None):
    """(dE/dtheta, info) by Algorithm 1 with N_h / m = per_group strings per group."""
    gphi, info = gate_gradient(prob, gates, theta, split(len(prob.ham_c), per_group), D, eps)
    return chain_rule(gates, gphi, prob.n_theta), dict(info, gphi=gphi)
