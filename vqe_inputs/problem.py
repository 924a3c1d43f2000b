"""Seeded synthetic problems: integrals, the qubit Hamiltonian and UCCSD.

The paper's molecules (PySCF integrals, Sec. 5) are not available; seeded
random real integrals with the same structure stand in for them:

* h_pq symmetric, upper triangle (p <= q, row-major) drawn from N(0, 1);
* (pq|rs) in chemists' notation with the 8-fold permutational symmetry, one
  N(0, 0.1) draw per class p >= q, r >= s, pq >= rs in compound-index order.

Spin orbitals are interleaved (qubit 2p = orbital p spin alpha, qubit 2p+1 =
spin beta) and the second-quantised Hamiltonian (Sec. 2, Eq. ham-pbc) is

    H = sum_{pq,s} h_pq a+_{ps} a_{qs}
        + 1/2 sum_{pqrs,st} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs},

i.e. the paper's g^{pq}_{rs} is (ps|qr).  Jordan-Wigner turns it into a real
weighted Pauli sum (Sec. 2, Eq. expect-val); identical strings are merged and
the identity string is kept apart as c0.

The ansatz is spin-orbital UCCSD (Sec. 2, Eq. uccansatz) with S_z-conserving
singles (i->a) and doubles (i<j -> a<b), one amplitude each, applied as a
first-order Trotter product in a fixed order: singles lexicographic in (i,a),
then doubles lexicographic in (i,j,a,b).  Each generator G = T - T^dagger is a
sum of mutually commuting Pauli strings, G = i sum_g d_g P_g, so that
exp(theta G) = prod_g exp(-i (c_g theta)/2 P_g) exactly with c_g = -2 d_g.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import pauli as pl


def integrals(n_orb: int, seed: int):
    rng = np.random.default_rng(seed)
    h = np.zeros((n_orb, n_orb))
    for p in range(n_orb):
        for q in range(p, n_orb):
            v = rng.normal(0.0, 1.0)
            h[p, q] = v
            h[q, p] = v
    g = np.zeros((n_orb,) * 4)
    pairs = [(p, q) for p in range(n_orb) for q in range(p + 1)]
    for I, (p, q) in enumerate(pairs):
        for (r, s) in pairs[: I + 1]:
            v = rng.normal(0.0, 0.1)
            for (a, b, c, d) in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                                 (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
                g[a, b, c, d] = v
    return h, g


def hamiltonian_pauli(h, g, chunk=200_000):
    """JW Pauli sum of the spin-orbital Hamiltonian: (x, z, coeff(real), c0)."""
    n_orb = h.shape[0]
    xs, zs, cs = [], [], []
    # one-body
    co, mo, da = [], [], []
    for p in range(n_orb):
        for q in range(n_orb):
            if h[p, q] == 0.0:
                continue
            for s in (0, 1):
                co.append(h[p, q])
                mo.append((2 * p + s, 2 * q + s))
                da.append((True, False))
    x, z, c = pl.fermion_products_to_pauli(co, mo, da)
    x, z, c = pl.merge(x, z, c, drop=0.0)
    xs.append(x); zs.append(z); cs.append(c)
    # two-body, in chunks to bound memory
    P, Q, R, S = np.nonzero(g)
    vals = g[P, Q, R, S]
    co, mo = [], []
    for s in (0, 1):
        for t in (0, 1):
            m = np.stack([2 * P + s, 2 * R + t, 2 * S + t, 2 * Q + s], axis=1)
            ok = (m[:, 0] != m[:, 1]) & (m[:, 2] != m[:, 3])
            co.append(0.5 * vals[ok])
            mo.append(m[ok])
    co = np.concatenate(co)
    mo = np.concatenate(mo)
    da = np.tile(np.array([True, True, False, False]), (len(co), 1))
    for lo in range(0, len(co), chunk):
        x, z, c = pl.fermion_products_to_pauli(co[lo:lo + chunk], mo[lo:lo + chunk],
                                               da[lo:lo + chunk])
        x, z, c = pl.merge(x, z, c, drop=0.0)
        xs.append(x); zs.append(z); cs.append(c)
    x, z, c = pl.merge(np.concatenate(xs), np.concatenate(zs), np.concatenate(cs), drop=1e-12)
    if np.max(np.abs(c.imag), initial=0.0) > 1e-12:
        raise ValueError("Hamiltonian Pauli coefficients are not real")
    c = c.real.copy()
    ident = (x == 0) & (z == 0)
    c0 = float(c[ident].sum())
    keep = ~ident
    return x[keep].astype(np.uint64), z[keep].astype(np.uint64), c[keep], c0


def uccsd_excitations(n_qubits: int, n_elec: int):
    occ = range(n_elec)
    vir = range(n_elec, n_qubits)
    singles = [(i, a) for i in occ for a in vir if i % 2 == a % 2]
    doubles = [(i, j, a, b)
               for i in occ for j in occ if i < j
               for a in vir for b in vir if a < b
               if (i % 2 + j % 2) == (a % 2 + b % 2)]
    return singles + doubles


def excitation_fermion_ops(exc):
    """(coeffs, modes, daggers) of G = T - T^dagger for one excitation."""
    if len(exc) == 2:
        i, a = exc
        modes = [(a, i), (i, a)]
        dag = [(True, False), (True, False)]
        co = [1.0, -1.0]
    else:
        i, j, a, b = exc
        modes = [(a, b, j, i), (i, j, b, a)]
        dag = [(True, True, False, False)] * 2
        co = [1.0, -1.0]
    return co, modes, dag


def excitation_rotations(exc):
    """Pauli rotations (x, z, c_g) with exp(theta G) = prod exp(-i c_g theta/2 P)."""
    co, mo, da = excitation_fermion_ops(exc)
    x, z, c = pl.fermion_products_to_pauli(co, mo, da)
    x, z, c = pl.merge(x, z, c, drop=1e-14)
    if np.max(np.abs(c.real), initial=0.0) > 1e-12:
        raise ValueError("excitation generator is not anti-Hermitian")
    d = c.imag
    for k in range(len(x)):
        for l in range(k):
            if not pl.commute(x[k], z[k], x[l], z[l]):
                raise ValueError("excitation strings do not commute")
    return x, z, -2.0 * d


@dataclass
class Problem:
    name: str
    n_qubits: int
    n_elec: int
    bond_dim: int
    eps: float
    h: np.ndarray
    g: np.ndarray
    occ: np.ndarray            # uint8 [n_qubits], 1 = occupied
    ham_x: np.ndarray          # uint64 [K]
    ham_z: np.ndarray          # uint64 [K]
    ham_c: np.ndarray          # float64 [K]
    c0: float
    excitations: list
    rot_x: np.ndarray          # uint64 [M]
    rot_z: np.ndarray          # uint64 [M]
    rot_c: np.ndarray          # float64 [M]  (c_g)
    rot_p: np.ndarray          # int32 [M]    (amplitude index)
    theta: np.ndarray          # float64 [n_theta]
    seeds: dict = field(default_factory=dict)

    @property
    def n_theta(self):
        return len(self.excitations)

    @property
    def n_terms(self):
        return len(self.ham_c)


def make_problem(name, n_qubits, n_elec, bond_dim, eps, seed_int, seed_theta,
                 theta_sigma=0.05):
    n_orb = n_qubits // 2
    h, g = integrals(n_orb, seed_int)
    hx, hz, hc, c0 = hamiltonian_pauli(h, g)
    exc = uccsd_excitations(n_qubits, n_elec)
    rx, rz, rc, rp = [], [], [], []
    for k, e in enumerate(exc):
        x, z, c = excitation_rotations(e)
        rx.append(x); rz.append(z); rc.append(c); rp.append(np.full(len(x), k))
    rng = np.random.default_rng(seed_theta)
    theta = rng.normal(0.0, theta_sigma, len(exc))
    occ = np.zeros(n_qubits, dtype=np.uint8)
    occ[:n_elec] = 1
    return Problem(name=name, n_qubits=n_qubits, n_elec=n_elec, bond_dim=bond_dim, eps=eps,
                   h=h, g=g, occ=occ, ham_x=hx, ham_z=hz, ham_c=hc, c0=c0,
                   excitations=exc,
                   rot_x=np.concatenate(rx).astype(np.uint64),
                   rot_z=np.concatenate(rz).astype(np.uint64),
                   rot_c=np.concatenate(rc), rot_p=np.concatenate(rp).astype(np.int32),
                   theta=theta,
                   seeds={"integrals": seed_int, "theta": seed_theta})
