"""Seeded inputs beyond the UCCSD workload: circuits of random complex
two-qubit gates (unitaries from the QR factorisation of complex Gaussian
matrices, phases fixed) on random bonds, about 40 % of them parametric
post @ RZZ(c theta_p) @ pre, and Pauli sums of random strings of every kind
with random real coefficients.  The states they make are genuinely complex,
and the strings include odd numbers of Y's, neither of which the molecular
workload exercises.  Input generation only: no part of the MPS method."""
from types import SimpleNamespace

import numpy as np

from vqe_inputs.compile import FIXED, PARAM, GateList


def unitary(rng, n=4):
    z = (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


def circuit(n_qubits, n_gates, n_theta, seed):
    rng = np.random.default_rng(seed)
    bond = rng.integers(0, n_qubits - 1, n_gates).astype(np.int32)
    kind = np.where(rng.random(n_gates) < 0.4, PARAM, FIXED).astype(np.int32)
    kind[:n_theta] = PARAM                      # every parameter appears at least once
    pre = np.array([unitary(rng) for _ in range(n_gates)])
    post = np.array([unitary(rng) if k == PARAM else np.eye(4, dtype=np.complex128) for k in kind])
    param = np.full(n_gates, -1, dtype=np.int32)
    param[:n_theta] = np.arange(n_theta)
    rest = kind[n_theta:] == PARAM
    param[n_theta:][rest] = rng.integers(0, n_theta, int(rest.sum()))
    coeff = np.where(kind == PARAM, rng.choice([-1.0, 0.5, 1.0, 2.0], n_gates), 0.0)
    gl = GateList(n_qubits=n_qubits, bond=bond, kind=kind, pre=pre, post=post, param=param, coeff=coeff,
                  n_rot_gates=n_gates)
    theta = rng.uniform(-np.pi, np.pi, n_theta)
    return gl, theta


def problem(n_qubits, n_terms, bond_dim, eps, seed, n_theta=10, max_weight=None):
    """The fields of a problem that the oracle reads, with a random Pauli sum
    and a random occupation.  max_weight: each string acts on 1..max_weight
    random qubits (on long chains a dense random string has a vanishing
    expectation); None: every qubit independently I, X, Y or Z."""
    rng = np.random.default_rng(seed)
    occ = rng.integers(0, 2, n_qubits).astype(np.uint8)
    if max_weight is None:
        x = rng.integers(0, 2 ** n_qubits, n_terms).astype(np.uint64)
        z = rng.integers(0, 2 ** n_qubits, n_terms).astype(np.uint64)
    else:
        x = np.zeros(n_terms, dtype=np.uint64)
        z = np.zeros(n_terms, dtype=np.uint64)
        for k in range(n_terms):
            for q in rng.choice(n_qubits, int(rng.integers(1, max_weight + 1)), replace=False):
                letter = int(rng.integers(1, 4))           # 1 = X, 2 = Z, 3 = Y
                x[k] |= np.uint64((letter & 1) << int(q))
                z[k] |= np.uint64(((letter >> 1) & 1) << int(q))
    c = rng.normal(size=n_terms)
    ident = (x | z) == 0                         # identity strings belong in c0
    c0 = 0.375 + float(np.sum(c[ident]))
    keep = ~ident
    return SimpleNamespace(n_qubits=n_qubits, occ=occ, ham_x=x[keep], ham_z=z[keep], ham_c=c[keep], c0=c0,
                           bond_dim=bond_dim, eps=eps, n_theta=n_theta)
