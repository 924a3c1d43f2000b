"""The synthetic workloads: five configurations and their seeds.

Config c in {1,2,3,5} draws integrals with seed 1000c+1 and theta with seed
1000c+2.  The batched set (c = 4) draws (n_qubits, D) for instance i from
default_rng(4999) and seeds 4000+10i+1 / 4000+10i+2; its electron count is
N/2 (half filling).

``eps`` is the truncation threshold on the Schmidt coefficients of the
normalised state.  The exact-parity default is 1e-12; the paper's own runs use
1e-6 (Sec. 5).
"""
from __future__ import annotations

import functools

import numpy as np

from .compile import compile_problem
from .problem import make_problem

PARITY_EPS = 1e-12
PAPER_EPS = 1e-6

CONFIGS = {
    "c1": dict(n_qubits=8, n_elec=4, bond_dim=16, theta_sigma=0.05, seed=1),
    "c2": dict(n_qubits=14, n_elec=10, bond_dim=64, theta_sigma=0.05, seed=2),
    "c3": dict(n_qubits=24, n_elec=12, bond_dim=128, theta_sigma=0.05, seed=3),
    "c5": dict(n_qubits=40, n_elec=4, bond_dim=256, theta_sigma=0.02, seed=5),
}

DESCRIPTION = {
    "c1": "UCCSD-MPS 8q (4 orbitals, 4 e) D=16",
    "c2": "UCCSD-MPS 14q (7 orbitals, 10 e) D=64",
    "c3": "UCCSD-MPS 24q (12 orbitals, 12 e) D=128",
    "c5": "UCCSD-MPS 40q (20 orbitals, 4 e) D=256",
}


@functools.lru_cache(maxsize=None)
def _cached(name, eps, bond_dim):
    cfg = CONFIGS[name]
    c = cfg["seed"]
    D = cfg["bond_dim"] if bond_dim is None else bond_dim
    prob = make_problem(name, cfg["n_qubits"], cfg["n_elec"], D, eps,
                        1000 * c + 1, 1000 * c + 2, cfg["theta_sigma"])
    gates = compile_problem(prob)
    return prob, gates


def load(name, eps=PARITY_EPS, bond_dim=None):
    """(Problem, GateList) of a named configuration (cached per process)."""
    return _cached(name, float(eps), bond_dim)


def small(n_qubits, n_elec, bond_dim, seed, eps=PARITY_EPS, theta_sigma=0.05):
    """A small seeded instance for tests (same generator, other sizes)."""
    prob = make_problem(f"n{n_qubits}e{n_elec}s{seed}", n_qubits, n_elec, bond_dim, eps,
                        7000 + 10 * seed + 1, 7000 + 10 * seed + 2, theta_sigma)
    return prob, compile_problem(prob)


def batched_instances(count=64):
    rng = np.random.default_rng(4999)
    out = []
    for i in range(count):
        n = int(rng.choice([12, 16, 20, 24]))
        D = int(rng.choice([32, 64, 128]))
        out.append((n, n // 2, D, 4000 + 10 * i + 1, 4000 + 10 * i + 2))
    return out
