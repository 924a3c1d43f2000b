"""A crafted case whose truncation cuts through an exactly degenerate pair of
Schmidt values that carries a cotangent (shared by the CPU and GPU tests).

Two qubits start in |00>; one PARAM gate on bond 0 with pre = H (x) H,
post = 1 and coefficient 1 gives RZZ(theta)|++>, whose Schmidt values are
|cos(theta/2)| and |sin(theta/2)|: equal at theta = pi/2.  With D = 1 the
update keeps one of the two, so E_D depends on which, and its fixed-rank
derivative through that SVD does not exist.  H = Z_0 + 0.5 X_1 + 0.3 Y_0 Y_1
is generic enough that the pair carries a cotangent."""
from types import SimpleNamespace

import numpy as np

HAD = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)


def problem():
    pre = np.kron(HAD, HAD)
    gates = SimpleNamespace(n_qubits=2, bond=np.array([0], dtype=np.int32), kind=np.array([1], dtype=np.int32),
                            pre=pre.reshape(1, 4, 4), post=np.eye(4, dtype=np.complex128).reshape(1, 4, 4),
                            param=np.array([0], dtype=np.int32), coeff=np.array([1.0]))
    gates.n_gates = 1
    # qubit q is bit q of the masks; Y = (x, z) = (1, 1)
    ham_x = np.array([0, 2, 3], dtype=np.uint64)
    ham_z = np.array([1, 0, 3], dtype=np.uint64)
    ham_c = np.array([1.0, 0.5, 0.3])
    prob = SimpleNamespace(n_qubits=2, occ=np.zeros(2, dtype=np.uint8), bond_dim=1, eps=1e-12,
                           ham_x=ham_x, ham_z=ham_z, ham_c=ham_c, c0=0.0, theta=np.array([np.pi / 2]))
    prob.n_terms = 3
    prob.n_theta = 1
    return prob, gates
