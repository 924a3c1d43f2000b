"""Compile Pauli rotations to a nearest-neighbour two-qubit gate list.

Each rotation exp(-i phi/2 P) with support S = [a..b] (s = b - a + 1 >= 2)
becomes, in time order (Sec. 2 V-shaped blocks; Sec. 3 gate fusion and SWAP
routing):

1. a basis change V_q on every q in S with V_q P_q V_q^dagger = Z
   (V = H for X, V = H S^dagger for Y, V = I for Z);
2. a parity ladder over bonds (a,a+1) ... (b-2,b-1): CNOT(q -> q+1) when q+1
   is in the support, SWAP(q, q+1) when q+1 carries identity, so that the
   parity of S \\ {b} ends on position b-1;
3. the parametric gate RZZ(phi) = exp(-i phi/2 Z(x)Z) on bond (b-1, b);
4. the reverse ladder and V_q^dagger.

That is 2s - 3 two-qubit gates per rotation.  Single-qubit gates are fused
into the neighbouring two-qubit gate that touches the qubit next (or, at the
very end, the last one that touched it), and two gates on the same bond with
no gate in between that touches either qubit are merged into one, as long as
at most one of them carries a parameter.  Fusion changes nothing about the
unitary; it fixes the gate list that the simulator consumes.

Gate convention: a 4x4 matrix acts on (qubit n, qubit n+1) of bond n with
row index 2 i'_n + i'_{n+1} and column index 2 i_n + i_{n+1}.  A FIXED gate
is ``pre``; a PARAM gate is ``post @ RZZ(coeff * theta[param]) @ pre``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
HAD = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
SDG = np.diag([1.0, -1.0j]).astype(np.complex128)
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)
ZZ = np.diag([1.0, -1.0, -1.0, 1.0]).astype(np.complex128)
FIXED, PARAM = 0, 1


def rzz(phi):
    e = np.exp(-0.5j * phi)
    return np.diag([e, np.conj(e), np.conj(e), e])


def basis_change(letter):
    if letter == "X":
        return HAD.copy()
    if letter == "Y":
        return HAD @ SDG
    return I2.copy()


@dataclass
class GateList:
    n_qubits: int
    bond: np.ndarray    # int32 [G]
    kind: np.ndarray    # int32 [G]
    pre: np.ndarray     # complex128 [G,4,4]
    post: np.ndarray    # complex128 [G,4,4]
    param: np.ndarray   # int32 [G]  (-1 for FIXED)
    coeff: np.ndarray   # float64 [G]
    n_rot_gates: int    # two-qubit gates before fusion

    @property
    def n_gates(self):
        return len(self.bond)

    def matrix(self, g, theta):
        if self.kind[g] == FIXED:
            return self.pre[g]
        return self.post[g] @ rzz(self.coeff[g] * theta[self.param[g]]) @ self.pre[g]


def _letters(x, z, n):
    out = {}
    for q in range(n):
        xb = (int(x) >> q) & 1
        zb = (int(z) >> q) & 1
        if xb or zb:
            out[q] = "X" if (xb and not zb) else ("Y" if (xb and zb) else "Z")
    return out


def rotation_ops(x, z, coeff, param, n):
    """Unfused op list of one rotation: ('1q', q, U) / ('2q', n, U) / ('rzz', n, c, p)."""
    let = _letters(x, z, n)
    S = sorted(let)
    if len(S) == 0:
        return []
    a, b = S[0], S[-1]
    if a == b:
        raise NotImplementedError("single-qubit rotations do not occur in UCCSD")
    ops = []
    for q in S:
        V = basis_change(let[q])
        if not np.allclose(V, I2):
            ops.append(("1q", q, V))
    ladder = [(q, CNOT if (q + 1) in let else SWAP) for q in range(a, b - 1)]
    for q, U in ladder:
        ops.append(("2q", q, U))
    ops.append(("rzz", b - 1, float(coeff), int(param)))
    for q, U in reversed(ladder):
        ops.append(("2q", q, U))
    for q in S:
        V = basis_change(let[q])
        if not np.allclose(V, I2):
            ops.append(("1q", q, V.conj().T))
    return ops


def compile_rotations(rot_x, rot_z, rot_c, rot_p, n_qubits, fuse=True):
    out = []          # dicts: bond, kind, pre, post, param, coeff
    last = [None] * n_qubits
    pending = [None] * n_qubits
    n_raw = 0

    def absorb_pre(n):
        P0 = pending[n] if pending[n] is not None else I2
        P1 = pending[n + 1] if pending[n + 1] is not None else I2
        pending[n] = None
        pending[n + 1] = None
        return np.kron(P0, P1)

    for x, z, c, p in zip(rot_x, rot_z, rot_c, rot_p):
        for op in rotation_ops(x, z, c, p, n_qubits):
            if op[0] == "1q":
                q, U = op[1], op[2]
                pending[q] = U if pending[q] is None else U @ pending[q]
                continue
            n_raw += 1
            n = op[1]
            P = absorb_pre(n)
            if op[0] == "2q":
                new = dict(bond=n, kind=FIXED, pre=op[2] @ P, post=np.eye(4, dtype=np.complex128),
                           param=-1, coeff=0.0)
            else:
                new = dict(bond=n, kind=PARAM, pre=P, post=np.eye(4, dtype=np.complex128),
                           param=op[3], coeff=op[2])
            j = last[n]
            if fuse and j is not None and last[n + 1] == j and out[j]["bond"] == n:
                old = out[j]
                if old["kind"] == FIXED and new["kind"] == FIXED:
                    old["pre"] = new["pre"] @ old["pre"]
                    continue
                if old["kind"] == FIXED and new["kind"] == PARAM:
                    new["pre"] = new["pre"] @ old["pre"]
                    out[j] = new
                    continue
                if old["kind"] == PARAM and new["kind"] == FIXED:
                    old["post"] = new["pre"] @ old["post"]
                    continue
            out.append(new)
            last[n] = last[n + 1] = len(out) - 1
    for q in range(n_qubits):
        if pending[q] is None:
            continue
        j = last[q]
        if j is None:
            raise ValueError("single-qubit gate on a qubit no two-qubit gate touches")
        g = out[j]
        K = np.kron(pending[q], I2) if q == g["bond"] else np.kron(I2, pending[q])
        if g["kind"] == FIXED:
            g["pre"] = K @ g["pre"]
        else:
            g["post"] = K @ g["post"]
        pending[q] = None
    G = len(out)
    return GateList(
        n_qubits=n_qubits,
        bond=np.array([g["bond"] for g in out], dtype=np.int32),
        kind=np.array([g["kind"] for g in out], dtype=np.int32),
        pre=np.array([g["pre"] for g in out], dtype=np.complex128).reshape(G, 4, 4),
        post=np.array([g["post"] for g in out], dtype=np.complex128).reshape(G, 4, 4),
        param=np.array([g["param"] for g in out], dtype=np.int32),
        coeff=np.array([g["coeff"] for g in out], dtype=np.float64),
        n_rot_gates=n_raw,
    )


def compile_problem(prob, fuse=True):
    return compile_rotations(prob.rot_x, prob.rot_z, prob.rot_c, prob.rot_p, prob.n_qubits,
                             fuse=fuse)
