"""Pauli-string algebra and the Jordan-Wigner map (input preparation).

A Pauli string on N <= 63 qubits is stored as two integer bit masks (x, z):
bit q of each mask belongs to qubit q, and the pair per qubit encodes
I=(0,0), X=(1,0), Z=(0,1), Y=(1,1).  The operator a pair denotes is the
canonical P(x, z) = i^{|x & z|} X^x Z^z, which gives exactly Y on a (1,1)
qubit.  Weighted strings carry a complex coefficient.

The paper maps the second-quantised Hamiltonian to a weighted sum of Pauli
strings with the Jordan-Wigner (or Bravyi-Kitaev) transformation before any
simulation (Sec. 2, Eq. expect-val); this module implements the
Jordan-Wigner choice with a_j = (prod_{k<j} Z_k) (X_j + i Y_j) / 2 and
|1> = occupied.  It holds no part of the MPS method itself.
"""
from __future__ import annotations

import numpy as np

_POP = np.bitwise_count


def popcount(a):
    return _POP(np.asarray(a, dtype=np.uint64)).astype(np.int64)


def multiply(x1, z1, c1, x2, z2, c2):
    """Product (c1 P(x1,z1)) (c2 P(x2,z2)) = c P(x1^x2, z1^z2), vectorised.

    X^x1 Z^z1 X^x2 Z^z2 = (-1)^{|z1&x2|} X^{x1^x2} Z^{z1^z2}; the canonical
    i^{|x&z|} factors of the three strings give the remaining power of i.
    """
    x1 = np.asarray(x1, dtype=np.uint64)
    z1 = np.asarray(z1, dtype=np.uint64)
    x2 = np.asarray(x2, dtype=np.uint64)
    z2 = np.asarray(z2, dtype=np.uint64)
    x3 = x1 ^ x2
    z3 = z1 ^ z2
    k = (popcount(x1 & z1) + popcount(x2 & z2) - popcount(x3 & z3)
         + 2 * popcount(z1 & x2)) % 4
    phase = np.array([1, 1j, -1, -1j])[k]
    return x3, z3, np.asarray(c1) * np.asarray(c2) * phase


def ladder(mode, dagger):
    """JW image of a_mode (dagger=False) or a+_mode as two weighted strings."""
    zstr = (1 << mode) - 1
    bit = 1 << mode
    xs = np.array([bit, bit], dtype=np.uint64)
    zs = np.array([zstr, zstr | bit], dtype=np.uint64)
    cs = np.array([0.5, (-0.5j if dagger else 0.5j)])
    return xs, zs, cs


def fermion_products_to_pauli(coeffs, modes, daggers):
    """JW map of sum_t coeffs[t] * prod_k op(modes[t,k], daggers[t,k]).

    ``modes``/``daggers`` have shape (T, k); the product is taken left to
    right as written.  Returns un-merged arrays (x, z, c) of length T*2^k.
    """
    coeffs = np.asarray(coeffs, dtype=np.complex128)
    modes = np.asarray(modes, dtype=np.int64)
    daggers = np.asarray(daggers, dtype=bool)
    T, k = modes.shape
    x = np.zeros(T, dtype=np.uint64)
    z = np.zeros(T, dtype=np.uint64)
    c = coeffs.copy()
    tidx = np.arange(T)
    for col in range(k):
        m = modes[tidx, col]
        d = daggers[tidx, col]
        bit = (np.uint64(1) << m.astype(np.uint64))
        zstr = bit - np.uint64(1)
        # option 0: (1/2) Zstr X_m ; option 1: (+-i/2) Zstr Y_m
        xa = np.stack([bit, bit], axis=1)
        za = np.stack([zstr, zstr | bit], axis=1)
        ca = np.stack([np.full(len(tidx), 0.5 + 0j), np.where(d, -0.5j, 0.5j)], axis=1)
        xn, zn, cn = multiply(x[:, None], z[:, None], c[:, None], xa, za, ca)
        x, z, c = xn.reshape(-1), zn.reshape(-1), cn.reshape(-1)
        tidx = np.repeat(tidx, 2)
    return x, z, c


def merge(x, z, c, drop=1e-12):
    """Sum coefficients of identical strings; drop |c| < drop."""
    x = np.asarray(x, dtype=np.uint64)
    z = np.asarray(z, dtype=np.uint64)
    key = np.stack([x, z], axis=1)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    acc = np.zeros(len(uniq), dtype=np.complex128)
    np.add.at(acc, inv, c)
    keep = np.abs(acc) >= drop
    return uniq[keep, 0], uniq[keep, 1], acc[keep]


def support(x, z):
    """(first, last) qubit of the non-identity part of each string (-1 if none)."""
    m = np.asarray(x, dtype=np.uint64) | np.asarray(z, dtype=np.uint64)
    first = np.full(m.shape, -1, dtype=np.int64)
    last = np.full(m.shape, -1, dtype=np.int64)
    nz = m != 0
    mm = m[nz]
    low = mm & (~mm + np.uint64(1))
    first[nz] = np.log2(low.astype(np.float64)).round().astype(np.int64)
    # highest set bit
    hb = np.zeros(mm.shape, dtype=np.int64)
    t = mm.copy()
    for s in (32, 16, 8, 4, 2, 1):
        big = t >= (np.uint64(1) << np.uint64(s))
        hb[big] += s
        t[big] >>= np.uint64(s)
    last[nz] = hb
    return first, last


def commute(x1, z1, x2, z2):
    """True iff P(x1,z1) and P(x2,z2) commute (symplectic product is even)."""
    return (int(popcount(np.uint64(x1) & np.uint64(z2)))
            + int(popcount(np.uint64(z1) & np.uint64(x2)))) % 2 == 0


def label(x, z, n):
    out = []
    for q in range(n):
        xb = (int(x) >> q) & 1
        zb = (int(z) >> q) & 1
        out.append("IZXY"[xb * 2 + zb])
    return "".join(out)
