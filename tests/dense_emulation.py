"""Brute-force references on 2^N state vectors for the truncating regime.

A truncation of a canonical MPS across one cut keeps the state's leading
Schmidt components across that cut (Sec. 3, the two-qubit gate update: the
singular values of the weighted two-site tensor are the Schmidt values).  A
dense SVD of the 2^N vector, reshaped at the cut, reproduces it.  These
helpers contain no MPS arithmetic: they serve the oracle's pins only."""
import numpy as np


def dense(m):
    """The 2^N amplitudes of an MPS (qubit 0 most significant)."""
    v = m.B[0].reshape(2, -1)
    for n in range(1, m.N):
        a, _, b = m.B[n].shape
        v = (v @ m.B[n].reshape(a, 2 * b)).reshape(-1, b)
    return v.reshape(-1)


def schmidt_cut(v, n_qubits, cut, D, eps, renorm):
    """Keeps r = min(D, #{s / |s| > eps}) >= 1 Schmidt components of v across
    the cut after qubit `cut`; returns (v', r, smallest relative gap at the
    cut, or 1.0 when nothing is cut)."""
    M = v.reshape(2 ** (cut + 1), -1)
    U, s, Vh = np.linalg.svd(M, full_matrices=False)
    sh = s / np.linalg.norm(s)
    r = max(1, min(D, int(np.count_nonzero(sh > eps))))
    gap = (sh[r - 1] - sh[r]) if r < len(s) and sh[r] > 1e-14 else 1.0
    out = (U[:, :r] * s[:r]) @ Vh[:r]
    if renorm:
        out = out / np.linalg.norm(s[:r])
    return out.reshape(-1), r, gap
