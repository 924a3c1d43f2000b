"""T3: plain FP64 complex MPS oracle with reverse-mode gradient.

TEST INFRASTRUCTURE: only tests, the smoke entry point and the benchmark's
CPU-baseline leg may import this module; the HIP path never does.

Forward (Sec. 3):
* product state B_n[0, b_n, 0] = 1, all Schmidt vectors [1] (Eq. hf);
* right-canonical form with stored Schmidt values (Eq.
  rightcanonicalcondition); a two-qubit gate Q on bond n follows the Hastings
  update: C = Q . (B_n B_{n+1}), C~ = lambda_{n-1} C, C~ = U s W (SVD with rows
  (alpha_{n-1}, i'_n), columns (i'_{n+1}, alpha_{n+1})), keep
  r = min(D, #{s > eps}) >= 1 values, B~_{n+1} = W_r, B~_n = C W_r^dagger,
  lambda_n = s_r.  Reading of the unstated normalisation: the kept part is
  renormalised, B~_n and lambda_n are divided by nu = ||s_r||.
* <Psi|P|Psi> contracts the one-dimensional network of Eq. paulistringexp
  with the bra copy conjugated; identity environments L^id / R^id let each
  term be swept over its own support only; E = c0 + sum_k c_k <P_k> / Z with
  Z = <Psi|Psi> from the same environments (exact Rayleigh quotient of the
  stored tensors) and a compensated (math.fsum) sum over terms.

Reverse mode (the "local" gradient of Sec. 4 through every site tensor and
SVD, with the complex back-propagation rules of App. A): a cotangent X_bar of
a complex array X is defined by dF = Re <X_bar, dX> = Re sum conj(X_bar) dX,
which is the paper's 2 dF/dX* convention (Eqs. bp1-bp4).  The truncated SVD
is differentiated with its full spectrum: kept singular triplets couple to
discarded ones and to the null space through F_ij = 1/(s_j^2 - s_i^2), plus
the imaginary diagonal gauge term of the complex SVD.  By default no
broadening is applied and a near-degenerate pair that carries a cotangent
raises.  With broaden = eta > 0 every such factor becomes the Lorentzian
d / (d^2 + eta^2), d = s_j^2 - s_i^2 (the regularisation of the SVD
derivative used in the tensor-network AD literature the paper builds on,
e.g. Liao et al. 2019): it is finite for every d, close to 1/d for
|d| >> eta and zero at d = 0, so a (near-)degenerate pair is then dropped
instead of raising.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

# LAPACK driver of the full SVD.  gesvd is the reference.  gesdd, another
# backward-stable SVD, serves only to measure how far the choice of a correct
# SVD moves a result where truncation makes it ill-conditioned.
SVD_DRIVER = "gesvd"

ZZ = np.diag([1.0, -1.0, -1.0, 1.0]).astype(np.complex128)


def site_phases(x, z, n):
    """For qubit n of string (x,z): flip bit and (o_0, o_1) with O[i^x, i] = o_i."""
    xb = (int(x) >> n) & 1
    zb = (int(z) >> n) & 1
    base = (1j) ** (xb * zb)
    return xb, np.array([base, base * (-1.0 if zb else 1.0)])


class SVDDegenerate(RuntimeError):
    pass


class MPS:
    def __init__(self, occ):
        self.N = len(occ)
        self.B = []
        for b in occ:
            t = np.zeros((1, 2, 1), dtype=np.complex128)
            t[0, int(b), 0] = 1.0
            self.B.append(t)
        # lam[k] sits left of site k (lam[0] = boundary, lam[n+1] = bond (n, n+1))
        self.lam = [np.ones(1) for _ in range(self.N + 1)]
        self.discarded = []
        self.ranks = []
        self.degenerate_cuts = 0

    def copy(self):
        m = MPS.__new__(MPS)
        m.N = self.N
        m.B = [b.copy() for b in self.B]
        m.lam = [l.copy() for l in self.lam]
        m.discarded = []
        m.ranks = []
        m.degenerate_cuts = 0
        return m

    def bond_dims(self):
        return [self.B[n].shape[2] for n in range(self.N - 1)]

    # --- S2-S4: two-site gate -------------------------------------------------
    def apply_gate(self, n, Q, D, eps, tape=None, rank=None):
        Bl, Br = self.B[n], self.B[n + 1]
        a, _, m = Bl.shape
        b = Br.shape[2]
        Theta = (Bl.reshape(2 * a, m) @ Br.reshape(m, 2 * b)).reshape(a, 2, 2, b)
        C = np.einsum("xyij,aijb->axyb", Q.reshape(2, 2, 2, 2), Theta)
        Cm = C.reshape(2 * a, 2 * b)
        lam_in = self.lam[n]
        M = (lam_in[:, None, None, None] * C).reshape(2 * a, 2 * b)
        U, s, Wh = sla.svd(M, full_matrices=True, lapack_driver=SVD_DRIVER)
        r = max(1, min(D, int(np.count_nonzero(s > eps)))) if rank is None else int(rank)
        self.ranks.append(r)
        nu = float(np.sqrt(np.sum(s[:r] ** 2)))
        W = Wh[:r]
        newBl = (Cm @ W.conj().T / nu).reshape(a, 2, r)
        self.B[n] = newBl
        self.B[n + 1] = W.reshape(r, 2, b).copy()
        self.lam[n + 1] = s[:r] / nu
        if r < len(s) and s[r] > 0 and (s[r - 1] - s[r]) < 1e-10 * s[0]:
            self.degenerate_cuts += 1
        tot = float(np.sum(s ** 2))
        self.discarded.append(float(np.sum(s[r:] ** 2)) / tot if tot > 0 else 0.0)
        if tape is not None:
            tape.append(dict(n=n, Bl=Bl, Br=Br, lam_in=lam_in, Theta=Theta, Cm=Cm, U=U, s=s,
                             Wh=Wh, r=r, nu=nu, newBl=newBl))

    # --- S5: environments and Pauli expectations ---------------------------------
    def left_env(self, L, n, x=0, z=0):
        B = self.B[n]
        xb, o = site_phases(x, z, n)
        out = 0
        for i in (0, 1):
            out = out + o[i] * (B[:, i ^ xb, :].conj().T @ L @ B[:, i, :])
        return out

    def right_env(self, R, n, x=0, z=0):
        B = self.B[n]
        xb, o = site_phases(x, z, n)
        out = 0
        for i in (0, 1):
            out = out + o[i] * (B[:, i ^ xb, :].conj() @ R @ B[:, i, :].T)
        return out

    def identity_envs(self):
        N = self.N
        L = [None] * (N + 1)
        R = [None] * (N + 1)
        L[0] = np.ones((1, 1), dtype=np.complex128)
        for n in range(N):
            L[n + 1] = self.left_env(L[n], n)
        R[N] = np.ones((1, 1), dtype=np.complex128)
        for n in range(N - 1, -1, -1):
            R[n] = self.right_env(R[n + 1], n)
        return L, R

    def term_values(self, hx, hz, envs=None):
        """Unnormalised <Psi|P_k|Psi> for every term (complex)."""
        L, R = envs if envs is not None else self.identity_envs()
        out = np.zeros(len(hx), dtype=np.complex128)
        for k, (x, z) in enumerate(zip(hx, hz)):
            m = int(x) | int(z)
            if m == 0:
                out[k] = L[self.N][0, 0]
                continue
            a = (m & -m).bit_length() - 1
            b = m.bit_length() - 1
            Lk = L[a]
            for n in range(a, b + 1):
                Lk = self.left_env(Lk, n, x, z)
            out[k] = np.sum(Lk * R[b + 1])
        return out

    def energy(self, hx, hz, hc, c0):
        L, R = self.identity_envs()
        Z = L[self.N][0, 0]
        vals = self.term_values(hx, hz, (L, R)) / Z
        e_re = math.fsum(list(hc * vals.real))
        e_im = math.fsum(list(hc * vals.imag))
        return c0 + e_re, e_im, Z, vals

    # --- S7: site cotangents of E --------------------------------------------------
    def energy_cotangents(self, hx, hz, hc, c0):
        N = self.N
        Lid, Rid = self.identity_envs()
        Z = Lid[N][0, 0].real
        E, _, _, _ = self.energy(hx, hz, hc, c0)
        Bbar = [np.zeros_like(b) for b in self.B]

        def add_site(n, L, R, x, z, w):
            B = self.B[n]
            xb, o = site_phases(x, z, n)
            for i in (0, 1):
                Bbar[n][:, i, :] += w * np.conj(o[i]) * (L @ B[:, i ^ xb, :] @ R.T)

        for x, z, c in zip(hx, hz, hc):
            m = int(x) | int(z)
            a = (m & -m).bit_length() - 1
            b = m.bit_length() - 1
            # full-chain left and right environments of this term
            Lk = [None] * (N + 1)
            Rk = [None] * (N + 1)
            Lk[0] = Lid[0]
            for n in range(N):
                Lk[n + 1] = Lid[n + 1] if n < a else self.left_env(Lk[n], n, x, z)
            Rk[N] = Rid[N]
            for n in range(N - 1, -1, -1):
                Rk[n] = Rid[n] if n > b else self.right_env(Rk[n + 1], n, x, z)
            for n in range(N):
                add_site(n, Lk[n], Rk[n + 1], x, z, 2.0 * c / Z)
        for n in range(N):
            add_site(n, Lid[n], Rid[n + 1], 0, 0, -2.0 * (E - c0) / Z)
        return E, Bbar


def gate_backward(t, Q, dQ, Bbar_l, Bbar_r, lbar, check=1e-10, broaden=0.0):
    """Cotangents of (B_n, B_{n+1}, lambda_{n-1}) and dE/dphi for one gate;
    broaden = eta of the Lorentzian factor (0: the plain 1/d)."""
    Bl, Br, lam_in, Theta, Cm = t["Bl"], t["Br"], t["lam_in"], t["Theta"], t["Cm"]
    U, s, Wh, r, nu, newBl = t["U"], t["s"], t["Wh"], t["r"], t["nu"], t["newBl"]
    a, _, m = Bl.shape
    b = Br.shape[2]
    p = len(s)
    n2 = 2 * b
    W = Wh[:r]
    # S4 adjoint: B~_n = C W_r^dagger / nu, B~_{n+1} = W_r, lambda_n = s_r / nu
    Xbar = Bbar_l.reshape(2 * a, r) / nu
    nubar = -np.vdot(Bbar_l, newBl).real / nu
    Wbar = Bbar_r.reshape(r, n2) + Xbar.conj().T @ Cm
    sbar = np.zeros(p)
    sbar[:r] = lbar / nu
    nubar += -float(np.sum(lbar * s[:r])) / nu ** 2
    sbar[:r] += nubar * s[:r] / nu
    Cbar = Xbar @ W
    # S3 adjoint (full-spectrum complex SVD derivative)
    V = Wh.conj().T
    Vbar = np.zeros((n2, n2), dtype=np.complex128)
    Vbar[:, :r] = Wbar.conj().T
    K = V.conj().T @ Vbar
    sx = np.zeros(n2)
    sx[:p] = s
    A = K - K.conj().T
    scale = s[0] if s[0] > 0 else 1.0
    kscale = float(np.max(np.abs(K))) if K.size else 0.0
    si = s[:, None]
    sj = sx[None, :]
    ii = np.arange(p)[:, None]
    jj = np.arange(n2)[None, :]
    active = (ii != jj) & ~((ii >= r) & (jj >= r))
    num = si * A[:p, :]
    # An exactly degenerate pair leaves E invariant under rotations inside the
    # block, so its A_ij vanishes and the term is dropped; a degenerate pair
    # with a real cotangent has no finite derivative and raises.
    deg = active & (np.abs(sj - si) < check * np.maximum(si, sj))
    if broaden <= 0.0 and np.any(deg & (np.abs(A[:p, :]) > 1e-8 * kscale)):
        raise SVDDegenerate("degenerate singular pair carries a cotangent")
    use = active & ~deg & (num != 0)
    d = sj ** 2 - si ** 2
    if broaden > 0.0:
        den = np.where(use, (d * d + broaden * broaden) / np.where(use, d, 1.0), 1.0)
    else:
        den = np.where(use, d, 1.0)
    Gam = np.where(use, num / den, 0.0).astype(np.complex128)
    for i in range(r):
        Gam[i, i] = sbar[i] - 1j * K[i, i].imag / s[i]
    Mbar = U[:, :p] @ Gam @ Wh
    # S2 adjoint: C~ = lambda C, C = Q Theta, Theta = B_n B_{n+1}
    Cbar = Cbar + lam_in.repeat(2)[:, None] * Mbar
    lbar_in = np.sum((Mbar.conj() * Cm).real.reshape(a, 2 * n2), axis=1)
    Cb4 = Cbar.reshape(a, 2, 2, b)
    Thetabar = np.einsum("xyij,axyb->aijb", Q.conj().reshape(2, 2, 2, 2), Cb4)
    dphi = 0.0
    if dQ is not None:
        dC = np.einsum("xyij,aijb->axyb", dQ.reshape(2, 2, 2, 2), Theta)
        dphi = np.vdot(Cb4, dC).real
    Tb = Thetabar.reshape(2 * a, 2 * b)
    Bbar_l_in = (Tb @ Br.reshape(m, 2 * b).conj().T).reshape(a, 2, m)
    Bbar_r_in = (Bl.reshape(2 * a, m).conj().T @ Tb).reshape(m, 2, b)
    return Bbar_l_in, Bbar_r_in, lbar_in, dphi


def gate_mats(gates, g, theta):
    """(Q, dQ/dphi or None) of gate g."""
    from vqe_inputs.compile import rzz
    if gates.kind[g] == 0:
        return gates.pre[g], None
    phi = gates.coeff[g] * theta[gates.param[g]]
    R = rzz(phi)
    Q = gates.post[g] @ R @ gates.pre[g]
    dQ = gates.post[g] @ (-0.5j * ZZ @ R) @ gates.pre[g]
    return Q, dQ


def forward(prob, gates, theta, D=None, eps=None, start=None, count=None, tape=None,
            snapshots=None, ckpt=None, ranks=None):
    """Run gates [0, count); ``ranks`` optionally freezes the kept rank of each gate."""
    D = prob.bond_dim if D is None else D
    eps = prob.eps if eps is None else eps
    mps = MPS(prob.occ) if start is None else start
    G = gates.n_gates if count is None else count
    for g in range(G):
        if snapshots is not None and ckpt and g % ckpt == 0:
            snapshots.append(mps.copy())
        Q, _ = gate_mats(gates, g, theta)
        mps.apply_gate(int(gates.bond[g]), Q, D, eps, tape, None if ranks is None else ranks[g])
    return mps


def energy(prob, gates, theta, D=None, eps=None, ranks=None):
    mps = forward(prob, gates, theta, D, eps, ranks=ranks)
    E, Eim, Z, _ = mps.energy(prob.ham_x, prob.ham_z, prob.ham_c, prob.c0)
    return E, dict(imag=Eim, Z=Z.real, bonds=mps.bond_dims(), discarded=mps.discarded,
                   ranks=mps.ranks, mps=mps, degenerate_cuts=mps.degenerate_cuts)


def energy_grad(prob, gates, theta, D=None, eps=None, ckpt=64, check=1e-10, broaden=0.0):
    """(E, dE/dtheta, info) by reverse mode with segment checkpoints and recompute;
    broaden = eta of the SVD adjoint's Lorentzian (0: none)."""
    D = prob.bond_dim if D is None else D
    eps = prob.eps if eps is None else eps
    snaps = []
    mps = forward(prob, gates, theta, D, eps, snapshots=snaps, ckpt=ckpt)
    E, Bbar = mps.energy_cotangents(prob.ham_x, prob.ham_z, prob.ham_c, prob.c0)
    N = mps.N
    lbar = [0.0 for _ in mps.lam]
    gphi = np.zeros(gates.n_gates)
    G = gates.n_gates
    for sidx in range(len(snaps) - 1, -1, -1):
        g0 = sidx * ckpt
        g1 = min(G, g0 + ckpt)
        st = snaps[sidx].copy()
        tape = []
        for g in range(g0, g1):
            Q, _ = gate_mats(gates, g, theta)
            st.apply_gate(int(gates.bond[g]), Q, D, eps, tape)
        for g in range(g1 - 1, g0 - 1, -1):
            t = tape[g - g0]
            n = t["n"]
            Q, dQ = gate_mats(gates, g, theta)
            bl, br, li, dphi = gate_backward(t, Q, dQ, Bbar[n], Bbar[n + 1], lbar[n + 1], check, broaden)
            Bbar[n], Bbar[n + 1] = bl, br
            lbar[n + 1] = 0.0
            lbar[n] = lbar[n] + li
            gphi[g] = dphi
        del tape
    grad = np.zeros(len(theta))
    np.add.at(grad, gates.param[gates.kind == 1], gates.coeff[gates.kind == 1] * gphi[gates.kind == 1])
    return E, grad, dict(gphi=gphi, bonds=mps.bond_dims(), discarded=mps.discarded, Bbar=Bbar)
