// The paper's memory-efficient back-propagation (Sec. 4, Algorithm 1) with
// the Hamiltonian split into groups of consecutive Pauli strings.
//
// The gradient is the adjoint of the circuit evolution applied to the adjoint
// of the expectation, 2 H |Psi_M> (Eq. expecgrad).  With one string per group
// the group state phi_k = 2 c_k P_k Psi_M is exactly an MPS of the same bonds
// (a Pauli string is a unitary on each site's physical index, which keeps the
// right-canonical form and the Schmidt values), so no compression is needed;
// with several, phi_j is their direct sum compressed to the plan's
// truncation (k_compress).  For each group the circuit is walked backwards
// with two states: Psi <- U_g^dagger Psi, dE/dphi_g += Re <phi| dU_g |Psi>,
// phi <- U_g^dagger phi, both through the forward pass's gate update
// (truncation to D, eps).  The update renormalises its output; Psi is a state
// and stays normalised, phi is a cotangent and is carried as eta * phi^ with
// eta multiplied by the kept norm of every truncation.  The strings'
// contributions add up; dE/dtheta_p sums c_g dE/dphi_g over the gates of p.
#include <complex>
#include <cstring>
#include <memory>
#include <vector>

#include "plan_impl.h"

// P(x, z) = i^{|x & z|} X^x Z^z on every site of st: on site n,
// P|i> = o_i |i ^ x_n> with o_0 = i^{x_n z_n} and o_1 = o_0 (-1)^{z_n}.
// Grid: (ceil(dcap^2 / 256), N); one thread per (alpha, beta) of a site.
__global__ __launch_bounds__(256) void k_apply_pauli(MpsView st, unsigned long long x, unsigned long long z) {
  const int n = blockIdx.y;
  const int a = st.dims[n], b = st.dims[n + 1];
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int al = e / st.dcap, be = e - al * st.dcap;
  if (al >= a || be >= b) return;
  zd* B = st.site(n);
  zd* p0 = B + ((size_t)al * 2 + 0) * st.dcap + be;
  zd* p1 = B + ((size_t)al * 2 + 1) * st.dcap + be;
  const zd v0 = *p0, v1 = *p1;
  const int xb = (int)((x >> n) & 1ull), zb = (int)((z >> n) & 1ull);
  const zd o0 = (xb & zb) ? zmk(0.0, 1.0) : zmk(1.0, 0.0);
  const zd o1 = zb ? zscale(o0, -1.0) : o0;
  const zd w0 = zmul(o0, v0), w1 = zmul(o1, v1);
  if (xb) {
    *p0 = w1;
    *p1 = w0;
  } else {
    *p0 = w0;
    *p1 = w1;
  }
}

// <phi| O_{n,n+1} |psi> for a 4x4 operator O (rows and columns 2 i_n + i_{n+1})
// between two MPS of the same qubit count and capacity.  One work-group:
// the mixed left environment through sites < n, the mixed right environment
// through sites > n+1, and the two-site centre, each phase a strided loop over
// its outputs.  work: 26 dcap^2 complex entries.  acc[0] += eta[0] * Re(the
// overlap).
__global__ __launch_bounds__(256) void k_overlap_op(MpsView phi, MpsView psi, int n, const zd* op, zd* work,
                                                    const double* eta, double* acc) {
  const int t = threadIdx.x, dc = psi.dcap, N = psi.N;
  const size_t dd = (size_t)dc * dc;
  zd* L = work;
  zd* T = work + dd;            // [2][dc][dc]
  zd* R = work + 3 * dd;
  zd* Xn = work + 4 * dd;       // next environment
  zd* Tp = work + 5 * dd;       // [a][4][b] psi centre with O applied
  zd* Tf = work + 9 * dd;       // [a][4][b] phi centre
  zd* Th = work + 13 * dd;      // [a][4][b] psi centre
  zd* Z = work + 17 * dd;       // [a_phi][4][b_psi]
  zd* X = work + 21 * dd;       // [a_phi][4][b_psi]
  __shared__ double red[2][256];
  auto Bf = [&](int k, int al, int i, int be) { return phi.site(k)[((size_t)al * 2 + i) * dc + be]; };
  auto Bp = [&](int k, int al, int i, int be) { return psi.site(k)[((size_t)al * 2 + i) * dc + be]; };
  // left environment L[a_phi][a_psi] (row stride dc)
  if (t == 0) L[0] = zmk(1.0, 0.0);
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const int af = phi.dims[k], bf = phi.dims[k + 1], ap = psi.dims[k], bp = psi.dims[k + 1];
    for (int e = t; e < 2 * af * bp; e += 256) {
      const int i = e / (af * bp), r = e - i * af * bp, x = r / bp, y = r - x * bp;
      zd acc = zmk(0.0, 0.0);
      for (int q = 0; q < ap; ++q) acc = zfma(L[(size_t)x * dc + q], Bp(k, q, i, y), acc);
      T[(size_t)i * dd + (size_t)x * dc + y] = acc;
    }
    __syncthreads();
    for (int e = t; e < bf * bp; e += 256) {
      const int x = e / bp, y = e - x * bp;
      zd acc = zmk(0.0, 0.0);
      for (int i = 0; i < 2; ++i)
        for (int q = 0; q < af; ++q) acc = zfma(zconj(Bf(k, q, i, x)), T[(size_t)i * dd + (size_t)q * dc + y], acc);
      Xn[(size_t)x * dc + y] = acc;
    }
    __syncthreads();
    for (int e = t; e < bf * bp; e += 256) {
      const int x = e / bp, y = e - x * bp;
      L[(size_t)x * dc + y] = Xn[(size_t)x * dc + y];
    }
    __syncthreads();
  }
  // right environment R[b_phi][b_psi]
  if (t == 0) R[0] = zmk(1.0, 0.0);
  __syncthreads();
  for (int k = N - 1; k > n + 1; --k) {
    const int af = phi.dims[k], bf = phi.dims[k + 1], ap = psi.dims[k], bp = psi.dims[k + 1];
    for (int e = t; e < 2 * bf * ap; e += 256) {
      const int i = e / (bf * ap), r = e - i * bf * ap, x = r / ap, y = r - x * ap;
      zd acc = zmk(0.0, 0.0);
      for (int q = 0; q < bp; ++q) acc = zfma(R[(size_t)x * dc + q], Bp(k, y, i, q), acc);
      T[(size_t)i * dd + (size_t)x * dc + y] = acc;
    }
    __syncthreads();
    for (int e = t; e < af * ap; e += 256) {
      const int x = e / ap, y = e - x * ap;
      zd acc = zmk(0.0, 0.0);
      for (int i = 0; i < 2; ++i)
        for (int q = 0; q < bf; ++q) acc = zfma(zconj(Bf(k, x, i, q)), T[(size_t)i * dd + (size_t)q * dc + y], acc);
      Xn[(size_t)x * dc + y] = acc;
    }
    __syncthreads();
    for (int e = t; e < af * ap; e += 256) {
      const int x = e / ap, y = e - x * ap;
      R[(size_t)x * dc + y] = Xn[(size_t)x * dc + y];
    }
    __syncthreads();
  }
  // centre: Th[a][2x+y][b] = sum_m B_n[a,x,m] B_{n+1}[m,y,b] for both states
  const int afn = phi.dims[n], bfn = phi.dims[n + 2], mf = phi.dims[n + 1];
  const int apn = psi.dims[n], bpn = psi.dims[n + 2], mp = psi.dims[n + 1];
  for (int e = t; e < 4 * apn * bpn; e += 256) {
    const int a = e / (4 * bpn), r = e - a * 4 * bpn, pq = r / bpn, b = r - pq * bpn;
    zd acc = zmk(0.0, 0.0);
    for (int m = 0; m < mp; ++m) acc = zfma(Bp(n, a, pq >> 1, m), Bp(n + 1, m, pq & 1, b), acc);
    Th[((size_t)a * 4 + pq) * dc + b] = acc;
  }
  for (int e = t; e < 4 * afn * bfn; e += 256) {
    const int a = e / (4 * bfn), r = e - a * 4 * bfn, pq = r / bfn, b = r - pq * bfn;
    zd acc = zmk(0.0, 0.0);
    for (int m = 0; m < mf; ++m) acc = zfma(Bf(n, a, pq >> 1, m), Bf(n + 1, m, pq & 1, b), acc);
    Tf[((size_t)a * 4 + pq) * dc + b] = acc;
  }
  __syncthreads();
  for (int e = t; e < 4 * apn * bpn; e += 256) {
    const int a = e / (4 * bpn), r = e - a * 4 * bpn, pq = r / bpn, b = r - pq * bpn;
    zd acc = zmk(0.0, 0.0);
    for (int q = 0; q < 4; ++q) acc = zfma(op[pq * 4 + q], Th[((size_t)a * 4 + q) * dc + b], acc);
    Tp[((size_t)a * 4 + pq) * dc + b] = acc;
  }
  __syncthreads();
  // X[a_phi][p][b_psi] = sum_{a_psi} L[a_phi][a_psi] Tp[a_psi][p][b_psi]
  // Z[a_phi][p][b_psi] = sum_{b_phi} conj(Tf[a_phi][p][b_phi]) R[b_phi][b_psi]
  for (int e = t; e < 4 * afn * bpn; e += 256) {
    const int a = e / (4 * bpn), r = e - a * 4 * bpn, pq = r / bpn, b = r - pq * bpn;
    zd x = zmk(0.0, 0.0), zz = zmk(0.0, 0.0);
    for (int q = 0; q < apn; ++q) x = zfma(L[(size_t)a * dc + q], Tp[((size_t)q * 4 + pq) * dc + b], x);
    for (int q = 0; q < bfn; ++q) zz = zfma(zconj(Tf[((size_t)a * 4 + pq) * dc + q]), R[(size_t)q * dc + b], zz);
    X[((size_t)a * 4 + pq) * dc + b] = x;
    Z[((size_t)a * 4 + pq) * dc + b] = zz;
  }
  __syncthreads();
  double re = 0.0, im = 0.0;
  for (int e = t; e < 4 * afn * bpn; e += 256) {
    const int a = e / (4 * bpn), r = e - a * 4 * bpn, pq = r / bpn, b = r - pq * bpn;
    const zd v = zmul(Z[((size_t)a * 4 + pq) * dc + b], X[((size_t)a * 4 + pq) * dc + b]);
    re += v.x;
    im += v.y;
  }
  red[0][t] = re;
  red[1][t] = im;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      red[0][t] += red[0][t + w];
      red[1][t] += red[1][t + w];
    }
    __syncthreads();
  }
  if (t == 0) acc[0] += eta[0] * red[0][0];
}

// eta <- v (start of a walk) and eta <- eta * nu after each truncation of phi
// (nu: the kept norm the SVD records in gdmeta[0]).
__global__ void k_eta_set(double* eta, double v) { eta[0] = v; }
__global__ void k_eta_scale(double* eta, const double* gdmeta) { eta[0] *= gdmeta[0]; }

// Sums of four doubles over the 256 threads, returned to every thread.
__device__ inline void block_sum4(double v[4], double (*red)[256]) {
  const int t = threadIdx.x;
  for (int q = 0; q < 4; ++q) red[q][t] = v[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w)
      for (int q = 0; q < 4; ++q) red[q][t] += red[q][t + w];
    __syncthreads();
  }
  for (int q = 0; q < 4; ++q) v[q] = red[q][0];
  __syncthreads();
}

// Compression of a group state phi_j = sum_k c_k P_k |psi> (Sec. 4, H split
// into groups) to bond dimension <= dmax, one work-group: the direct sum of
// the K Pauli images (block-diagonal bonds, the first site concatenated along
// its right bond and weighted by c_k, the last stacked along its left bond);
// QR from the left (Gram-Schmidt with a second orthogonalisation pass); SVDs
// from the right (one-sided Jacobi on M^H with the rotations accumulated),
// keeping r = min(dmax, #{s_i / |s| > eps}) >= 1 values; then the same two
// sweeps again without truncation, so that the stored Schmidt values are
// exact.  Output: phi^ = the normalised result in right-canonical form with
// its Schmidt values (capacity phi.dcap), eta[0] = its norm.  ws: the wide
// sites [N][Dw][2][Dw] followed by (8 Dw^2 + N Dw) complex scratch entries,
// Dw = K psi.dcap <= 128.
__global__ __launch_bounds__(256) void k_compress(MpsView psi, const unsigned long long* xs,
                                                  const unsigned long long* zs, const double* cs, int K, int dmax,
                                                  double eps, MpsView phi, zd* ws, double* eta, GateStats* stats) {
  const int t = threadIdx.x, N = psi.N, dc = psi.dcap, Dw = K * dc;
  __shared__ int wd[65];
  __shared__ double sv[128];
  __shared__ int perm[128];
  __shared__ int sh_rot, sh_r;
  __shared__ double red[4][256];
  zd* S = ws;
  const size_t nS = (size_t)N * Dw * 2 * Dw;
  zd* Qm = ws + nS;                        // [Dw cols][2 Dw rows]
  zd* Rm = Qm + (size_t)2 * Dw * Dw;       // [Dw][Dw] row-major
  zd* Gm = Rm + (size_t)Dw * Dw;           // [Dw cols][2 Dw rows]
  zd* Vm = Gm + (size_t)2 * Dw * Dw;       // [Dw cols][Dw rows]
  zd* Tm = Vm + (size_t)Dw * Dw;           // [Dw][2][Dw] scratch site ... shares the next block
  double* lamw = (double*)(Tm + (size_t)2 * Dw * Dw);   // [N][Dw]
  auto SI = [&](int n, int al, int i, int be) -> zd& { return S[(((size_t)n * Dw + al) * 2 + i) * Dw + be]; };
  auto TI = [&](int al, int i, int be) -> zd& { return Tm[((size_t)al * 2 + i) * Dw + be]; };
  // ---- direct sum
  for (size_t e = t; e < nS; e += 256) S[e] = zmk(0.0, 0.0);
  if (t == 0) {
    wd[0] = 1;
    wd[N] = 1;
    for (int n = 1; n < N; ++n) wd[n] = K * psi.dims[n];
  }
  __syncthreads();
  for (int e = t; e < N * K * dc * dc; e += 256) {
    const int n = e / (K * dc * dc), r0 = e - n * K * dc * dc, k = r0 / (dc * dc), r1 = r0 - k * dc * dc;
    const int al = r1 / dc, be = r1 - al * dc;
    const int a = psi.dims[n], b = psi.dims[n + 1];
    if (al >= a || be >= b) continue;
    const int ol = n == 0 ? 0 : k * a, orr = n == N - 1 ? 0 : k * b;
    const int xb = (int)((xs[k] >> n) & 1ull), zb = (int)((zs[k] >> n) & 1ull);
    const zd o0 = (xb & zb) ? zmk(0.0, 1.0) : zmk(1.0, 0.0);
    const zd o1 = zb ? zscale(o0, -1.0) : o0;
    const double w = n == 0 ? cs[k] : 1.0;
    const zd* B = psi.site(n);
    const zd v0 = zscale(zmul(o0, B[((size_t)al * 2 + 0) * dc + be]), w);
    const zd v1 = zscale(zmul(o1, B[((size_t)al * 2 + 1) * dc + be]), w);
    SI(n, ol + al, 0 ^ xb, orr + be) = v0;
    SI(n, ol + al, 1 ^ xb, orr + be) = v1;
  }
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    // ---- QR from the left: A_n = Q R, A_n <- Q, A_{n+1} <- R A_{n+1}
    for (int n = 0; n + 1 < N; ++n) {
      const int a = wd[n], b = wd[n + 1], c2 = wd[n + 2], m = 2 * a;
      for (int e = t; e < b * b; e += 256) Rm[e / b * Dw + e % b] = zmk(0.0, 0.0);
      for (int j = 0; j < b; ++j) {
        zd* q = Qm + (size_t)j * 2 * Dw;
        for (int r = t; r < m; r += 256) q[r] = SI(n, r >> 1, r & 1, j);
        __syncthreads();
        for (int rep = 0; rep < 2; ++rep)
          for (int l = 0; l < j; ++l) {
            const zd* ql = Qm + (size_t)l * 2 * Dw;
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            for (int r = t; r < m; r += 256) {
              const zd u = zmul(zconj(ql[r]), q[r]);
              v[0] += u.x;
              v[1] += u.y;
            }
            block_sum4(v, red);
            const zd pr = zmk(v[0], v[1]);
            for (int r = t; r < m; r += 256) q[r] = zsub(q[r], zmul(pr, ql[r]));
            if (t == 0) Rm[(size_t)l * Dw + j] = zadd(Rm[(size_t)l * Dw + j], pr);
            __syncthreads();
          }
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int r = t; r < m; r += 256) v[0] += zabs2(q[r]);
        block_sum4(v, red);
        const double nrm = sqrt(v[0]);
        for (int r = t; r < m; r += 256) q[r] = nrm > 0.0 ? zscale(q[r], 1.0 / nrm) : zmk(0.0, 0.0);
        if (t == 0) Rm[(size_t)j * Dw + j] = zmk(nrm, 0.0);
        __syncthreads();
      }
      for (int e = t; e < m * b; e += 256) {
        const int r = e / b, j = e - r * b;
        SI(n, r >> 1, r & 1, j) = Qm[(size_t)j * 2 * Dw + r];
      }
      for (int e = t; e < b * 2 * c2; e += 256) {
        const int be = e / (2 * c2), r = e - be * 2 * c2, i = r / c2, ga = r - i * c2;
        zd acc = zmk(0.0, 0.0);
        for (int q = be; q < b; ++q) acc = zfma(Rm[(size_t)be * Dw + q], SI(n + 1, q, i, ga), acc);
        TI(be, i, ga) = acc;
      }
      __syncthreads();
      for (int e = t; e < b * 2 * c2; e += 256) {
        const int be = e / (2 * c2), r = e - be * 2 * c2, i = r / c2, ga = r - i * c2;
        SI(n + 1, be, i, ga) = TI(be, i, ga);
      }
      __syncthreads();
    }
    // ---- SVDs from the right: A_n = U s Vh, A_n <- Vh_r, A_{n-1} <- A_{n-1} U_r s_r
    for (int n = N - 1; n >= 1; --n) {
      const int a = wd[n], b = wd[n + 1], m2 = 2 * b, al0 = wd[n - 1];
      // G = A_n^H: column p holds conj(row p of A_n), row c = i b + gamma
      for (int e = t; e < a * m2; e += 256) {
        const int p = e / m2, c = e - p * m2;
        Gm[(size_t)p * 2 * Dw + c] = zconj(SI(n, p, c / b, c % b));
      }
      for (int e = t; e < a * a; e += 256) Vm[(size_t)(e / a) * Dw + e % a] = zmk(e / a == e % a ? 1.0 : 0.0, 0.0);
      __syncthreads();
      // pairs below 1e-28 |M|_F^2 are negligible columns and are left alone
      double fv[4] = {0.0, 0.0, 0.0, 0.0};
      for (int e = t; e < a * m2; e += 256) fv[0] += zabs2(Gm[(size_t)(e / m2) * 2 * Dw + e % m2]);
      block_sum4(fv, red);
      const double floor_g = 1e-28 * fv[0];
      bool converged = false;
      for (int sweep = 0; sweep < 60; ++sweep) {
        if (t == 0) sh_rot = 0;
        __syncthreads();
        for (int p = 0; p + 1 < a; ++p)
          for (int q = p + 1; q < a; ++q) {
            zd* gp = Gm + (size_t)p * 2 * Dw;
            zd* gq = Gm + (size_t)q * 2 * Dw;
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            for (int c = t; c < m2; c += 256) {
              v[0] += zabs2(gp[c]);
              v[1] += zabs2(gq[c]);
              const zd u = zmul(zconj(gp[c]), gq[c]);
              v[2] += u.x;
              v[3] += u.y;
            }
            block_sum4(v, red);
            const double g = sqrt(v[2] * v[2] + v[3] * v[3]);
            if (g > 1e-15 * sqrt(v[0] * v[1]) && g > floor_g && g > 1e-300) {
              const double zeta = (v[1] - v[0]) / (2.0 * g);
              const double tt = fabs(zeta) > 1e150 ? 0.5 / zeta
                                                   : (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
              const double cc = 1.0 / sqrt(1.0 + tt * tt), ss = cc * tt;
              const zd ph = zmk(v[2] / g, v[3] / g);            // e^{i phi}
              // g_p' = c g_p - s e^{-i phi} g_q,  g_q' = s e^{i phi} g_p + c g_q
              for (int c = t; c < m2; c += 256) {
                const zd x = gp[c], y = gq[c];
                gp[c] = zsub(zscale(x, cc), zscale(zmul(zconj(ph), y), ss));
                gq[c] = zadd(zscale(zmul(ph, x), ss), zscale(y, cc));
              }
              zd* vp = Vm + (size_t)p * Dw;
              zd* vq = Vm + (size_t)q * Dw;
              for (int c = t; c < a; c += 256) {
                const zd x = vp[c], y = vq[c];
                vp[c] = zsub(zscale(x, cc), zscale(zmul(zconj(ph), y), ss));
                vq[c] = zadd(zscale(zmul(ph, x), ss), zscale(y, cc));
              }
              if (t == 0) sh_rot = 1;
            }
            __syncthreads();
          }
        if (!sh_rot) {
          converged = true;
          break;
        }
        __syncthreads();
      }
      // a compression whose Jacobi sweeps did not converge is reported like a
      // gate SVD that did not (the host then fails with MPS_ENOCONV)
      if (!converged && t == 0) atomicAdd(&stats->noconv, 1);
      for (int p = 0; p < a; ++p) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int c = t; c < m2; c += 256) v[0] += zabs2(Gm[(size_t)p * 2 * Dw + c]);
        block_sum4(v, red);
        if (t == 0) sv[p] = sqrt(v[0]);
      }
      if (t == 0) {
        for (int p = 0; p < a; ++p) perm[p] = p;
        for (int p = 0; p < a; ++p) {
          int best = p;
          for (int q = p + 1; q < a; ++q)
            if (sv[perm[q]] > sv[perm[best]]) best = q;
          const int tmp = perm[p];
          perm[p] = perm[best];
          perm[best] = tmp;
        }
        double tot = 0.0;
        for (int p = 0; p < a; ++p) tot += sv[p] * sv[p];
        tot = sqrt(tot);
        int cnt = 0;
        for (int p = 0; p < a; ++p)
          if (tot > 0.0 && sv[perm[p]] / tot > (pass == 0 ? eps : 1e-15)) ++cnt;
        int r = pass == 0 ? (cnt < dmax ? cnt : dmax) : cnt;
        if (r < 1) r = 1;
        double kept = 0.0;
        for (int p = 0; p < r; ++p) kept += sv[perm[p]] * sv[perm[p]];
        kept = sqrt(kept);
        for (int p = 0; p < r; ++p) lamw[(size_t)n * Dw + p] = kept > 0.0 ? sv[perm[p]] / kept : 0.0;
        sh_r = r;
      }
      __syncthreads();
      const int r = sh_r;
      for (int e = t; e < r * m2; e += 256) {
        const int rho = e / m2, c = e - rho * m2, p = perm[rho];
        SI(n, rho, c / b, c % b) = sv[p] > 0.0 ? zscale(zconj(Gm[(size_t)p * 2 * Dw + c]), 1.0 / sv[p]) : zmk(0.0, 0.0);
      }
      for (int e = t; e < al0 * 2 * r; e += 256) {
        const int x = e / (2 * r), rr = e - x * 2 * r, i = rr / r, rho = rr - i * r, p = perm[rho];
        zd acc = zmk(0.0, 0.0);
        for (int be = 0; be < a; ++be) acc = zfma(SI(n - 1, x, i, be), Vm[(size_t)p * Dw + be], acc);
        TI(x, i, rho) = zscale(acc, sv[p]);
      }
      __syncthreads();
      for (int e = t; e < al0 * 2 * r; e += 256) {
        const int x = e / (2 * r), rr = e - x * 2 * r, i = rr / r, rho = rr - i * r;
        SI(n - 1, x, i, rho) = TI(x, i, rho);
      }
      if (t == 0) wd[n] = r;
      __syncthreads();
    }
  }
  // ---- normalise and store in the capacity layout
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int e = t; e < 2 * wd[1]; e += 256) v[0] += zabs2(SI(0, 0, e / wd[1], e % wd[1]));
  block_sum4(v, red);
  const double nrm = sqrt(v[0]);
  for (size_t e = t; e < (size_t)N * phi.dcap * 2 * phi.dcap; e += 256) phi.B[e] = zmk(0.0, 0.0);
  __syncthreads();
  for (int n = 0; n < N; ++n) {
    const int a = wd[n], b = wd[n + 1];
    for (int e = t; e < a * 2 * b; e += 256) {
      const int x = e / (2 * b), rr = e - x * 2 * b, i = rr / b, be = rr - i * b;
      const zd val = SI(n, x, i, be);
      phi.site(n)[((size_t)x * 2 + i) * phi.dcap + be] = n == 0 && nrm > 0.0 ? zscale(val, 1.0 / nrm) : val;
    }
  }
  for (int e = t; e <= N; e += 256) phi.dims[e] = wd[e];
  for (size_t e = t; e < (size_t)(N + 1) * phi.dcap; e += 256) phi.lam[e] = 0.0;
  __syncthreads();
  if (t == 0) {
    phi.lam[0] = 1.0;
    phi.lam[(size_t)N * phi.dcap] = 1.0;
    eta[0] = nrm;
  }
  for (int n = 1; n < N; ++n)
    for (int q = t; q < wd[n]; q += 256) phi.lam[(size_t)n * phi.dcap + q] = lamw[(size_t)n * Dw + q];
}

namespace {

typedef std::complex<double> cplx;

// 4x4 complex matrix of gate g from [G][4][4] device-layout host copies.
void mat_of(const std::vector<zd>& m, int g, cplx Q[16]) {
  for (int e = 0; e < 16; ++e) Q[e] = cplx(m[(size_t)g * 16 + e].x, m[(size_t)g * 16 + e].y);
}

void dagger(const cplx A[16], double out[32]) {
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      const cplx v = std::conj(A[c * 4 + r]);
      out[(r * 4 + c) * 2] = v.real();
      out[(r * 4 + c) * 2 + 1] = v.imag();
    }
}

void matmul(const cplx A[16], const cplx B[16], cplx C[16]) {
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      cplx acc = 0.0;
      for (int k = 0; k < 4; ++k) acc += A[r * 4 + k] * B[k * 4 + c];
      C[r * 4 + c] = acc;
    }
}

// The inverse circuit: gate G-1-g is U_g^dagger, i.e. pre^dagger for a FIXED
// gate and pre^dagger RZZ(-phi) post^dagger for a PARAM gate (same parameter,
// coefficient negated).
void build_inverse(mps_plan* p, const std::vector<zd>& pre, const std::vector<zd>& post) {
  const int G = p->C.G;
  std::vector<int32_t> bond(G), kind(G), param(G);
  std::vector<double> ipre((size_t)G * 32), ipost((size_t)G * 32, 0.0), coeff(G, 0.0);
  for (int g = 0; g < G; ++g) {
    const int k = G - 1 - g;
    bond[k] = p->C.bond_h[g];
    kind[k] = p->C.kind_h[g];
    param[k] = p->C.param_h[g];
    cplx A[16];
    if (kind[k] == 1) {
      mat_of(post, g, A);
      dagger(A, &ipre[(size_t)k * 32]);
      mat_of(pre, g, A);
      dagger(A, &ipost[(size_t)k * 32]);
      coeff[k] = -p->C.coeff_h[g];
    } else {
      mat_of(pre, g, A);
      dagger(A, &ipre[(size_t)k * 32]);
    }
  }
  mps_circuit c{p->N, G, bond.data(), kind.data(), ipre.data(), ipost.data(), param.data(), coeff.data()};
  p->Cinv.upload_from(&c, p->ctx->stream);
  HIPCHK(hipStreamSynchronize(p->ctx->stream));   // the host arrays go out of scope
}

struct StateDel {
  void operator()(mps_state* s) const { delete s; }
};

}  // namespace

void plan_energy_grad_alg1(mps_plan* p, const double* theta, int n_theta, int per_group, double* energy,
                           double* grad, double* gate_grad, mps_stats* stats) {
  mps_ctx* ctx = p->ctx;
  hipStream_t s = ctx->stream;
  if (per_group < 1) fail(MPS_EINVAL, "strings_per_group must be >= 1");
  if (per_group > 1 && per_group * p->state->dcap > 128)
    fail(MPS_EINVAL, "strings_per_group times the bond capacity must be <= 128");
  if (n_theta != p->n_theta) fail(MPS_EINVAL, "n_theta does not match the circuit");
  if (n_theta > 0 && !theta) fail(MPS_EINVAL, "NULL theta");
  validate_theta(theta, n_theta);
  const int N = p->N, G = p->C.G;
  double* th = (double*)p->theta.ensure((size_t)std::max(1, n_theta) * sizeof(double));
  if (n_theta > 0) HIPCHK(hipMemcpyAsync(th, theta, (size_t)n_theta * sizeof(double), hipMemcpyHostToDevice, s));
  // host copies of the gate matrices (device layout [G][16] complex)
  std::vector<zd> pre((size_t)G * 16), post((size_t)G * 16);
  if (G > 0) {
    HIPCHK(hipMemcpyAsync(pre.data(), p->C.tab.pre, pre.size() * sizeof(zd), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(post.data(), p->C.tab.post, post.size() * sizeof(zd), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  if (!p->cinv_built) {
    build_inverse(p, pre, post);
    p->cinv_built = true;
  }
  std::unique_ptr<mps_state, StateDel> psiM(plan_new_state(ctx, N, p->trunc, nullptr));
  std::unique_ptr<mps_state, StateDel> psi(plan_new_state(ctx, N, p->trunc, nullptr));
  std::unique_ptr<mps_state, StateDel> phi(plan_new_state(ctx, N, p->trunc, nullptr));
  const int dc = psiM->dcap;
  // forward pass and energy
  init_product(psiM.get(), (const uint8_t*)p->state->occ.p);
  ctx->ensure_gate_work(dc, p->trunc, p->opts.max_sweeps);
  ctx->reset_stats();
  run_gates(psiM.get(), p->C, th, 0, G, GATE_TAPE);
  run_energy(psiM.get(), p->H);
  double ev[3];
  HIPCHK(hipMemcpyAsync(ev, ctx->sb.energy, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  read_stats(ctx, stats, G);   // synchronises
  // reverse walks, one per string; the walk runs on the stream without host
  // synchronisation: eta and dE/dphi_g live on the device
  zd* work = (zd*)p->alg1_work.ensure((size_t)26 * dc * dc * sizeof(zd));
  double* etad = (double*)p->alg1_op.ensure(((size_t)std::max(1, G) + 1) * sizeof(double));
  double* gphid = etad + 1;
  zd* dq = (zd*)p->alg1_dq.ensure((size_t)std::max(1, G) * 16 * sizeof(zd));
  std::vector<zd> dqh((size_t)std::max(1, G) * 16, zmk(0.0, 0.0));
  for (int g = 0; g < G; ++g) {
    if (p->C.kind_h[g] != 1) continue;
    // dU/dphi = post (-i ZZ / 2) RZZ(phi) pre
    const double ph = p->C.coeff_h[g] * theta[p->C.param_h[g]];
    const cplx e = std::exp(cplx(0.0, -0.5 * ph));
    const cplx d[4] = {cplx(0.0, -0.5) * e, cplx(0.0, 0.5) * std::conj(e), cplx(0.0, 0.5) * std::conj(e),
                       cplx(0.0, -0.5) * e};
    cplx P[16], Q[16], D[16] = {}, T1[16], dQ[16];
    mat_of(post, g, P);
    mat_of(pre, g, Q);
    for (int i = 0; i < 4; ++i) D[i * 4 + i] = d[i];
    matmul(D, Q, T1);
    matmul(P, T1, dQ);
    for (int i = 0; i < 16; ++i) dqh[(size_t)g * 16 + i] = zmk(dQ[i].real(), dQ[i].imag());
  }
  HIPCHK(hipMemcpyAsync(dq, dqh.data(), dqh.size() * sizeof(zd), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(gphid, 0, (size_t)std::max(1, G) * sizeof(double), s));
  const MpsView vphi = view_of(phi.get()), vpsi = view_of(psi.get()), vpsiM = view_of(psiM.get());
  const dim3 pgrid((dc * dc + 255) / 256, N);
  // groups of several strings: the strings' masks and weights 2 c_k on the
  // device, and the compression workspace
  const int64_t K = p->H.K;
  unsigned long long* xsd = nullptr;
  unsigned long long* zsd = nullptr;
  double* csd = nullptr;
  zd* cws = nullptr;
  std::vector<double> c2(std::max<int64_t>(1, K));
  if (per_group > 1 && K > 0) {
    for (int64_t k = 0; k < K; ++k) c2[k] = 2.0 * p->H.coeff_h[k];
    char* tb = (char*)p->alg1_terms.ensure((size_t)K * (2 * sizeof(unsigned long long) + sizeof(double)));
    xsd = (unsigned long long*)tb;
    zsd = xsd + K;
    csd = (double*)(zsd + K);
    HIPCHK(hipMemcpyAsync(xsd, p->H.xs.data(), (size_t)K * sizeof(unsigned long long), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(zsd, p->H.zs.data(), (size_t)K * sizeof(unsigned long long), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(csd, c2.data(), (size_t)K * sizeof(double), hipMemcpyHostToDevice, s));
    const size_t Dw = (size_t)per_group * dc;
    cws = (zd*)p->alg1_cws.ensure(((size_t)N * Dw * 2 * Dw + 8 * Dw * Dw + (size_t)N * Dw) * sizeof(zd));
  }
  const int64_t n_groups = per_group > 1 ? (K + per_group - 1) / per_group : K;
  for (int64_t grp = 0; grp < n_groups; ++grp) {
    copy_state(psi.get(), psiM.get(), s);
    if (per_group > 1) {
      const int64_t k0 = grp * per_group;
      const int kj = (int)std::min<int64_t>(per_group, K - k0);
      hipLaunchKernelGGL(k_compress, dim3(1), dim3(256), 0, s, vpsiM, (const unsigned long long*)(xsd + k0),
                         (const unsigned long long*)(zsd + k0), (const double*)(csd + k0), kj, p->trunc.d_max,
                         p->trunc.eps, vphi, cws, etad, ctx->gw.stats);
      // A group whose strings cancel to rounding noise (norm eta below 1e-14
      // of its weights sum |2 c_k|) contributes nothing; its walk is skipped,
      // which also keeps an exactly cancelling group (eta = 0, a zero state
      // whose normalisation has no meaning) out of the gradient.
      double eta_h = 0.0, wsum = 0.0;
      for (int k = 0; k < kj; ++k) wsum += std::fabs(c2[k0 + k]);
      HIPCHK(hipMemcpyAsync(&eta_h, etad, sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (!(eta_h > 1e-14 * wsum)) continue;
    } else {
      const double ck = p->H.coeff_h[grp];
      if (ck == 0.0) continue;
      copy_state(phi.get(), psiM.get(), s);
      hipLaunchKernelGGL(k_apply_pauli, pgrid, dim3(256), 0, s, vphi, (unsigned long long)p->H.xs[grp],
                         (unsigned long long)p->H.zs[grp]);
      hipLaunchKernelGGL(k_eta_set, dim3(1), dim3(1), 0, s, etad, 2.0 * ck);
    }
    HIPCHK(hipGetLastError());
    for (int g = G - 1; g >= 0; --g) {
      const int gi = G - 1 - g, n = p->C.bond_h[g];
      run_gates(psi.get(), p->Cinv, th, gi, gi + 1, GATE_TAPE);
      if (p->C.kind_h[g] == 1)
        hipLaunchKernelGGL(k_overlap_op, dim3(1), dim3(256), 0, s, vphi, vpsi, n, (const zd*)(dq + (size_t)g * 16),
                           work, (const double*)etad, gphid + g);
      run_gates(phi.get(), p->Cinv, th, gi, gi + 1, GATE_TAPE);
      hipLaunchKernelGGL(k_eta_scale, dim3(1), dim3(1), 0, s, etad, (const double*)ctx->gw.gdmeta);
    }
    HIPCHK(hipGetLastError());
  }
  std::vector<double> gphi(std::max(1, G), 0.0);
  HIPCHK(hipMemcpyAsync(gphi.data(), gphid, gphi.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  read_stats(ctx, nullptr, 0);   // fails on a barrier timeout or a non-converged SVD of the walks
  *energy = ev[0];
  if (n_theta > 0) {
    std::vector<double> gth(n_theta, 0.0);
    for (int g = 0; g < G; ++g)
      if (p->C.kind_h[g] == 1) gth[p->C.param_h[g]] += p->C.coeff_h[g] * gphi[g];
    std::memcpy(grad, gth.data(), (size_t)n_theta * sizeof(double));
  }
  if (gate_grad && G > 0) std::memcpy(gate_grad, gphi.data(), (size_t)G * sizeof(double));
}
