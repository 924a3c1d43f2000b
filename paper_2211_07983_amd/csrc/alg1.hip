// The paper's memory-efficient back-propagation (Sec. 4, Algorithm 1) with
// one Pauli string per group of the Hamiltonian split (m = N_h).
//
// The gradient is the adjoint of the circuit evolution applied to the adjoint
// of the expectation, 2 H |Psi_M> (Eq. expecgrad).  With H split into groups
// of single strings, the group state phi_k = 2 c_k P_k Psi_M is exactly an
// MPS of the same bonds (a Pauli string is a unitary on each site's physical
// index, which keeps the right-canonical form and the Schmidt values), so no
// compression is needed.  For each string the circuit is walked backwards
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
  if (per_group != 1) fail(MPS_EINVAL, "only one Pauli string per group is supported (strings_per_group = 1)");
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
  const MpsView vphi = view_of(phi.get()), vpsi = view_of(psi.get());
  const dim3 pgrid((dc * dc + 255) / 256, N);
  for (int64_t k = 0; k < p->H.K; ++k) {
    const double ck = p->H.coeff_h[k];
    if (ck == 0.0) continue;
    copy_state(phi.get(), psiM.get(), s);
    copy_state(psi.get(), psiM.get(), s);
    hipLaunchKernelGGL(k_apply_pauli, pgrid, dim3(256), 0, s, vphi, (unsigned long long)p->H.xs[k],
                       (unsigned long long)p->H.zs[k]);
    hipLaunchKernelGGL(k_eta_set, dim3(1), dim3(1), 0, s, etad, 2.0 * ck);
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
