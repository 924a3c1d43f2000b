// Pauli-string expectation values on the MPS (arXiv:2211.07983, Sec. 3, Eq.
// paulistringexp) and the energy sum (Sec. 2, Eq. expect-val).
//
// A left transfer through site n with operator O (O[i^x, i] = o_i) is
//   L' = sum_i o_i (B^{i^x})^dagger L B^i,
// done as two GEMMs: Y = L [B^0 | B^1] (a x 2b), then L' = sum over (i, alpha')
// of o_i conj(B^{i^x}[alpha', .]) Y[alpha', i, .] (b x b).  Identity
// environments L^id / R^id let every term be swept over its own support only;
// a term's value is <L, R^id_{b+1}> after its last site, and E = c0 +
// sum_k c_k <P_k> / Z with a Neumaier-compensated sum.
#include "engine.h"

__global__ void k_init_product(MpsView st, const uint8_t* occ) {
  const int n = blockIdx.x;
  const int t = threadIdx.x;
  if (n <= st.N) {
    if (t == 0) st.dims[n] = 1;
    for (int q = t; q < st.dcap; q += blockDim.x) st.lam[(size_t)n * st.dcap + q] = q == 0 ? 1.0 : 0.0;
  }
  if (n < st.N && t < 2) st.site(n)[t * st.dcap] = zmk(occ[n] == t ? 1.0 : 0.0, 0.0);
}

__device__ inline zd* env_ptr(const SweepBuffers& sb, int dc, int slot, int site) {
  return slot < 0 ? sb.Lid + (size_t)site * dc * dc : sb.Lslots + (size_t)slot * dc * dc;
}

// Stage 1 (left): Y_z = L_in [B^0 | B^1]; GEMM column c = i*b + beta.
__global__ __launch_bounds__(256) void k_left_stage1(MpsView st, SweepBuffers sb, int n, const SweepJob* jobs,
                                                     int identity) {
  const int a = st.dims[n], b = st.dims[n + 1];
  const int dc = st.dcap;
  const int z = blockIdx.z;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  if (i0 >= a || j0 >= 2 * b) return;
  const int in_slot = identity ? -1 : jobs[z].in_slot;
  const zd* L = env_ptr(sb, dc, in_slot, n);
  zd* Y = identity ? sb.Yid : sb.Y + (size_t)z * dc * 2 * dc;
  const zd* B = st.site(n);
  auto fa = [&](int r, int k) { return L[(size_t)r * dc + k]; };
  auto fb = [&](int k, int c) {
    const int i = c >= b, be = c - i * b;
    return B[(size_t)k * 2 * dc + i * dc + be];
  };
  zd acc[2][2];
  ztile_acc(a, 2 * b, a, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int r = r0 + x, c = c0 + y;
      if (r < a && c < 2 * b) {
        const int i = c >= b, be = c - i * b;
        Y[(size_t)r * 2 * dc + i * dc + be] = acc[x][y];
      }
    }
}

// Stage 2 (left): L_out[b', b] = sum_{i, a'} o_i conj(B^{i^x}[a', b']) Y[a', i, b].
__global__ __launch_bounds__(256) void k_left_stage2(MpsView st, SweepBuffers sb, int n, const SweepJob* jobs,
                                                     int identity) {
  const int a = st.dims[n], b = st.dims[n + 1];
  const int dc = st.dcap;
  const int z = blockIdx.z;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  if (i0 >= b || j0 >= b) return;
  int xb = 0;
  zd o0 = zmk(1.0, 0.0), o1 = zmk(1.0, 0.0);
  int out_slot = -1;
  if (!identity) {
    xb = jobs[z].xb;
    o0 = jobs[z].o0;
    o1 = jobs[z].o1;
    out_slot = jobs[z].out_slot;
  }
  const zd* Y = identity ? sb.Yid : sb.Y + (size_t)z * dc * 2 * dc;
  const zd* B = st.site(n);
  zd* Lo = env_ptr(sb, dc, out_slot, n + 1);
  auto fa = [&](int r, int k) {
    const int i = k >= a, al = k - i * a;
    const zd v = zconj(B[(size_t)al * 2 * dc + (i ^ xb) * dc + r]);
    return zmul(i ? o1 : o0, v);
  };
  auto fb = [&](int k, int c) {
    const int i = k >= a, al = k - i * a;
    return Y[(size_t)al * 2 * dc + i * dc + c];
  };
  zd acc[2][2];
  ztile_acc(b, b, 2 * a, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int r = r0 + x, c = c0 + y;
      if (r < b && c < b) Lo[(size_t)r * dc + c] = acc[x][y];
    }
}

// Right identity environments: Yr[(i,a'), b] = sum_b' conj(B^i[a', b']) R[b', b];
// R_n[a', a] = sum_{i,b} Yr[(i,a'), b] B^i[a, b].
__global__ __launch_bounds__(256) void k_right_stage1(MpsView st, SweepBuffers sb, int n) {
  const int a = st.dims[n], b = st.dims[n + 1];
  const int dc = st.dcap;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  if (i0 >= 2 * a || j0 >= b) return;
  const zd* R = sb.Rid + (size_t)(n + 1) * dc * dc;
  const zd* B = st.site(n);
  auto fa = [&](int r, int k) {
    const int i = r >= a, al = r - i * a;
    return zconj(B[(size_t)al * 2 * dc + i * dc + k]);
  };
  auto fb = [&](int k, int c) { return R[(size_t)k * dc + c]; };
  zd acc[2][2];
  ztile_acc(2 * a, b, b, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int r = r0 + x, c = c0 + y;
      if (r < 2 * a && c < b) sb.Yid[(size_t)r * dc + c] = acc[x][y];
    }
}

__global__ __launch_bounds__(256) void k_right_stage2(MpsView st, SweepBuffers sb, int n) {
  const int a = st.dims[n], b = st.dims[n + 1];
  const int dc = st.dcap;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  if (i0 >= a || j0 >= a) return;
  const zd* B = st.site(n);
  zd* Ro = sb.Rid + (size_t)n * dc * dc;
  auto fa = [&](int r, int k) {
    const int i = k >= b, be = k - i * b;
    return sb.Yid[(size_t)(i * a + r) * dc + be];
  };
  auto fb = [&](int k, int c) {
    const int i = k >= b, be = k - i * b;
    return B[(size_t)c * 2 * dc + i * dc + be];
  };
  zd acc[2][2];
  ztile_acc(a, a, 2 * b, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int r = r0 + x, c = c0 + y;
      if (r < a && c < a) Ro[(size_t)r * dc + c] = acc[x][y];
    }
}

__global__ void k_set_unit_env(SweepBuffers sb, int dc, int site_left, int site_right) {
  if (threadIdx.x == 0) {
    sb.Lid[(size_t)site_left * dc * dc] = zmk(1.0, 0.0);
    sb.Rid[(size_t)site_right * dc * dc] = zmk(1.0, 0.0);
  }
}

hipError_t launch_identity_envs(const MpsView& st, SweepBuffers& sb, hipStream_t stream) {
  if (!sb.Lid || !sb.Rid || !sb.Yid) return hipErrorInvalidValue;   // buffers not set up
  const int dc = st.dcap, N = st.N;
  hipLaunchKernelGGL(k_set_unit_env, dim3(1), dim3(64), 0, stream, sb, dc, 0, N);
  const int t1 = (dc + ZT_M - 1) / ZT_M, t2 = (2 * dc + ZT_N - 1) / ZT_N;
  for (int n = 0; n < N; ++n) {
    hipLaunchKernelGGL(k_left_stage1, dim3(t2, t1, 1), dim3(256), 0, stream, st, sb, n, (const SweepJob*)nullptr, 1);
    hipLaunchKernelGGL(k_left_stage2, dim3(t1, t1, 1), dim3(256), 0, stream, st, sb, n, (const SweepJob*)nullptr, 1);
  }
  for (int n = N - 1; n >= 0; --n) {
    hipLaunchKernelGGL(k_right_stage1, dim3(t1, t2, 1), dim3(256), 0, stream, st, sb, n);
    hipLaunchKernelGGL(k_right_stage2, dim3(t1, t1, 1), dim3(256), 0, stream, st, sb, n);
  }
  return hipGetLastError();
}

hipError_t launch_transfer(const MpsView& st, SweepBuffers& sb, int n, const SweepJob* jobs, int njobs,
                           hipStream_t stream) {
  if (!sb.Lid || !sb.Lslots || !sb.Y) return hipErrorInvalidValue;
  const int dc = st.dcap;
  const int t1 = (dc + ZT_M - 1) / ZT_M, t2 = (2 * dc + ZT_N - 1) / ZT_N;
  for (int z0 = 0; z0 < njobs; z0 += 65535) {
    const int nz = njobs - z0 < 65535 ? njobs - z0 : 65535;
    hipLaunchKernelGGL(k_left_stage1, dim3(t2, t1, nz), dim3(256), 0, stream, st, sb, n, jobs + z0, 0);
    hipLaunchKernelGGL(k_left_stage2, dim3(t1, t1, nz), dim3(256), 0, stream, st, sb, n, jobs + z0, 0);
  }
  return hipGetLastError();
}

// e_t = sum_{b',b} L_slot[b'][b] R^id_{n+1}[b'][b]
__global__ __launch_bounds__(256) void k_finalize(MpsView st, SweepBuffers sb, int n, const int* slots,
                                                  const int* terms) {
  __shared__ double red[256];
  const int z = blockIdx.x;
  const int dc = st.dcap;
  const int b = st.dims[n + 1];
  const zd* L = sb.Lslots + (size_t)slots[z] * dc * dc;
  const zd* R = sb.Rid + (size_t)(n + 1) * dc * dc;
  double re = 0.0, im = 0.0;
  for (int e = threadIdx.x; e < b * b; e += 256) {
    const int r = e / b, c = e % b;
    const zd l = L[(size_t)r * dc + c], q = R[(size_t)r * dc + c];
    re = fma(l.x, q.x, fma(-l.y, q.y, re));
    im = fma(l.x, q.y, fma(l.y, q.x, im));
  }
  re = block_sum256(re, red);
  im = block_sum256(im, red);
  if (threadIdx.x == 0) sb.termval[terms[z]] = zmk(re, im);
}

hipError_t launch_finalize(const MpsView& st, SweepBuffers& sb, int n, const int* slots, const int* terms,
                           int nfin, hipStream_t stream) {
  if (nfin > 0) hipLaunchKernelGGL(k_finalize, dim3(nfin), dim3(256), 0, stream, st, sb, n, slots, terms);
  return hipGetLastError();
}

// Neumaier-compensated sum, one work-group, fixed order (deterministic).
__device__ inline void neumaier_add(double& s, double& c, double x) {
  const double t = s + x;
  if (fabs(s) >= fabs(x))
    c += (s - t) + x;
  else
    c += (x - t) + s;
  s = t;
}

__global__ __launch_bounds__(256) void k_energy_sum(MpsView st, SweepBuffers sb, const double* coeff, int64_t K,
                                                    double c0) {
  __shared__ double sre[256], cre[256], sim[256], cim[256];
  const int t = threadIdx.x;
  double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
  for (int64_t k = t; k < K; k += 256) {
    const zd v = sb.termval[k];
    neumaier_add(s1, c1, coeff[k] * v.x);
    neumaier_add(s2, c2, coeff[k] * v.y);
  }
  sre[t] = s1;
  cre[t] = c1;
  sim[t] = s2;
  cim[t] = c2;
  __syncthreads();
  if (t == 0) {
    double S1 = 0.0, C1 = 0.0, S2 = 0.0, C2 = 0.0;
    for (int q = 0; q < 256; ++q) {
      neumaier_add(S1, C1, sre[q]);
      neumaier_add(S1, C1, cre[q]);
      neumaier_add(S2, C2, sim[q]);
      neumaier_add(S2, C2, cim[q]);
    }
    const double Z = sb.Lid[(size_t)st.N * st.dcap * st.dcap].x;
    sb.energy[0] = c0 + (S1 + C1) / Z;
    sb.energy[1] = (S2 + C2) / Z;
    sb.energy[2] = Z;
  }
}

hipError_t launch_energy_sum(const MpsView& st, SweepBuffers& sb, const double* coeff, int64_t K, double c0,
                             hipStream_t stream) {
  hipLaunchKernelGGL(k_energy_sum, dim3(1), dim3(256), 0, stream, st, sb, coeff, K, c0);
  return hipGetLastError();
}
