// Pauli-string expectation values with FP32 matrix-core transfers
// (arXiv:2211.07983, Sec. 3, Eq. paulistringexp; precision mode 1).
//
// The same sweep as the FP64 path -- identity environments L^id / R^id, one
// left transfer L' = sum_i o_i (B^{i^x})^dagger L B^i per (term, site) job,
// a term's value <L, R^id_{b+1}> after its last site -- with the sites and
// environments held as complex FP32 and every transfer GEMM on
// v_mfma_f32_16x16x4f32.  A complex product takes three real products
// (Ar Br, Ai Bi, (Ar+Ai)(Br+Bi)) with FP32 accumulation.  The term inner
// products, the normalisation Z and the energy sum stay FP64.
#include "engine.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ inline cf cmk(float r, float i) { return make_float2(r, i); }
__device__ inline cf cconj(cf a) { return make_float2(a.x, -a.y); }
__device__ inline cf cmul(cf a, cf b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// ---------------------------------------------------------------------------
// A 64x64 output tile of C = A * B (complex FP32) on the matrix cores, 256
// threads.  Wave w owns the 32x32 quarter (rows 32 (w/2), columns 32 (w%2)),
// four 16x16 MFMA blocks, each with three accumulators (the three real
// products).  K advances in stages of 16: every thread fetches 4 elements of
// each operand (the next stage is fetched while the current one is
// multiplied) and stores them to LDS as three planes (re, im, re + im),
// k-major so that the operand reads of a 16x16x4 step are unit-stride.
// AKC / BKC: the operand is contiguous along k in memory (the fetch mapping
// puts consecutive threads along k), otherwise along m / n.  fa(m, k) and
// fb(k, n) are called in range only; out-of-range elements are zero.
// fo(m, n, value) is called for every in-range output element.
// ---------------------------------------------------------------------------
#define CT_M 64
#define CT_N 64
#define CT_K 16
#define CT_P 68

template <bool KC>
__device__ inline void ct_coord(int e, int& mn, int& k) {
  if (KC) {
    k = e & (CT_K - 1);
    mn = e >> 4;
  } else {
    mn = e & (CT_M - 1);
    k = e >> 6;
  }
}

template <bool AKC, bool BKC, class FA, class FB, class FO>
__device__ inline void ctile_mfma(int M, int N, int K, int i0, int j0, FA fa, FB fb, FO fo) {
  __shared__ float sA[3][CT_K][CT_P];
  __shared__ float sB[3][CT_K][CT_P];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  floatx4 acc[3][2][2];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[p][x][y] = floatx4{0.f, 0.f, 0.f, 0.f};
  cf ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q;
      int m, k, n, kb;
      ct_coord<AKC>(e, m, k);
      ct_coord<BKC>(e, n, kb);
      ra[q] = (i0 + m < M && k0 + k < K) ? fa(i0 + m, k0 + k) : cmk(0.f, 0.f);
      rb[q] = (j0 + n < N && k0 + kb < K) ? fb(k0 + kb, j0 + n) : cmk(0.f, 0.f);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += CT_K) {
    __syncthreads();   // the previous stage has been read by every wave
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q;
      int m, k, n, kb;
      ct_coord<AKC>(e, m, k);
      ct_coord<BKC>(e, n, kb);
      sA[0][k][m] = ra[q].x;
      sA[1][k][m] = ra[q].y;
      sA[2][k][m] = ra[q].x + ra[q].y;
      sB[0][kb][n] = rb[q].x;
      sB[1][kb][n] = rb[q].y;
      sB[2][kb][n] = rb[q].x + rb[q].y;
    }
    __syncthreads();
    if (k0 + CT_K < K) fetch(k0 + CT_K);
#pragma unroll
    for (int k4 = 0; k4 < CT_K / 4; ++k4) {
      const int kk = k4 * 4 + lk;
      float av[3][2], bv[3][2];
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          av[p][x] = sA[p][kk][wm + x * 16 + lr];
          bv[p][x] = sB[p][kk][wn + x * 16 + lr];
        }
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
            acc[p][x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[p][x], bv[p][y], acc[p][x][y], 0, 0, 0);
    }
  }
  // 16x16 block result: element (4 (lane / 16) + q, lane % 16) in register q
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = i0 + wm + x * 16 + 4 * lk + q, c = j0 + wn + y * 16 + lr;
        if (r < M && c < N) {
          const float t1 = acc[0][x][y][q], t2 = acc[1][x][y][q], t3 = acc[2][x][y][q];
          fo(r, c, cmk(t1 - t2, t3 - t1 - t2));
        }
      }
}

// ---------------------------------------------------------------------------
// Kernels.  B32 is [N][dcap][2][dcap] (the FP64 site layout), environments
// [dcap][dcap] row-major, Y [dcap][2][dcap].
// ---------------------------------------------------------------------------
__global__ void k_sites_f32(MpsView st, cf* B32) {
  const size_t total = (size_t)st.N * st.site_elems();
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const zd v = st.B[e];
    B32[e] = cmk((float)v.x, (float)v.y);
  }
}

__device__ inline cf* env32(const Sweep32& s, int dc, int slot, int site) {
  return slot < 0 ? s.Lid + (size_t)site * dc * dc : s.Lslots + (size_t)slot * dc * dc;
}

// Y_z = L_in [B^0 | B^1] (a x 2b); column c = i b + beta
__global__ __launch_bounds__(256) void k_left1_f32(MpsView st, Sweep32 s, int n, const SweepJob* jobs,
                                                   int identity) {
  const int a = st.dims[n], b = st.dims[n + 1];
  const int dc = st.dcap;
  const int i0 = blockIdx.y * CT_M, j0 = blockIdx.x * CT_N;
  if (i0 >= a || j0 >= 2 * b) return;
  const int z = blockIdx.z;
  const cf* L = env32(s, dc, identity ? -1 : jobs[z].in_slot, n);
  cf* Y = identity ? s.Yid : s.Y + (size_t)z * dc * 2 * dc;
  const cf* B = s.B + (size_t)n * dc * 2 * dc;
  ctile_mfma<true, false>(
      a, 2 * b, a, i0, j0, [&](int r, int k) { return L[(size_t)r * dc + k]; },
      [&](int k, int c) {
        const int i = c >= b, be = c - i * b;
        return B[(size_t)k * 2 * dc + i * dc + be];
      },
      [&](int r, int c, cf v) {
        const int i = c >= b, be = c - i * b;
        Y[(size_t)r * 2 * dc + i * dc + be] = v;
      });
}

// L_out[b', b] = sum_{i, a'} o_i conj(B^{i^x}[a', b']) Y[a', i, b]
__global__ __launch_bounds__(256) void k_left2_f32(MpsView st, Sweep32 s, int n, const SweepJob* jobs,
                                                   int identity) {
  const int a = st.dims[n], b = st.dims[n + 1];
  const int dc = st.dcap;
  const int i0 = blockIdx.y * CT_M, j0 = blockIdx.x * CT_N;
  if (i0 >= b || j0 >= b) return;
  const int z = blockIdx.z;
  int xb = 0, out_slot = -1;
  cf o0 = cmk(1.f, 0.f), o1 = cmk(1.f, 0.f);
  if (!identity) {
    const SweepJob& jb = jobs[z];
    xb = jb.xb;
    out_slot = jb.out_slot;
    o0 = cmk((float)jb.o0.x, (float)jb.o0.y);
    o1 = cmk((float)jb.o1.x, (float)jb.o1.y);
  }
  const cf* Y = identity ? s.Yid : s.Y + (size_t)z * dc * 2 * dc;
  const cf* B = s.B + (size_t)n * dc * 2 * dc;
  cf* Lo = env32(s, dc, out_slot, n + 1);
  ctile_mfma<false, false>(
      b, b, 2 * a, i0, j0,
      [&](int r, int k) {
        const int i = k >= a, al = k - i * a;
        return cmul(i ? o1 : o0, cconj(B[(size_t)al * 2 * dc + (i ^ xb) * dc + r]));
      },
      [&](int k, int c) {
        const int i = k >= a, al = k - i * a;
        return Y[(size_t)al * 2 * dc + i * dc + c];
      },
      [&](int r, int c, cf v) { Lo[(size_t)r * dc + c] = v; });
}

// Yr[(i, a'), b] = sum_b' conj(B^i[a', b']) R[b', b]
__global__ __launch_bounds__(256) void k_right1_f32(MpsView st, Sweep32 s, int n) {
  const int a = st.dims[n], b = st.dims[n + 1];
  const int dc = st.dcap;
  const int i0 = blockIdx.y * CT_M, j0 = blockIdx.x * CT_N;
  if (i0 >= 2 * a || j0 >= b) return;
  const cf* R = s.Rid + (size_t)(n + 1) * dc * dc;
  const cf* B = s.B + (size_t)n * dc * 2 * dc;
  ctile_mfma<true, false>(
      2 * a, b, b, i0, j0,
      [&](int r, int k) {
        const int i = r >= a, al = r - i * a;
        return cconj(B[(size_t)al * 2 * dc + i * dc + k]);
      },
      [&](int k, int c) { return R[(size_t)k * dc + c]; },
      [&](int r, int c, cf v) { s.Yid[(size_t)r * dc + c] = v; });
}

// R_n[a', a] = sum_{i, b} Yr[(i, a'), b] B^i[a, b]
__global__ __launch_bounds__(256) void k_right2_f32(MpsView st, Sweep32 s, int n) {
  const int a = st.dims[n], b = st.dims[n + 1];
  const int dc = st.dcap;
  const int i0 = blockIdx.y * CT_M, j0 = blockIdx.x * CT_N;
  if (i0 >= a || j0 >= a) return;
  const cf* B = s.B + (size_t)n * dc * 2 * dc;
  cf* Ro = s.Rid + (size_t)n * dc * dc;
  ctile_mfma<true, true>(
      a, a, 2 * b, i0, j0,
      [&](int r, int k) {
        const int i = k >= b, be = k - i * b;
        return s.Yid[(size_t)(i * a + r) * dc + be];
      },
      [&](int k, int c) {
        const int i = k >= b, be = k - i * b;
        return B[(size_t)c * 2 * dc + i * dc + be];
      },
      [&](int r, int c, cf v) { Ro[(size_t)r * dc + c] = v; });
}

__global__ void k_unit_env_f32(Sweep32 s, int dc, int site_left, int site_right) {
  if (threadIdx.x == 0) {
    s.Lid[(size_t)site_left * dc * dc] = cmk(1.f, 0.f);
    s.Rid[(size_t)site_right * dc * dc] = cmk(1.f, 0.f);
  }
}

// e_t = sum_{b', b} L_slot[b'][b] R^id_{n+1}[b'][b], accumulated in FP64
__global__ __launch_bounds__(256) void k_finalize_f32(MpsView st, Sweep32 s, zd* termval, int n, const int* slots,
                                                      const int* terms) {
  __shared__ double red[256];
  const int z = blockIdx.x;
  const int dc = st.dcap;
  const int b = st.dims[n + 1];
  const cf* L = s.Lslots + (size_t)slots[z] * dc * dc;
  const cf* R = s.Rid + (size_t)(n + 1) * dc * dc;
  double re = 0.0, im = 0.0;
  for (int e = threadIdx.x; e < b * b; e += 256) {
    const int r = e / b, c = e % b;
    const cf l = L[(size_t)r * dc + c], q = R[(size_t)r * dc + c];
    re = fma((double)l.x, (double)q.x, fma(-(double)l.y, (double)q.y, re));
    im = fma((double)l.x, (double)q.y, fma((double)l.y, (double)q.x, im));
  }
  re = block_sum256(re, red);
  im = block_sum256(im, red);
  if (threadIdx.x == 0) termval[terms[z]] = zmk(re, im);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_sites_f32(const MpsView& st, cf* B32, hipStream_t stream) {
  const size_t total = (size_t)st.N * st.site_elems();
  const int blocks = (int)std::min<size_t>(4096, (total + 255) / 256);
  hipLaunchKernelGGL(k_sites_f32, dim3(blocks), dim3(256), 0, stream, st, B32);
  return hipGetLastError();
}

hipError_t launch_identity_envs_f32(const MpsView& st, Sweep32& s, hipStream_t stream) {
  if (!s.B || !s.Lid || !s.Rid || !s.Yid) return hipErrorInvalidValue;   // buffers not set up
  const int dc = st.dcap, N = st.N;
  hipLaunchKernelGGL(k_unit_env_f32, dim3(1), dim3(64), 0, stream, s, dc, 0, N);
  const int t1 = (dc + CT_M - 1) / CT_M, t2 = (2 * dc + CT_N - 1) / CT_N;
  for (int n = 0; n < N; ++n) {
    hipLaunchKernelGGL(k_left1_f32, dim3(t2, t1, 1), dim3(256), 0, stream, st, s, n, (const SweepJob*)nullptr, 1);
    hipLaunchKernelGGL(k_left2_f32, dim3(t1, t1, 1), dim3(256), 0, stream, st, s, n, (const SweepJob*)nullptr, 1);
  }
  for (int n = N - 1; n >= 0; --n) {
    hipLaunchKernelGGL(k_right1_f32, dim3(t1, t2, 1), dim3(256), 0, stream, st, s, n);
    hipLaunchKernelGGL(k_right2_f32, dim3(t1, t1, 1), dim3(256), 0, stream, st, s, n);
  }
  return hipGetLastError();
}

hipError_t launch_transfer_f32(const MpsView& st, Sweep32& s, int n, const SweepJob* jobs, int njobs,
                               hipStream_t stream) {
  if (!s.B || !s.Lid || !s.Lslots || !s.Y) return hipErrorInvalidValue;
  const int dc = st.dcap;
  const int t1 = (dc + CT_M - 1) / CT_M, t2 = (2 * dc + CT_N - 1) / CT_N;
  for (int z0 = 0; z0 < njobs; z0 += 65535) {
    const int nz = njobs - z0 < 65535 ? njobs - z0 : 65535;
    hipLaunchKernelGGL(k_left1_f32, dim3(t2, t1, nz), dim3(256), 0, stream, st, s, n, jobs + z0, 0);
    hipLaunchKernelGGL(k_left2_f32, dim3(t1, t1, nz), dim3(256), 0, stream, st, s, n, jobs + z0, 0);
  }
  return hipGetLastError();
}

hipError_t launch_finalize_f32(const MpsView& st, Sweep32& s, zd* termval, int n, const int* slots,
                               const int* terms, int nfin, hipStream_t stream) {
  if (nfin > 0)
    hipLaunchKernelGGL(k_finalize_f32, dim3(nfin), dim3(256), 0, stream, st, s, termval, n, slots, terms);
  return hipGetLastError();
}

// Z = <psi|psi> of the FP32 identity environment, as the FP64 energy sum reads it
__global__ void k_norm_from_f32(Sweep32 s, zd* dst) {
  if (threadIdx.x == 0) *dst = zmk((double)s.Lid[0].x, 0.0);
}

hipError_t launch_norm_from_f32(const MpsView& st, Sweep32& s, zd* dst, hipStream_t stream) {
  Sweep32 at = s;
  at.Lid = s.Lid + (size_t)st.N * st.dcap * st.dcap;
  hipLaunchKernelGGL(k_norm_from_f32, dim3(1), dim3(64), 0, stream, at, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sweep adjoint, precision 1: the per-term environment transfers of the
// cotangent sweep on the matrix cores (the same GEMM shapes as the energy
// sweep); contributions and injections accumulate into FP64 cotangents.
// ---------------------------------------------------------------------------
__device__ inline cf cf_of(zd z) { return cmk((float)z.x, (float)z.y); }

// Y = in [B^0 | B^1] (a x 2b), column c = i b + beta
__global__ __launch_bounds__(256) void k_env32_left1(const EnvJob32* jobs, const cf* B, int a, int b, int dc) {
  const EnvJob32& jb = jobs[blockIdx.z];
  const int i0 = blockIdx.y * CT_M, j0 = blockIdx.x * CT_N;
  if (i0 >= a || j0 >= 2 * b) return;
  const cf* in = jb.in;
  cf* y = jb.y;
  ctile_mfma<true, false>(
      a, 2 * b, a, i0, j0, [&](int r, int k) { return in[(size_t)r * dc + k]; },
      [&](int k, int c) {
        const int i = c >= b, be = c - i * b;
        return B[(size_t)k * 2 * dc + i * dc + be];
      },
      [&](int r, int c, cf v) {
        const int i = c >= b, be = c - i * b;
        y[(size_t)r * 2 * dc + i * dc + be] = v;
      });
}

// out[b', b] (+)= sum_{i, a'} o_i conj(B^{i^x}[a', b']) Y[a', i, b]
__global__ __launch_bounds__(256) void k_env32_left2(const EnvJob32* jobs, const cf* B, int a, int b, int dc) {
  const EnvJob32& jb = jobs[blockIdx.z];
  const int i0 = blockIdx.y * CT_M, j0 = blockIdx.x * CT_N;
  if (i0 >= b || j0 >= b) return;
  const cf o0 = cf_of(jb.o0), o1 = cf_of(jb.o1);
  const int xb = jb.xb, acc = jb.acc;
  const cf* y = jb.y;
  cf* out = jb.out;
  ctile_mfma<false, false>(
      b, b, 2 * a, i0, j0,
      [&](int r, int k) {
        const int i = k >= a, al = k - i * a;
        return cmul(i ? o1 : o0, cconj(B[(size_t)al * 2 * dc + (i ^ xb) * dc + r]));
      },
      [&](int k, int c) {
        const int i = k >= a, al = k - i * a;
        return y[(size_t)al * 2 * dc + i * dc + c];
      },
      [&](int r, int c, cf v) {
        cf* o = out + (size_t)r * dc + c;
        *o = acc ? cmk(o->x + v.x, o->y + v.y) : v;
      });
}

// Yr[(i, a'), b] = sum_b' conj(B^{i^x}[a', b']) in[b', b]   (2a x b, ld dc)
__global__ __launch_bounds__(256) void k_env32_right1(const EnvJob32* jobs, const cf* B, int a, int b, int dc) {
  const EnvJob32& jb = jobs[blockIdx.z];
  const int i0 = blockIdx.y * CT_M, j0 = blockIdx.x * CT_N;
  if (i0 >= 2 * a || j0 >= b) return;
  const int xb = jb.xb;
  const cf* in = jb.in;
  cf* y = jb.y;
  ctile_mfma<true, false>(
      2 * a, b, b, i0, j0,
      [&](int r, int k) {
        const int i = r >= a, al = r - i * a;
        return cconj(B[(size_t)al * 2 * dc + (i ^ xb) * dc + k]);
      },
      [&](int k, int c) { return in[(size_t)k * dc + c]; },
      [&](int r, int c, cf v) { y[(size_t)r * dc + c] = v; });
}

// out[a', a] (+)= sum_{i, b} o_i Yr[(i, a'), b] B^i[a, b]
__global__ __launch_bounds__(256) void k_env32_right2(const EnvJob32* jobs, const cf* B, int a, int b, int dc) {
  const EnvJob32& jb = jobs[blockIdx.z];
  const int i0 = blockIdx.y * CT_M, j0 = blockIdx.x * CT_N;
  if (i0 >= a || j0 >= a) return;
  const cf o0 = cf_of(jb.o0), o1 = cf_of(jb.o1);
  const int acc = jb.acc;
  const cf* y = jb.y;
  cf* out = jb.out;
  ctile_mfma<true, true>(
      a, a, 2 * b, i0, j0,
      [&](int r, int k) {
        const int i = k >= b, be = k - i * b;
        return cmul(i ? o1 : o0, y[(size_t)(i * a + r) * dc + be]);
      },
      [&](int k, int c) {
        const int i = k >= b, be = k - i * b;
        return B[(size_t)c * 2 * dc + i * dc + be];
      },
      [&](int r, int c, cf v) {
        cf* o = out + (size_t)r * dc + c;
        *o = acc ? cmk(o->x + v.x, o->y + v.y) : v;
      });
}

// g[a][i][b] = c conj(o_i) sum_b' Y[a][i^x][b'] rr[b][b']; blockIdx.y = i * tiles_a + row tile
__global__ __launch_bounds__(256) void k_env32_contrib(const EnvJob32* jobs, int a, int b, int dc) {
  const EnvJob32& jb = jobs[blockIdx.z];
  const int tiles_a = (a + CT_M - 1) / CT_M;
  const int i = blockIdx.y / tiles_a;
  const int i0 = (blockIdx.y % tiles_a) * CT_M, j0 = blockIdx.x * CT_N;
  if (i0 >= a || j0 >= b) return;
  const int src = i ^ jb.xb;
  const zd o = i ? jb.o1 : jb.o0;
  const cf w = cmk((float)(jb.c * o.x), (float)(-jb.c * o.y));
  const cf* y = jb.y;
  const cf* rr = jb.rr;
  cf* g = jb.g;
  ctile_mfma<true, true>(
      a, b, b, i0, j0, [&](int r, int k) { return y[(size_t)r * 2 * dc + src * dc + k]; },
      [&](int k, int c) { return rr[(size_t)c * dc + k]; },
      [&](int r, int c, cf v) { g[(size_t)r * 2 * dc + i * dc + c] = cmul(w, v); });
}

// Bbar_n[a][i][b] += sum_z g_z[a][i][b] in FP64 (fixed order)
__global__ void k_env32_reduce(const EnvJob32* jobs, int nj, zd* Bbar, int a, int b, int dc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a * 2 * b) return;
  const int al = e / (2 * b), rem = e % (2 * b), i = rem / b, be = rem % b;
  const size_t off = (size_t)al * 2 * dc + i * dc + be;
  zd s = Bbar[off];
  for (int z = 0; z < nj; ++z) {
    const cf v = jobs[z].g[off];
    s = zmk(s.x + (double)v.x, s.y + (double)v.y);
  }
  Bbar[off] = s;
}

// dst[r][c] += sum_z coeff_z src_z[r][c] for r, c < d, in FP64 (fixed order)
__global__ void k_inject32(const InjectItem32* items, int ni, zd* dst, int d, int dc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d * d) return;
  const size_t off = (size_t)(e / d) * dc + (e % d);
  zd s = dst[off];
  for (int z = 0; z < ni; ++z) {
    const cf v = items[z].src[off];
    s = zmk(fma(items[z].c, (double)v.x, s.x), fma(items[z].c, (double)v.y, s.y));
  }
  dst[off] = s;
}

static inline dim3 grid64(int M, int N, int z) { return dim3((N + CT_N - 1) / CT_N, (M + CT_M - 1) / CT_M, z); }

hipError_t launch_env32_right(const EnvJob32* jobs, int nj, const cf* B, int a, int b, int dc, hipStream_t s) {
  hipLaunchKernelGGL(k_env32_right1, grid64(2 * a, b, nj), dim3(256), 0, s, jobs, B, a, b, dc);
  hipLaunchKernelGGL(k_env32_right2, grid64(a, a, nj), dim3(256), 0, s, jobs, B, a, b, dc);
  return hipGetLastError();
}

hipError_t launch_env32_left(const EnvJob32* jobs, int nj, const cf* B, zd* Bbar, int a, int b, int dc,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_env32_left1, grid64(a, 2 * b, nj), dim3(256), 0, s, jobs, B, a, b, dc);
  const int ta = (a + CT_M - 1) / CT_M;
  hipLaunchKernelGGL(k_env32_contrib, dim3((b + CT_N - 1) / CT_N, 2 * ta, nj), dim3(256), 0, s, jobs, a, b, dc);
  hipLaunchKernelGGL(k_env32_reduce, dim3((a * 2 * b + 255) / 256), dim3(256), 0, s, jobs, nj, Bbar, a, b, dc);
  hipLaunchKernelGGL(k_env32_left2, grid64(b, b, nj), dim3(256), 0, s, jobs, B, a, b, dc);
  return hipGetLastError();
}

hipError_t launch_inject32(const InjectItem32* items, int ni, zd* dst, int d, int dc, hipStream_t s) {
  hipLaunchKernelGGL(k_inject32, dim3((d * d + 255) / 256), dim3(256), 0, s, items, ni, dst, d, dc);
  return hipGetLastError();
}
