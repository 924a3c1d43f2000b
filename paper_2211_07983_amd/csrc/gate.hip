// Two-qubit gate update on the MPS (arXiv:2211.07983, Sec. 3, the Hastings
// update for a nearest-neighbour gate):
//   C  = Q . (B_n B_{n+1})            (contraction, k_contract)
//   C~ = lambda_{n-1} C               (row weighting, fused into k_contract)
//   C~ = U s W  truncated to r values (one-sided Jacobi SVD, k_svd_jacobi)
//   B~_n = C W_r^dagger / nu, B~_{n+1} = W_r, lambda_n = s_r / nu   (k_update_*)
// All sizes are read from the device-side bond dimensions, so a whole circuit
// is enqueued without any host synchronisation.
#include <hip/hip_cooperative_groups.h>

#include "engine.h"

namespace cg = cooperative_groups;

// ----------------------------------------------------------------------------
// k_contract: C[(a,i'),(j',b)] = sum_{ij} Q[(i'j'),(ij)] sum_g B_n[a,i,g] B_{n+1}[g,j,b]
// and A = lambda_{n-1}[a] C.  GEMM rows r = 2a + i, columns c = 2b + j so that
// each thread holds the four (i, j) values of one (alpha, beta) pair.
// C and A are column-major with leading dimension ldc; column index j'*b + beta.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_contract(MpsView st, GateTable gt, int g, const double* theta,
                                                  zd* C, zd* A, int ldc, double* nrm_part) {
  __shared__ zd Q[16];
  __shared__ double red[256];
  const int n = gt.bond[g];
  const int a = st.dims[n], m = st.dims[n + 1], b = st.dims[n + 2];
  const int Mr = 2 * a, Nc = 2 * b;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  const int part = blockIdx.y * gridDim.x + blockIdx.x;
  if (i0 >= Mr || j0 >= Nc) {
    if (threadIdx.x == 0) nrm_part[part] = 0.0;
    return;
  }
  gate_matrix(gt, g, theta, Q);
  const zd* Bl = st.site(n);
  const zd* Br = st.site(n + 1);
  const int dc = st.dcap;
  auto fa = [&](int r, int k) { return Bl[(size_t)(r >> 1) * 2 * dc + (r & 1) * dc + k]; };
  auto fb = [&](int k, int c) { return Br[(size_t)k * 2 * dc + (c & 1) * dc + (c >> 1)]; };
  zd acc[2][2];
  ztile_acc(Mr, Nc, m, i0, j0, fa, fb, acc);
  __syncthreads();
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  double nrm = 0.0;
  if (r0 < Mr && c0 < Nc) {
    const int al = r0 >> 1, be = c0 >> 1;
    const double w = st.lam[(size_t)n * dc + al];
    for (int ip = 0; ip < 2; ++ip)
      for (int jp = 0; jp < 2; ++jp) {
        zd v = zmk(0.0, 0.0);
        for (int i = 0; i < 2; ++i)
          for (int j = 0; j < 2; ++j) v = zfma(Q[(ip * 2 + jp) * 4 + i * 2 + j], acc[i][j], v);
        const size_t idx = (size_t)(jp * b + be) * ldc + (2 * al + ip);
        const zd wv = zscale(v, w);
        C[idx] = v;
        A[idx] = wv;
        nrm += zabs2(wv);
      }
  }
  nrm = block_sum256(nrm, red);
  if (threadIdx.x == 0) nrm_part[part] = nrm;
}

// ----------------------------------------------------------------------------
// One-sided block Jacobi SVD of A (M x ncol, column-major), accumulating the
// right rotations in V (ncol x ncol).  P work-groups each hold a pair of
// column blocks of width W in LDS; the pairs follow a round-robin tournament,
// with a grid barrier between rounds.  Round 0 of a sweep orthogonalises all
// pairs inside both blocks, later rounds the cross pairs only, so a sweep
// visits every column pair exactly once.  A rotation is skipped when
// |a_i^H a_j| <= tol sqrt(|a_i|^2 |a_j|^2); the sweep loop stops after a sweep
// with no rotation.  At the end: s_j = |a_j|, the descending order, the kept
// rank r = min(D, #{s > eps}), nu = |s_r| and lambda_n.
// ----------------------------------------------------------------------------
__device__ inline void tourney(int P, int k, int p, int& q0, int& q1) {
  const int R = 2 * P - 1;
  if (p == 0) {
    q0 = R;
    q1 = k % R;
  } else {
    q0 = (k + p) % R;
    q1 = (k - p + R) % R;
  }
}

template <int W>
__global__ __launch_bounds__(256) void k_svd_jacobi(SvdArgs s) {
  cg::grid_group grid = cg::this_grid();
  extern __shared__ zd lds[];
  const int n = s.bond;
  const int a = s.dims[n], b = s.dims[n + 2];
  const int M = 2 * a, ncol = 2 * b;
  const int P = (ncol + 2 * W - 1) / (2 * W);
  const int p = blockIdx.x;
  const int t = threadIdx.x;
  const int mpad = s.lda;          // LDS column stride for A
  const int vpad = s.ldv;          // LDS column stride for V
  zd* Al = lds;                    // [2W][mpad]
  zd* Vl = lds + 2 * W * mpad;     // [2W][vpad]
  __shared__ int sh_rot;
  __shared__ int sh_stop;
  const int TPP = 256 / W;         // threads per pair
  const int pr = t / TPP, lt = t % TPP;
  const double tol = s.tol;
  // |gamma| below floor = 1e-28 |A|_F^2 means both columns are negligible (far
  // below any kept Schmidt value): such pairs are left alone, which keeps wide
  // matrices, whose surplus columns must shrink to zero, from sweeping forever.
  double fro = 0.0;
  for (int q = 0; q < s.nparts; ++q) fro += s.nrm_part[q];
  const double floor_g = 1e-28 * fro;
  int sweep = 0;
  for (; sweep < s.max_sweeps; ++sweep) {
    if (t == 0) sh_rot = 0;
    for (int k = 0; k < 2 * P - 1; ++k) {
      int q0, q1;
      tourney(P, k, p, q0, q1);
      if (p < P) {
        // load both blocks (columns >= ncol are zero padding, V = I there)
        for (int c = 0; c < 2 * W; ++c) {
          const int gc = (c < W ? q0 : q1) * W + (c % W);
          for (int r = t; r < M; r += 256)
            Al[c * mpad + r] = gc < ncol ? s.A[(size_t)gc * s.lda + r] : zmk(0.0, 0.0);
          for (int r = t; r < ncol; r += 256) {
            zd v;
            if (sweep == 0 && k == 0)
              v = zmk(r == gc ? 1.0 : 0.0, 0.0);
            else
              v = gc < ncol ? s.V[(size_t)gc * s.ldv + r] : zmk(0.0, 0.0);
            Vl[c * vpad + r] = v;
          }
        }
        __syncthreads();
        const int nsub = (k == 0) ? (2 * W - 1) : W;
        for (int sub = 0; sub < nsub; ++sub) {
          int c0, c1;
          if (k == 0) {
            const int R = 2 * W - 1;
            if (pr == 0) {
              c0 = R;
              c1 = sub % R;
            } else {
              c0 = (sub + pr) % R;
              c1 = (sub - pr + R) % R;
            }
          } else {
            c0 = pr;
            c1 = W + (pr + sub) % W;
          }
          zd* x = Al + c0 * mpad;
          zd* y = Al + c1 * mpad;
          double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
          for (int r = lt; r < M; r += TPP) {
            const zd u = x[r], v = y[r];
            al = fma(u.x, u.x, fma(u.y, u.y, al));
            be = fma(v.x, v.x, fma(v.y, v.y, be));
            gr = fma(u.x, v.x, fma(u.y, v.y, gr));
            gi = fma(u.x, v.y, fma(-u.y, v.x, gi));
          }
          for (int o = TPP / 2; o > 0; o >>= 1) {
            al += __shfl_xor(al, o, TPP);
            be += __shfl_xor(be, o, TPP);
            gr += __shfl_xor(gr, o, TPP);
            gi += __shfl_xor(gi, o, TPP);
          }
          const double ag = sqrt(fma(gr, gr, gi * gi));
          const double ab = al * be;
          if (ab > 1e-300 && ag > tol * sqrt(ab) && ag > floor_g) {
            const double zeta = (be - al) / (2.0 * ag);
            const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
            const double cs = 1.0 / sqrt(fma(tt, tt, 1.0));
            const double sn = cs * tt;
            // e^{-i phi} with gamma = |gamma| e^{i phi}
            const zd em = zmk(gr / ag, -gi / ag);
            const zd sem = zscale(em, sn), cem = zscale(em, cs);
            for (int r = lt; r < M; r += TPP) {
              const zd u = x[r], v = y[r];
              x[r] = zsub(zscale(u, cs), zmul(sem, v));
              y[r] = zadd(zscale(u, sn), zmul(cem, v));
            }
            zd* xv = Vl + c0 * vpad;
            zd* yv = Vl + c1 * vpad;
            for (int r = lt; r < ncol; r += TPP) {
              const zd u = xv[r], v = yv[r];
              xv[r] = zsub(zscale(u, cs), zmul(sem, v));
              yv[r] = zadd(zscale(u, sn), zmul(cem, v));
            }
            if (lt == 0) sh_rot = 1;
          }
          __syncthreads();
        }
        for (int c = 0; c < 2 * W; ++c) {
          const int gc = (c < W ? q0 : q1) * W + (c % W);
          if (gc >= ncol) continue;
          for (int r = t; r < M; r += 256) s.A[(size_t)gc * s.lda + r] = Al[c * mpad + r];
          for (int r = t; r < ncol; r += 256) s.V[(size_t)gc * s.ldv + r] = Vl[c * vpad + r];
        }
      }
      __threadfence();
      grid.sync();
      __threadfence();
    }
    // Sweep finished: count the work-groups that rotated.  The counter of this
    // sweep (zeroed by the host before the launch) is only incremented before
    // the barrier and only read after it, so every work-group reads the same
    // value and all of them leave the loop after the same number of barriers.
    if (t == 0 && sh_rot) __hip_atomic_fetch_add(&s.rotflag[sweep], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    grid.sync();
    __threadfence();
    if (t == 0) sh_stop = __hip_atomic_load(&s.rotflag[sweep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    __syncthreads();
    if (sh_stop) break;
  }
  const int used = sweep + 1;
  // singular values: column norms
  for (int c = p; c < ncol; c += gridDim.x) {
    double acc = 0.0;
    for (int r = t; r < M; r += 256) acc += zabs2(s.A[(size_t)c * s.lda + r]);
    __shared__ double red[256];
    acc = block_sum256(acc, red);
    if (t == 0) s.sv[c] = sqrt(acc);
  }
  __threadfence();
  grid.sync();
  __threadfence();
  if (p != 0) return;
  // work-group 0: order, rank, normalisation, lambda, statistics
  __shared__ double shs[1024];
  for (int c = t; c < ncol; c += 256) shs[c] = s.sv[c];
  __syncthreads();
  for (int c = t; c < ncol; c += 256) {
    const double v = shs[c];
    int rank = 0;
    for (int q = 0; q < ncol; ++q) {
      const double u = shs[q];
      rank += (u > v) || (u == v && q < c);
    }
    s.perm[rank] = c;
  }
  __syncthreads();
  if (t == 0) {
    int cnt = 0;
    double tot = 0.0;
    for (int q = 0; q < ncol; ++q) {
      const double v = shs[s.perm[q]];
      cnt += v > s.eps;
      tot += v * v;
    }
    int r = cnt < s.dmax ? cnt : s.dmax;
    if (r < 1) r = 1;
    double kept = 0.0;
    for (int q = 0; q < r; ++q) {
      const double v = shs[s.perm[q]];
      kept += v * v;
    }
    const double nu = sqrt(kept);
    s.gmeta[0] = r;
    s.gmeta[8] = M;
    s.gmeta[9] = ncol;
    s.gmeta[10] = used;
    s.gdmeta[0] = nu;
    const double disc = tot > 0.0 ? (tot - kept) / tot : 0.0;
    GateStats* gs = s.stats;
    gs->disc_sum += disc;
    if (disc > gs->disc_max) gs->disc_max = disc;
    if (disc > 0.0) gs->truncated += 1;
    if (used > gs->max_sweeps) gs->max_sweeps = used;
    if (!(sweep < s.max_sweeps)) gs->noconv += 1;
    if (r < ncol) {
      const double s0 = shs[s.perm[0]], sr1 = shs[s.perm[r - 1]], sr = shs[s.perm[r]];
      if (sr > 0.0 && (sr1 - sr) < 1e-10 * s0) gs->degenerate_cuts += 1;
    }
    if (r > gs->max_bond) gs->max_bond = r;
    gs->gates += 1;
    s.dims[n + 1] = r;
  }
  __syncthreads();
  const int r = s.gmeta[0];
  const double nu = s.gdmeta[0];
  for (int q = t; q < r; q += 256) s.lam_out[q] = shs[s.perm[q]] / nu;
}

// ----------------------------------------------------------------------------
// k_update_left: B~_n[(a,i'), mu] = sum_c C[(a,i'), c] V[c, perm[mu]] / nu.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_update_left(MpsView st, int n, const zd* C, int ldc, const zd* V,
                                                     int ldv, const int* perm, const int* gmeta,
                                                     const double* gdmeta) {
  const int a = st.dims[n], b = st.dims[n + 2];
  const int r = gmeta[0];
  const double inv = 1.0 / gdmeta[0];
  const int Mr = 2 * a, Nc = r, K = 2 * b;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  if (i0 >= Mr || j0 >= Nc) return;
  auto fa = [&](int row, int k) { return C[(size_t)k * ldc + row]; };
  auto fb = [&](int k, int mu) { return V[(size_t)perm[mu] * ldv + k]; };
  zd acc[2][2];
  ztile_acc(Mr, Nc, K, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  zd* Bn = st.site(n);
  const int dc = st.dcap;
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int row = r0 + x, mu = c0 + y;
      if (row < Mr && mu < Nc) Bn[(size_t)(row >> 1) * 2 * dc + (row & 1) * dc + mu] = zscale(acc[x][y], inv);
    }
}

// k_update_right: B~_{n+1}[mu, j', beta] = conj(V[j'*b + beta, perm[mu]]).
__global__ __launch_bounds__(256) void k_update_right(MpsView st, int n, const zd* V, int ldv, const int* perm,
                                                      const int* gmeta) {
  const int b = st.dims[n + 2];
  const int r = gmeta[0];
  const int mu = blockIdx.x;
  if (mu >= r) return;
  zd* Br = st.site(n + 1);
  const int dc = st.dcap;
  const int col = perm[mu];
  for (int e = threadIdx.x; e < 2 * b; e += 256) {
    const int jp = e / b, be = e % b;
    Br[(size_t)mu * 2 * dc + jp * dc + be] = zconj(V[(size_t)col * ldv + e]);
  }
}

// ----------------------------------------------------------------------------
// Host launchers
// ----------------------------------------------------------------------------
int svd_width(int dcap) { return dcap <= 128 ? 8 : 4; }

static SvdArgs svd_args(const MpsView& st, int bond, GateWork& w) {
  SvdArgs s;
  s.A = w.A;
  s.lda = w.ldc;
  s.V = w.V;
  s.ldv = w.ldv;
  s.dims = st.dims;
  s.bond = bond;
  s.sv = w.sv;
  s.perm = w.perm;
  s.gmeta = w.gmeta;
  s.gdmeta = w.gdmeta;
  s.rotflag = w.rotflag;
  s.lam_out = st.lam + (size_t)(bond + 1) * st.dcap;
  s.stats = w.stats;
  s.eps = w.eps;
  s.dmax = w.dmax;
  s.tol = w.tol;
  s.max_sweeps = w.max_sweeps;
  s.nrm_part = w.nrm_part;
  const int tiles = (2 * st.dcap + ZT_M - 1) / ZT_M;
  s.nparts = tiles * tiles;
  return s;
}

hipError_t launch_contract(const MpsView& st, const GateTable& gt, int g, const double* theta, GateWork& w,
                           hipStream_t stream) {
  const int tiles = (2 * st.dcap + ZT_M - 1) / ZT_M;
  hipLaunchKernelGGL(k_contract, dim3(tiles, tiles), dim3(256), 0, stream, st, gt, g, theta, w.C, w.A, w.ldc,
                     w.nrm_part);
  return hipGetLastError();
}

hipError_t launch_svd(const MpsView& st, int bond, GateWork& w, hipStream_t stream) {
  SvdArgs s = svd_args(st, bond, w);
  const int W = svd_width(st.dcap);
  const int P = (w.ncap + 2 * W - 1) / (2 * W);
  const size_t shm = (size_t)2 * W * (w.ldc + w.ldv) * sizeof(zd);
  void* args[] = {&s};
  hipError_t e = hipMemsetAsync(w.rotflag, 0, 128 * sizeof(int), stream);
  if (e != hipSuccess) return e;
  if (W == 8)
    e = hipLaunchCooperativeKernel((const void*)k_svd_jacobi<8>, dim3(P), dim3(256), args, shm, stream);
  else
    e = hipLaunchCooperativeKernel((const void*)k_svd_jacobi<4>, dim3(P), dim3(256), args, shm, stream);
  return e;
}

hipError_t launch_update(const MpsView& st, int bond, GateWork& w, hipStream_t stream) {
  const int dc = st.dcap;
  const int tm = (2 * dc + ZT_M - 1) / ZT_M, tn = (dc + ZT_N - 1) / ZT_N;
  hipLaunchKernelGGL(k_update_left, dim3(tn, tm), dim3(256), 0, stream, st, bond, (const zd*)w.C, w.ldc,
                     (const zd*)w.V, w.ldv, (const int*)w.perm, (const int*)w.gmeta, (const double*)w.gdmeta);
  hipLaunchKernelGGL(k_update_right, dim3(dc), dim3(256), 0, stream, st, bond, (const zd*)w.V, w.ldv,
                     (const int*)w.perm, (const int*)w.gmeta);
  return hipGetLastError();
}

hipError_t launch_gate(const MpsView& st, const GateTable& gt, int g, int bond, const double* theta,
                       GateWork& w, hipStream_t stream) {
  hipError_t e = launch_contract(st, gt, g, theta, w, stream);
  if (e != hipSuccess) return e;
  e = launch_svd(st, bond, w, stream);
  if (e != hipSuccess) return e;
  return launch_update(st, bond, w, stream);
}

hipError_t svd_set_attributes(int dcap, size_t shm) {
  hipError_t e = hipFuncSetAttribute((const void*)k_svd_jacobi<8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)shm);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_svd_jacobi<4>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}
