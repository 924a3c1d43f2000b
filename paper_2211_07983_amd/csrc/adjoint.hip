// Reverse pass of the MPS energy (arXiv:2211.07983, Sec. 4 and App. A).
//
// The loss E(theta) = <psi|H|psi>/<psi|psi> is differentiated through every
// elementary step of the forward pass -- the "local" gradient that Sec. 4
// discusses -- using the complex back-propagation rules of App. A (Eqs.
// bp1-bp4).  A cotangent X_bar of a complex array X is defined by
// dE = Re <X_bar, dX> = Re sum conj(X_bar) dX (the paper's 2 dE/dX* rule).
//
// S7 (sweep adjoint): X_bar_n = (2/Z) [sum_k c_k G^(k)_n - (E - c0) G^id_n] with
//   G^i = conj(o_i) L B^{i^x} R^T, per term inside its support and through
//   aggregated environments outside it.
// S8 (gate adjoint): for each gate in reverse order, recomputed from the last
//   checkpoint with a tape, the adjoints of the site update, of the truncated
//   SVD (full spectrum: F_ij = 1/(s_j^2 - s_i^2), the imaginary diagonal gauge
//   term and the null space) and of the contraction; dE/dphi = Re <C_bar, D C>
//   with D = dQ/dphi Q^dagger = -(i/2) post ZZ post^dagger.
// S9: dE/dtheta_p = sum over gates with param p of coeff * dE/dphi.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "engine.h"
#include "plan_impl.h"

void plan_restore(mps_plan* p, int seg, mps_state* dst);

// ============================================================================
// Environment transfers with per-job pointers (sweep adjoint)
// ============================================================================
struct EnvJob {
  const zd* in;   // input environment
  zd* out;        // output environment
  zd* y;          // stage-1 buffer ([dc][2 dc])
  const zd* rr;   // right environment of the contribution
  zd* g;          // contribution buffer ([dc][2 dc])
  double c;       // term coefficient
  int xb;         // bit flip of the site operator
  int acc;        // stage 2 accumulates into out
  zd o0, o1;      // O[i^x, i] = o_i
};

// Y = in [B^0 | B^1] (a x 2b), column c = i*b + beta
__global__ __launch_bounds__(256) void k_env_left1(const EnvJob* jobs, const zd* B, int a, int b, int dc) {
  const EnvJob jb = jobs[blockIdx.z];
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  if (i0 >= a || j0 >= 2 * b) return;
  auto fa = [&](int r, int k) { return jb.in[(size_t)r * dc + k]; };
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
        jb.y[(size_t)r * 2 * dc + i * dc + be] = acc[x][y];
      }
    }
}

// out[b', b] (+)= sum_{i, a'} o_i conj(B^{i^x}[a', b']) Y[a', i, b]
__global__ __launch_bounds__(256) void k_env_left2(const EnvJob* jobs, const zd* B, int a, int b, int dc) {
  const EnvJob jb = jobs[blockIdx.z];
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  if (i0 >= b || j0 >= b) return;
  auto fa = [&](int r, int k) {
    const int i = k >= a, al = k - i * a;
    return zmul(i ? jb.o1 : jb.o0, zconj(B[(size_t)al * 2 * dc + (i ^ jb.xb) * dc + r]));
  };
  auto fb = [&](int k, int c) {
    const int i = k >= a, al = k - i * a;
    return jb.y[(size_t)al * 2 * dc + i * dc + c];
  };
  zd acc[2][2];
  ztile_acc(b, b, 2 * a, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int r = r0 + x, c = c0 + y;
      if (r < b && c < b) {
        zd* o = jb.out + (size_t)r * dc + c;
        *o = jb.acc ? zadd(*o, acc[x][y]) : acc[x][y];
      }
    }
}

// Yr[(i, a'), b] = sum_b' conj(B^{i^x}[a', b']) in[b', b]   (2a x b, ld dc)
__global__ __launch_bounds__(256) void k_env_right1(const EnvJob* jobs, const zd* B, int a, int b, int dc) {
  const EnvJob jb = jobs[blockIdx.z];
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  if (i0 >= 2 * a || j0 >= b) return;
  auto fa = [&](int r, int k) {
    const int i = r >= a, al = r - i * a;
    return zconj(B[(size_t)al * 2 * dc + (i ^ jb.xb) * dc + k]);
  };
  auto fb = [&](int k, int c) { return jb.in[(size_t)k * dc + c]; };
  zd acc[2][2];
  ztile_acc(2 * a, b, b, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int r = r0 + x, c = c0 + y;
      if (r < 2 * a && c < b) jb.y[(size_t)r * dc + c] = acc[x][y];
    }
}

// out[a', a] (+)= sum_{i, b} o_i Yr[(i, a'), b] B^i[a, b]
__global__ __launch_bounds__(256) void k_env_right2(const EnvJob* jobs, const zd* B, int a, int b, int dc) {
  const EnvJob jb = jobs[blockIdx.z];
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  if (i0 >= a || j0 >= a) return;
  auto fa = [&](int r, int k) {
    const int i = k >= b, be = k - i * b;
    return zmul(i ? jb.o1 : jb.o0, jb.y[(size_t)(i * a + r) * dc + be]);
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
      if (r < a && c < a) {
        zd* o = jb.out + (size_t)r * dc + c;
        *o = jb.acc ? zadd(*o, acc[x][y]) : acc[x][y];
      }
    }
}

// g[a][i][b] = c conj(o_i) sum_b' Y[a][i^x][b'] rr[b][b']
__global__ __launch_bounds__(256) void k_env_contrib(const EnvJob* jobs, int a, int b, int dc) {
  const EnvJob jb = jobs[blockIdx.z];
  const int tiles_a = (a + ZT_M - 1) / ZT_M;
  const int i = blockIdx.y / tiles_a;
  const int i0 = (blockIdx.y % tiles_a) * ZT_M, j0 = blockIdx.x * ZT_N;
  if (i0 >= a || j0 >= b) return;
  const int src = i ^ jb.xb;
  auto fa = [&](int r, int k) { return jb.y[(size_t)r * 2 * dc + src * dc + k]; };
  auto fb = [&](int k, int c) { return jb.rr[(size_t)c * dc + k]; };
  zd acc[2][2];
  ztile_acc(a, b, b, i0, j0, fa, fb, acc);
  const zd w = zscale(zconj(i ? jb.o1 : jb.o0), jb.c);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int r = r0 + x, c = c0 + y;
      if (r < a && c < b) jb.g[(size_t)r * 2 * dc + i * dc + c] = zmul(w, acc[x][y]);
    }
}

// Bbar_n[a][i][b] += sum_z g_z[a][i][b]  (fixed order)
__global__ void k_env_reduce(const EnvJob* jobs, int nj, zd* Bbar, int a, int b, int dc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a * 2 * b) return;
  const int al = e / (2 * b), rem = e % (2 * b), i = rem / b, be = rem % b;
  const size_t off = (size_t)al * 2 * dc + i * dc + be;
  zd s = Bbar[off];
  for (int z = 0; z < nj; ++z) s = zadd(s, jobs[z].g[off]);
  Bbar[off] = s;
}

// dst[r][c] += sum_z coeff_z src_z[r][c] for r, c < d  (fixed order)
struct InjectItem {
  const zd* src;
  double c;
  double pad;
};
__global__ void k_inject(const InjectItem* items, int ni, zd* dst, int d, int dc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d * d) return;
  const size_t off = (size_t)(e / d) * dc + (e % d);
  zd s = dst[off];
  for (int z = 0; z < ni; ++z) s = zadd(s, zscale(items[z].src[off], items[z].c));
  dst[off] = s;
}

__global__ void k_scale_sites(zd* Bbar, const int* dims, int N, int dc, double w) {
  const int n = blockIdx.y;
  const int a = dims[n], b = dims[n + 1];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < a * 2 * b; e += gridDim.x * blockDim.x) {
    const int al = e / (2 * b), rem = e % (2 * b), i = rem / b, be = rem % b;
    const size_t off = (size_t)n * dc * 2 * dc + (size_t)al * 2 * dc + i * dc + be;
    Bbar[off] = zscale(Bbar[off], w);
  }
}

// ============================================================================
// Gate adjoint kernels (sizes known on the host from the tape)
// ============================================================================
struct GateRec {      // device pointers of one tape record
  zd* Bl;
  zd* Br;
  double* lam;
  zd* C;
  zd* A;
  zd* V;
  double* sv;
  int* perm;
  int* meta;        // [0] = r, [4..6] = a, m, b
  double* dmeta;    // [0] = nu
};

struct AdjWork {
  zd* Wbar;   // [dc][ldw]
  zd* Kt;     // [ncap][dc]
  zd* Phi;    // [ncap][ldw]
  zd* T;      // [2dc][ldw]
  zd* Mbar;   // [2dc][ldw]
  zd* Cbar;   // [2dc][ldw]
  zd* Thb;    // [2dc][ldw]
  double* sbar;   // [dc]
  double* scal;   // [8]: nubar, kscale
  double* dpart;  // [1024] dphi partial sums
  int ldw;
};

struct GateDims {
  int n, a, m, b, r;
  double nu;
};

// One lane of a batched gate adjoint: the gate's tape record, a workspace and
// the cotangent buffers of the evaluation it belongs to.  Launches cover nl
// lanes with blockIdx.z = lane; grids are sized for the largest lane.
struct AdjLane {
  GateRec R;
  AdjWork W;
  GateDims d;
  zd* Bbn;            // Bbar_n of this evaluation
  zd* Bbn1;           // Bbar_{n+1}
  double* lb_out;     // lambar_{n} (bond of the gate, read then cleared)
  double* lb_in;      // lambar_{n-1} (accumulated)
  double* gphi;       // [G] dE/dphi of this evaluation
  const double* theta;
  GateTable gt;       // the lane's circuit
  int g;              // gate index in gt
  int kind;           // 1: PARAM gate (dE/dphi is written)
  int dc, ldc, ldv;   // bond capacity and leading dimensions of the tape's C, A and V
  double eta;         // Lorentzian broadening of the SVD adjoint (0: none)
};

// A1: Wbar[mu, c] = sum_row conj(Bbar_n[row, mu]) / nu * C[row, c] + Bbar_{n+1}[mu, c]
__global__ __launch_bounds__(256) void k_adj_wbar(const AdjLane* AL) {
  const AdjLane& ln = AL[blockIdx.z];
  const int dc = ln.dc, ldc = ln.ldc;
  const GateRec& R = ln.R;
  const AdjWork& W = ln.W;
  const GateDims& d = ln.d;
  const zd* Bbn = ln.Bbn;
  const zd* Bbn1 = ln.Bbn1;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  if (i0 >= d.r || j0 >= 2 * d.b) return;
  const double inv = 1.0 / d.nu;
  auto fa = [&](int mu, int row) {
    return zscale(zconj(Bbn[(size_t)(row >> 1) * 2 * dc + (row & 1) * dc + mu]), inv);
  };
  auto fb = [&](int row, int c) { return R.C[(size_t)c * ldc + row]; };
  zd acc[2][2];
  ztile_acc(d.r, 2 * d.b, 2 * d.a, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int mu = r0 + x, c = c0 + y;
      if (mu < d.r && c < 2 * d.b) {
        const int jp = c / d.b, be = c % d.b;
        W.Wbar[(size_t)mu * W.ldw + c] = zadd(acc[x][y], Bbn1[(size_t)mu * 2 * dc + jp * dc + be]);
      }
    }
}

// A2: nu_bar and s_bar of the kept values (one block)
__global__ __launch_bounds__(256) void k_adj_scalars(const AdjLane* AL) {
  const AdjLane& ln = AL[blockIdx.z];
  const int dc = ln.dc, ldv = ln.ldv;
  const GateRec& R = ln.R;
  const AdjWork& W = ln.W;
  const GateDims& d = ln.d;
  const zd* Bbn1 = ln.Bbn1;
  const double* lbar_out = ln.lb_out;
  __shared__ double red[256];
  const int t = threadIdx.x;
  double d1 = 0.0;
  for (int e = t; e < d.r * 2 * d.b; e += 256) {
    const int mu = e / (2 * d.b), c = e % (2 * d.b);
    const int jp = c / d.b, be = c % d.b;
    const zd g1 = zsub(W.Wbar[(size_t)mu * W.ldw + c], Bbn1[(size_t)mu * 2 * dc + jp * dc + be]);
    const zd v = R.V[(size_t)R.perm[mu] * ldv + c];
    d1 += g1.x * v.x - g1.y * v.y;
  }
  d1 = block_sum256(d1, red);
  double d2 = 0.0;
  for (int mu = t; mu < d.r; mu += 256) d2 += lbar_out[mu] * R.sv[R.perm[mu]];
  d2 = block_sum256(d2, red);
  const double nubar = -d1 / d.nu - d2 / (d.nu * d.nu);
  for (int mu = t; mu < d.r; mu += 256) W.sbar[mu] = lbar_out[mu] / d.nu + nubar * R.sv[R.perm[mu]] / d.nu;
  if (t == 0) W.scal[0] = nubar;
}

// A3: Kt[i, mu] = sum_c conj(P[c, i]) conj(Wbar[mu, c]),  P = V[:, perm]
__global__ __launch_bounds__(256) void k_adj_K(const AdjLane* AL) {
  const AdjLane& ln = AL[blockIdx.z];
  const int dc = ln.dc, ldv = ln.ldv;
  const GateRec& R = ln.R;
  const AdjWork& W = ln.W;
  const GateDims& d = ln.d;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  const int nb = 2 * d.b;
  if (i0 >= nb || j0 >= d.r) return;
  auto fa = [&](int i, int c) { return zconj(R.V[(size_t)R.perm[i] * ldv + c]); };
  auto fb = [&](int c, int mu) { return zconj(W.Wbar[(size_t)mu * W.ldw + c]); };
  zd acc[2][2];
  ztile_acc(nb, d.r, nb, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int i = r0 + x, mu = c0 + y;
      if (i < nb && mu < d.r) W.Kt[(size_t)i * dc + mu] = acc[x][y];
    }
}

// A4: kscale = max |Kt| (one block, deterministic)
__global__ __launch_bounds__(256) void k_adj_kscale(const AdjLane* AL) {
  const AdjLane& ln = AL[blockIdx.z];
  const int dc = ln.dc;
  const AdjWork& W = ln.W;
  const GateDims& d = ln.d;
  __shared__ double red[256];
  const int t = threadIdx.x;
  double m = 0.0;
  for (int e = t; e < 2 * d.b * d.r; e += 256) {
    const int i = e / d.r, mu = e % d.r;
    m = fmax(m, sqrt(zabs2(W.Kt[(size_t)i * dc + mu])));
  }
  red[t] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) red[t] = fmax(red[t], red[t + s]);
    __syncthreads();
  }
  if (t == 0) W.scal[1] = red[0];
}

// A5: Phi (sorted basis), Gamma_ij / s_i of the complex SVD adjoint
__global__ void k_adj_phi(const AdjLane* AL, GateStats* st) {
  const AdjLane& ln = AL[blockIdx.z];
  const double eta = ln.eta;
  const int dc = ln.dc;
  const GateRec& R = ln.R;
  const AdjWork& W = ln.W;
  const GateDims& d = ln.d;
  const int nb = 2 * d.b;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nb * nb) return;
  const int i = e / nb, j = e % nb;
  const int r = d.r;
  const double si = R.sv[R.perm[i]], sj = R.sv[R.perm[j]];
  zd phi = zmk(0.0, 0.0);
  if (i == j) {
    if (i < r) {
      const zd kii = W.Kt[(size_t)i * dc + i];
      phi = zmk(W.sbar[i] / si, -kii.y / (si * si));
    }
  } else if (i < r || j < r) {
    const zd kij = j < r ? W.Kt[(size_t)i * dc + j] : zmk(0.0, 0.0);
    const zd kji = i < r ? W.Kt[(size_t)j * dc + i] : zmk(0.0, 0.0);
    const zd aij = zsub(kij, zconj(kji));
    if (fabs(sj - si) < 1e-10 * fmax(si, sj)) {
      // exactly degenerate pair: the energy is invariant under rotations inside a
      // kept block, so a_ij vanishes; one that does not has no finite derivative
      if (sqrt(zabs2(aij)) > 1e-8 * W.scal[1]) atomicAdd(&st->degen_grad, 1);
    } else {
      const double dd = sj * sj - si * si;
      const double F = eta > 0.0 ? dd / (dd * dd + eta * eta) : 1.0 / dd;
      phi = zscale(aij, F);
    }
  }
  W.Phi[(size_t)i * W.ldw + j] = phi;
}

// A6: T[row, j] = sum_i A[row, perm i] Phi[i, j]
__global__ __launch_bounds__(256) void k_adj_T(const AdjLane* AL) {
  const AdjLane& ln = AL[blockIdx.z];
  const int ldc = ln.ldc;
  const GateRec& R = ln.R;
  const AdjWork& W = ln.W;
  const GateDims& d = ln.d;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  const int M = 2 * d.a, nb = 2 * d.b;
  if (i0 >= M || j0 >= nb) return;
  auto fa = [&](int row, int i) { return R.A[(size_t)R.perm[i] * ldc + row]; };
  auto fb = [&](int i, int j) { return W.Phi[(size_t)i * W.ldw + j]; };
  zd acc[2][2];
  ztile_acc(M, nb, nb, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y)
      if (r0 + x < M && c0 + y < nb) W.T[(size_t)(r0 + x) * W.ldw + c0 + y] = acc[x][y];
}

// A7: Mbar[row, c] = sum_j T[row, j] conj(P[c, j])
__global__ __launch_bounds__(256) void k_adj_Mbar(const AdjLane* AL) {
  const AdjLane& ln = AL[blockIdx.z];
  const int ldv = ln.ldv;
  const GateRec& R = ln.R;
  const AdjWork& W = ln.W;
  const GateDims& d = ln.d;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  const int M = 2 * d.a, nb = 2 * d.b;
  if (i0 >= M || j0 >= nb) return;
  auto fa = [&](int row, int j) { return W.T[(size_t)row * W.ldw + j]; };
  auto fb = [&](int j, int c) { return zconj(R.V[(size_t)R.perm[j] * ldv + c]); };
  zd acc[2][2];
  ztile_acc(M, nb, nb, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y)
      if (r0 + x < M && c0 + y < nb) W.Mbar[(size_t)(r0 + x) * W.ldw + c0 + y] = acc[x][y];
}

// A8: Cbar[row, c] = sum_mu Bbar_n[row, mu]/nu conj(P[c, mu]) + lambda_in[alpha] Mbar[row, c]
__global__ __launch_bounds__(256) void k_adj_Cbar(const AdjLane* AL) {
  const AdjLane& ln = AL[blockIdx.z];
  const int dc = ln.dc, ldv = ln.ldv;
  const GateRec& R = ln.R;
  const AdjWork& W = ln.W;
  const GateDims& d = ln.d;
  const zd* Bbn = ln.Bbn;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  const int M = 2 * d.a, nb = 2 * d.b;
  if (i0 >= M || j0 >= nb) return;
  const double inv = 1.0 / d.nu;
  auto fa = [&](int row, int mu) {
    return zscale(Bbn[(size_t)(row >> 1) * 2 * dc + (row & 1) * dc + mu], inv);
  };
  auto fb = [&](int mu, int c) { return zconj(R.V[(size_t)R.perm[mu] * ldv + c]); };
  zd acc[2][2];
  ztile_acc(M, nb, d.r, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int row = r0 + x, c = c0 + y;
      if (row < M && c < nb) {
        const size_t o = (size_t)row * W.ldw + c;
        W.Cbar[o] = zadd(acc[x][y], zscale(W.Mbar[o], R.lam[row >> 1]));
      }
    }
}

// A9: lambar_{n-1}[alpha] += Re sum conj(Mbar[(alpha,i'), c]) C[(alpha,i'), c]
__global__ __launch_bounds__(256) void k_adj_lambar(const AdjLane* AL) {
  const AdjLane& ln = AL[blockIdx.z];
  const int ldc = ln.ldc;
  const GateRec& R = ln.R;
  const AdjWork& W = ln.W;
  const GateDims& d = ln.d;
  double* lbar_in = ln.lb_in;
  __shared__ double red[256];
  const int al = blockIdx.x;
  if (al >= d.a) return;
  const int nb = 2 * d.b;
  double s = 0.0;
  for (int e = threadIdx.x; e < 2 * nb; e += 256) {
    const int ip = e / nb, c = e % nb;
    const int row = 2 * al + ip;
    const zd mb = W.Mbar[(size_t)row * W.ldw + c], cc = R.C[(size_t)c * ldc + row];
    s += mb.x * cc.x + mb.y * cc.y;
  }
  s = block_sum256(s, red);
  if (threadIdx.x == 0) lbar_in[al] += s;
}

// A10: Theta_bar = Q^dagger C_bar on (i', j'); dphi partial sums Re <C_bar, D C>
__global__ __launch_bounds__(256) void k_adj_theta(const AdjLane* AL) {
  const AdjLane& ln = AL[blockIdx.z];
  const GateTable& gt = ln.gt;
  const int g = ln.g, ldc = ln.ldc;
  const GateRec& R = ln.R;
  const AdjWork& W = ln.W;
  const GateDims& d = ln.d;
  const double* theta = ln.theta;
  __shared__ zd Q[16];
  __shared__ zd D[16];
  __shared__ double red[256];
  const int t = threadIdx.x;
  gate_matrix(gt, g, theta, Q);
  const bool param = gt.kind[g] == 1;
  if (param && t < 16) {
    // D = -(i/2) post ZZ post^dagger
    const zd* post = gt.post + (size_t)g * 16;
    const int r = t >> 2, c = t & 3;
    zd acc = zmk(0.0, 0.0);
    for (int k = 0; k < 4; ++k) {
      const double zz = (k == 0 || k == 3) ? 1.0 : -1.0;
      acc = zfma(zscale(post[r * 4 + k], zz), zconj(post[c * 4 + k]), acc);
    }
    D[t] = zmk(0.5 * acc.y, -0.5 * acc.x);
  }
  __syncthreads();
  const int e = blockIdx.x * 256 + t;
  double part = 0.0;
  if (e < d.a * d.b) {
    const int al = e / d.b, be = e % d.b;
    zd cb[4], cc[4];
    for (int ip = 0; ip < 2; ++ip)
      for (int jp = 0; jp < 2; ++jp) {
        const int row = 2 * al + ip, col = jp * d.b + be;
        cb[ip * 2 + jp] = W.Cbar[(size_t)row * W.ldw + col];
        cc[ip * 2 + jp] = R.C[(size_t)col * ldc + row];
      }
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        zd v = zmk(0.0, 0.0);
        for (int k = 0; k < 4; ++k) v = zfmac(Q[k * 4 + i * 2 + j], cb[k], v);
        W.Thb[(size_t)(2 * al + i) * W.ldw + j * d.b + be] = v;
      }
    if (param)
      for (int k = 0; k < 4; ++k) {
        zd dc_ = zmk(0.0, 0.0);
        for (int l = 0; l < 4; ++l) dc_ = zfma(D[k * 4 + l], cc[l], dc_);
        part += cb[k].x * dc_.x + cb[k].y * dc_.y;
      }
  }
  part = block_sum256(part, red);
  if (t == 0) W.dpart[blockIdx.x] = part;
}

// A11: Bbar_n[(alpha,i), gamma] = sum_c Theta_bar[(alpha,i), c] conj(B_{n+1}[gamma, c])
__global__ __launch_bounds__(256) void k_adj_Bl(const AdjLane* AL) {
  const AdjLane& ln = AL[blockIdx.z];
  const int dc = ln.dc;
  const GateRec& R = ln.R;
  const AdjWork& W = ln.W;
  const GateDims& d = ln.d;
  zd* Bbn = ln.Bbn;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  const int M = 2 * d.a;
  if (i0 >= M || j0 >= d.m) return;
  auto fa = [&](int row, int c) { return W.Thb[(size_t)row * W.ldw + c]; };
  auto fb = [&](int c, int ga) {
    const int jp = c / d.b, be = c % d.b;
    return zconj(R.Br[(size_t)ga * 2 * dc + jp * dc + be]);
  };
  zd acc[2][2];
  ztile_acc(M, d.m, 2 * d.b, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int row = r0 + x, ga = c0 + y;
      if (row < M && ga < d.m) Bbn[(size_t)(row >> 1) * 2 * dc + (row & 1) * dc + ga] = acc[x][y];
    }
}

// A12: Bbar_{n+1}[gamma, c] = sum_row conj(B_n[row, gamma]) Theta_bar[row, c]
__global__ __launch_bounds__(256) void k_adj_Br(const AdjLane* AL) {
  const AdjLane& ln = AL[blockIdx.z];
  const int dc = ln.dc;
  const GateRec& R = ln.R;
  const AdjWork& W = ln.W;
  const GateDims& d = ln.d;
  zd* Bbn1 = ln.Bbn1;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  const int nb = 2 * d.b;
  if (i0 >= d.m || j0 >= nb) return;
  auto fa = [&](int ga, int row) { return zconj(R.Bl[(size_t)(row >> 1) * 2 * dc + (row & 1) * dc + ga]); };
  auto fb = [&](int row, int c) { return W.Thb[(size_t)row * W.ldw + c]; };
  zd acc[2][2];
  ztile_acc(d.m, nb, 2 * d.a, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      const int ga = r0 + x, c = c0 + y;
      if (ga < d.m && c < nb) {
        const int jp = c / d.b, be = c % d.b;
        Bbn1[(size_t)ga * 2 * dc + jp * dc + be] = acc[x][y];
      }
    }
}

// A13: lambar_n = 0 (the old lambda_n was overwritten by this gate); dE/dphi
__global__ void k_adj_finish(const AdjLane* AL, int nparts) {
  const AdjLane& ln = AL[blockIdx.z];
  const int dc = ln.dc, g = ln.g, param = ln.kind;
  const AdjWork& W = ln.W;
  double* lbar_out = ln.lb_out;
  double* gphi = ln.gphi;
  for (int q = threadIdx.x; q < dc; q += blockDim.x) lbar_out[q] = 0.0;
  if (threadIdx.x == 0 && param) {
    double s = 0.0;
    for (int k = 0; k < nparts; ++k) s += W.dpart[k];
    gphi[g] = s;
  }
}

// S9: grad[p] = sum_{g: param_g = p} coeff_g gphi[g]  (fixed order per parameter)
__global__ void k_chain_rule(const int* gstart, const int* glist, GateTable gt, const double* gphi, double* grad,
                             int n_theta) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_theta) return;
  double s = 0.0;
  for (int k = gstart[p]; k < gstart[p + 1]; ++k) {
    const int g = glist[k];
    s += gt.coeff[g] * gphi[g];
  }
  grad[p] = s;
}

// ============================================================================
// Host: sweep adjoint
// ============================================================================
static inline dim3 gemm_grid(int M, int N, int z = 1) {
  return dim3((N + ZT_N - 1) / ZT_N, (M + ZT_M - 1) / ZT_M, z);
}

struct SweepAdjPlan {
  bool built = false;
  int dc = 0;
  std::vector<int> dims;          // final MPS dims used to build
  // per chunk, per site: job ranges in d_jobs
  struct SiteJobs { size_t off = 0; int nj = 0; };
  struct ChunkJobs {
    int lo = 0, hi = -1;
    std::vector<SiteJobs> right, left;
    std::vector<SiteJobs> injR, injL;   // per site m (index m - lo), items in d_inj
  };
  std::vector<ChunkJobs> chunks;
  std::vector<EnvJob> jobs_h;
  std::vector<InjectItem> inj_h;
  DevBuf d_jobs, d_inj, d_small;
  DevBuf Rslots, Lslots, Y, Gb, Lagg, Ragg;
  const zd* lid = nullptr;   // environment buffers the job pointers refer to
  const zd* rid = nullptr;
  int chunk_slots = 0;
  // precision 1: the term jobs on FP32 copies of the buffers
  bool f32 = false;
  DevBuf Rslots32, Lslots32, Y32, Gb32, d_jobs32, d_inj32;
  const cf* lid32 = nullptr;
  const cf* rid32 = nullptr;
};

struct BatchSet;
struct MixSet;
struct PlanAdj {
  SweepAdjPlan sw;
  DevBuf chain_start, chain_list;
  bool chain_built = false;
  BatchSet* batch = nullptr;   // lanes of the batched form (allocated on first use)
  MixSet* mix = nullptr;       // lanes of mixed-instance calls led by this plan
  ~PlanAdj();
};

static PlanAdj& adj_of(mps_plan* p) {
  if (!p->adj) p->adj = new PlanAdj();
  return *(PlanAdj*)p->adj;
}

void plan_adj_free(void* a) { delete (PlanAdj*)a; }

static zd* envp(zd* base, int dc, int k) { return base + (size_t)k * dc * dc; }

static void build_sweep_adjoint(mps_plan* p, SweepAdjPlan& S, const std::vector<int>& dims) {
  mps_ctx* ctx = p->ctx;
  DevHamiltonian& H = p->H;
  const int N = p->N;
  const int dc = p->state->dcap;
  const size_t dd = (size_t)dc * dc;
  const int64_t K = H.K;
  // chunking by memory: R slots (one per site of the support) + L slot + Y + G
  const size_t budget = ctx->sweep_budget;
  std::vector<std::pair<int64_t, int64_t>> ranges;
  int max_slots = 0, max_terms = 0;
  {
    int64_t lo = 0;
    size_t slots = 0;
    for (int64_t j = 0; j < K; ++j) {
      const int64_t k = H.order[j];
      const size_t s = (size_t)(H.b_t[k] - H.a_t[k] + 1);
      const size_t need = (slots + s + 5 * (size_t)(j - lo + 1)) * dd * sizeof(zd);
      if (j > lo && (need > budget || j - lo >= 60000)) {
        ranges.push_back({lo, j});
        max_slots = std::max<int>(max_slots, (int)slots);
        max_terms = std::max<int>(max_terms, (int)(j - lo));
        lo = j;
        slots = 0;
      }
      slots += s;
    }
    if (K > lo) {
      ranges.push_back({lo, K});
      max_slots = std::max<int>(max_slots, (int)slots);
      max_terms = std::max<int>(max_terms, (int)(K - lo));
    }
  }
  max_terms = std::max(max_terms, 3);
  zd* Rs = (zd*)S.Rslots.ensure((size_t)std::max(1, max_slots) * dd * sizeof(zd));
  zd* Ls = (zd*)S.Lslots.ensure((size_t)max_terms * dd * sizeof(zd));
  zd* Yb = (zd*)S.Y.ensure((size_t)max_terms * 2 * dd * sizeof(zd));
  zd* Gb = (zd*)S.Gb.ensure((size_t)max_terms * 2 * dd * sizeof(zd));
  zd* Lagg = (zd*)S.Lagg.ensure((size_t)(N + 1) * dd * sizeof(zd));
  zd* Ragg = (zd*)S.Ragg.ensure((size_t)(N + 1) * dd * sizeof(zd));
  (void)Lagg;
  (void)Ragg;
  zd* Lid = ctx->sb.Lid;
  zd* Rid = ctx->sb.Rid;
  S.jobs_h.clear();
  S.inj_h.clear();
  S.chunks.clear();
  for (auto& rg : ranges) {
    SweepAdjPlan::ChunkJobs ch;
    ch.lo = N;
    ch.hi = -1;
    std::vector<int> base(rg.second - rg.first);
    int slots = 0;
    for (int64_t j = rg.first; j < rg.second; ++j) {
      const int64_t k = H.order[j];
      ch.lo = std::min(ch.lo, H.a_t[k]);
      ch.hi = std::max(ch.hi, H.b_t[k]);
      base[j - rg.first] = slots;
      slots += H.b_t[k] - H.a_t[k] + 1;
    }
    auto rslot = [&](int64_t j, int m) {   // R^{(k)}_m for m in [a_k, b_k]
      const int64_t k = H.order[j];
      return envp(Rs, dc, base[j - rg.first] + (m - H.a_t[k]));
    };
    auto phases = [&](int64_t k, int n, EnvJob& jb) {
      const int xb = (H.xs[k] >> n) & 1, zb = (H.zs[k] >> n) & 1;
      const zd base_ = (xb && zb) ? zmk(0.0, 1.0) : zmk(1.0, 0.0);
      jb.xb = xb;
      jb.o0 = base_;
      jb.o1 = zb ? zmk(-base_.x, -base_.y) : base_;
    };
    const int ns = ch.hi - ch.lo + 1;
    ch.right.resize(ns);
    ch.left.resize(ns);
    ch.injR.resize(ns);
    ch.injL.resize(ns);
    // right sweep: site m, R^{(k)}_m = T_m(R^{(k)}_{m+1})
    for (int m = ch.hi; m >= ch.lo; --m) {
      SweepAdjPlan::SiteJobs sj;
      sj.off = S.jobs_h.size();
      int z = 0;
      for (int64_t j = rg.first; j < rg.second; ++j) {
        const int64_t k = H.order[j];
        if (!(H.a_t[k] <= m && m <= H.b_t[k])) continue;
        EnvJob jb{};
        jb.in = (m == H.b_t[k]) ? envp(Rid, dc, m + 1) : rslot(j, m + 1);
        jb.out = rslot(j, m);
        jb.y = Yb + (size_t)z * 2 * dd;
        jb.acc = 0;
        jb.c = H.coeff_h[k];
        phases(k, m, jb);
        S.jobs_h.push_back(jb);
        ++z;
      }
      sj.nj = z;
      ch.right[m - ch.lo] = sj;
    }
    // injections of rho_k = R^{(k)}_{a_k} into Ragg[a_k]
    for (int m = ch.lo; m <= ch.hi; ++m) {
      SweepAdjPlan::SiteJobs sj;
      sj.off = S.inj_h.size();
      for (int64_t j = rg.first; j < rg.second; ++j) {
        const int64_t k = H.order[j];
        if (H.a_t[k] == m) S.inj_h.push_back(InjectItem{rslot(j, m), H.coeff_h[k], 0.0});
      }
      sj.nj = (int)(S.inj_h.size() - sj.off);
      ch.injR[m - ch.lo] = sj;
    }
    // left sweep with contributions; L slot per term
    for (int n = ch.lo; n <= ch.hi; ++n) {
      SweepAdjPlan::SiteJobs sj;
      sj.off = S.jobs_h.size();
      int z = 0;
      for (int64_t j = rg.first; j < rg.second; ++j) {
        const int64_t k = H.order[j];
        if (!(H.a_t[k] <= n && n <= H.b_t[k])) continue;
        EnvJob jb{};
        zd* Lk = envp(Ls, dc, (int)(j - rg.first));
        jb.in = (n == H.a_t[k]) ? envp(Lid, dc, n) : Lk;
        jb.out = Lk;
        jb.y = Yb + (size_t)z * 2 * dd;
        jb.g = Gb + (size_t)z * 2 * dd;
        jb.rr = (n == H.b_t[k]) ? envp(Rid, dc, n + 1) : rslot(j, n + 1);
        jb.c = H.coeff_h[k];
        jb.acc = 0;
        phases(k, n, jb);
        S.jobs_h.push_back(jb);
        ++z;
      }
      sj.nj = z;
      ch.left[n - ch.lo] = sj;
      SweepAdjPlan::SiteJobs ij;
      ij.off = S.inj_h.size();
      for (int64_t j = rg.first; j < rg.second; ++j) {
        const int64_t k = H.order[j];
        if (H.b_t[k] == n) S.inj_h.push_back(InjectItem{envp(Ls, dc, (int)(j - rg.first)), H.coeff_h[k], 0.0});
      }
      ij.nj = (int)(S.inj_h.size() - ij.off);
      ch.injL[n - ch.lo] = ij;
    }
    S.chunks.push_back(ch);
  }
  upload(S.d_jobs, S.jobs_h.data(), S.jobs_h.size(), ctx->stream);
  upload(S.d_inj, S.inj_h.data(), S.inj_h.size(), ctx->stream);
  S.d_small.ensure(16 * sizeof(EnvJob));
  // precision 1: the same jobs on FP32 copies of the slot, scratch and identity
  // environment buffers (a pointer keeps its element offset)
  S.f32 = p->trunc.precision == 1;
  if (S.f32) {
    struct Map {
      const zd* b64;
      size_t n;
      cf* b32;
    };
    const Map maps[] = {
        {Rs, (size_t)std::max(1, max_slots) * dd, (cf*)S.Rslots32.ensure((size_t)std::max(1, max_slots) * dd * sizeof(cf))},
        {Ls, (size_t)max_terms * dd, (cf*)S.Lslots32.ensure((size_t)max_terms * dd * sizeof(cf))},
        {Yb, (size_t)max_terms * 2 * dd, (cf*)S.Y32.ensure((size_t)max_terms * 2 * dd * sizeof(cf))},
        {Gb, (size_t)max_terms * 2 * dd, (cf*)S.Gb32.ensure((size_t)max_terms * 2 * dd * sizeof(cf))},
        {Lid, (size_t)(N + 1) * dd, ctx->s32.Lid},
        {Rid, (size_t)(N + 1) * dd, ctx->s32.Rid}};
    auto tr = [&](const zd* q) -> cf* {
      if (!q) return nullptr;
      for (const Map& m : maps)
        if (q >= m.b64 && q < m.b64 + m.n) return m.b32 + (q - m.b64);
      fail(MPS_EDEVICE, "sweep adjoint: job pointer outside its buffers");
      return nullptr;
    };
    std::vector<EnvJob32> j32(S.jobs_h.size());
    for (size_t q = 0; q < S.jobs_h.size(); ++q) {
      const EnvJob& jb = S.jobs_h[q];
      j32[q] = EnvJob32{tr(jb.in), tr(jb.out), tr(jb.y), tr(jb.rr), tr(jb.g), jb.c, jb.xb, jb.acc, jb.o0, jb.o1};
    }
    std::vector<InjectItem32> i32(S.inj_h.size());
    for (size_t q = 0; q < S.inj_h.size(); ++q) i32[q] = InjectItem32{tr(S.inj_h[q].src), S.inj_h[q].c, 0.0};
    upload(S.d_jobs32, j32.data(), j32.size(), ctx->stream);
    upload(S.d_inj32, i32.data(), i32.size(), ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));   // j32 / i32 are released at the end of this block
    S.lid32 = ctx->s32.Lid;
    S.rid32 = ctx->s32.Rid;
  }
  S.dims = dims;
  S.dc = dc;
  S.lid = Lid;
  S.rid = Rid;
  S.built = true;
}

// Site cotangents of E = c0 + sum_k c_k <P_k> / Z for the state st (final
// bond dims `dims`, energy E, norm Z) into Bbar.
static void run_sweep_adjoint(mps_plan* p, const std::vector<int>& dims, const mps_state* st, zd* Bbar, double E,
                              double Z) {
  mps_ctx* ctx = p->ctx;
  hipStream_t s = ctx->stream;
  SweepAdjPlan& S = adj_of(p).sw;
  // precision 1 computed the energy on FP32 environments: the adjoint takes
  // the FP64 ones of the same state
  if (st->trunc.precision == 1) run_identity_envs(const_cast<mps_state*>(st));
  const bool f32 = st->trunc.precision == 1;
  if (!S.built || S.dims != dims || S.lid != ctx->sb.Lid || S.rid != ctx->sb.Rid || S.f32 != f32 ||
      (f32 && (S.lid32 != ctx->s32.Lid || S.rid32 != ctx->s32.Rid)))
    build_sweep_adjoint(p, S, dims);
  const int N = p->N, dc = S.dc;
  const size_t dd = (size_t)dc * dc;
  zd* Lagg = (zd*)S.Lagg.p;
  zd* Ragg = (zd*)S.Ragg.p;
  const zd* B = (const zd*)st->B.p;
  const size_t site = (size_t)dc * 2 * dc;
  HIPCHK(hipMemsetAsync(Bbar, 0, (size_t)N * site * sizeof(zd), s));
  HIPCHK(hipMemsetAsync(Lagg, 0, (size_t)(N + 1) * dd * sizeof(zd), s));
  HIPCHK(hipMemsetAsync(Ragg, 0, (size_t)(N + 1) * dd * sizeof(zd), s));
  const EnvJob* J = (const EnvJob*)S.d_jobs.p;
  const InjectItem* I = (const InjectItem*)S.d_inj.p;
  const EnvJob32* J32 = (const EnvJob32*)S.d_jobs32.p;
  const InjectItem32* I32 = (const InjectItem32*)S.d_inj32.p;
  const cf* B32 = ctx->s32.B;   // the FP32 sites of st (converted by its energy sweep)
  for (auto& ch : S.chunks) {
    if (f32) {
      // the per-term transfers on the matrix cores; cotangents accumulate in FP64
      for (int m = ch.hi; m >= ch.lo; --m) {
        const auto& sj = ch.right[m - ch.lo];
        if (sj.nj) HIPCHK(launch_env32_right(J32 + sj.off, sj.nj, B32 + (size_t)m * site, dims[m], dims[m + 1], dc, s));
      }
      for (int m = ch.lo; m <= ch.hi; ++m) {
        const auto& ij = ch.injR[m - ch.lo];
        if (ij.nj) HIPCHK(launch_inject32(I32 + ij.off, ij.nj, Ragg + (size_t)m * dd, dims[m], dc, s));
      }
      for (int n = ch.lo; n <= ch.hi; ++n) {
        const auto& sj = ch.left[n - ch.lo];
        if (sj.nj)
          HIPCHK(launch_env32_left(J32 + sj.off, sj.nj, B32 + (size_t)n * site, Bbar + (size_t)n * site, dims[n],
                                   dims[n + 1], dc, s));
        const auto& ij = ch.injL[n - ch.lo];
        if (ij.nj) HIPCHK(launch_inject32(I32 + ij.off, ij.nj, Lagg + (size_t)(n + 1) * dd, dims[n + 1], dc, s));
      }
      continue;
    }
    for (int m = ch.hi; m >= ch.lo; --m) {
      const auto& sj = ch.right[m - ch.lo];
      const int a = dims[m], b = dims[m + 1];
      if (sj.nj) {
        hipLaunchKernelGGL(k_env_right1, gemm_grid(2 * a, b, sj.nj), dim3(256), 0, s, J + sj.off, B + (size_t)m * site, a, b, dc);
        hipLaunchKernelGGL(k_env_right2, gemm_grid(a, a, sj.nj), dim3(256), 0, s, J + sj.off, B + (size_t)m * site, a, b, dc);
      }
    }
    for (int m = ch.lo; m <= ch.hi; ++m) {
      const auto& ij = ch.injR[m - ch.lo];
      const int d = dims[m];
      if (ij.nj) hipLaunchKernelGGL(k_inject, dim3((d * d + 255) / 256), dim3(256), 0, s, I + ij.off, ij.nj, Ragg + (size_t)m * dd, d, dc);
    }
    for (int n = ch.lo; n <= ch.hi; ++n) {
      const auto& sj = ch.left[n - ch.lo];
      const int a = dims[n], b = dims[n + 1];
      const zd* Bn = B + (size_t)n * site;
      if (sj.nj) {
        hipLaunchKernelGGL(k_env_left1, gemm_grid(a, 2 * b, sj.nj), dim3(256), 0, s, J + sj.off, Bn, a, b, dc);
        const int ta = (a + ZT_M - 1) / ZT_M;
        hipLaunchKernelGGL(k_env_contrib, dim3((b + ZT_N - 1) / ZT_N, 2 * ta, sj.nj), dim3(256), 0, s, J + sj.off, a, b, dc);
        hipLaunchKernelGGL(k_env_reduce, dim3((a * 2 * b + 255) / 256), dim3(256), 0, s, J + sj.off, sj.nj,
                           Bbar + (size_t)n * site, a, b, dc);
        hipLaunchKernelGGL(k_env_left2, gemm_grid(b, b, sj.nj), dim3(256), 0, s, J + sj.off, Bn, a, b, dc);
      }
      const auto& ij = ch.injL[n - ch.lo];
      const int d = dims[n + 1];
      if (ij.nj) hipLaunchKernelGGL(k_inject, dim3((d * d + 255) / 256), dim3(256), 0, s, I + ij.off, ij.nj, Lagg + (size_t)(n + 1) * dd, d, dc);
    }
  }
  // aggregated environments outside the supports, and the Z term
  zd* Yb = (zd*)S.Y.p;
  zd* Gb = (zd*)S.Gb.p;
  EnvJob* dj = (EnvJob*)S.d_small.p;
  std::vector<EnvJob> hj(3);
  const zd one = zmk(1.0, 0.0);
  // Lagg_{m+1} += T_m(Lagg_m)
  for (int m = 0; m < N; ++m) {
    const int a = dims[m], b = dims[m + 1];
    EnvJob jb{};
    jb.in = Lagg + (size_t)m * dd;
    jb.out = Lagg + (size_t)(m + 1) * dd;
    jb.y = Yb;
    jb.acc = 1;
    jb.o0 = one;
    jb.o1 = one;
    HIPCHK(hipMemcpyAsync(dj + 0, &jb, sizeof(EnvJob), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_env_left1, gemm_grid(a, 2 * b), dim3(256), 0, s, dj, B + (size_t)m * site, a, b, dc);
    hipLaunchKernelGGL(k_env_left2, gemm_grid(b, b), dim3(256), 0, s, dj, B + (size_t)m * site, a, b, dc);
    HIPCHK(hipStreamSynchronize(s));   // dj is reused
  }
  for (int m = N - 1; m >= 0; --m) {
    const int a = dims[m], b = dims[m + 1];
    EnvJob jb{};
    jb.in = Ragg + (size_t)(m + 1) * dd;
    jb.out = Ragg + (size_t)m * dd;
    jb.y = Yb;
    jb.acc = 1;
    jb.o0 = one;
    jb.o1 = one;
    HIPCHK(hipMemcpyAsync(dj + 0, &jb, sizeof(EnvJob), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_env_right1, gemm_grid(2 * a, b), dim3(256), 0, s, dj, B + (size_t)m * site, a, b, dc);
    hipLaunchKernelGGL(k_env_right2, gemm_grid(a, a), dim3(256), 0, s, dj, B + (size_t)m * site, a, b, dc);
    HIPCHK(hipStreamSynchronize(s));
  }
  const double zc = -(E - p->H.c0);
  for (int n = 0; n < N; ++n) {
    const int a = dims[n], b = dims[n + 1];
    const zd* Bn = B + (size_t)n * site;
    for (int q = 0; q < 3; ++q) {
      EnvJob jb{};
      jb.y = Yb + (size_t)(q == 0 ? 0 : 1) * 2 * dd;
      jb.g = Gb + (size_t)q * 2 * dd;
      jb.o0 = one;
      jb.o1 = one;
      jb.c = q == 2 ? zc : 1.0;
      jb.in = q == 0 ? Lagg + (size_t)n * dd : ctx->sb.Lid + (size_t)n * dd;
      jb.rr = q == 1 ? Ragg + (size_t)(n + 1) * dd : ctx->sb.Rid + (size_t)(n + 1) * dd;
      hj[q] = jb;
    }
    HIPCHK(hipMemcpyAsync(dj, hj.data(), 3 * sizeof(EnvJob), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_env_left1, gemm_grid(a, 2 * b, 2), dim3(256), 0, s, dj, Bn, a, b, dc);
    const int ta = (a + ZT_M - 1) / ZT_M;
    hipLaunchKernelGGL(k_env_contrib, dim3((b + ZT_N - 1) / ZT_N, 2 * ta, 3), dim3(256), 0, s, dj, a, b, dc);
    hipLaunchKernelGGL(k_env_reduce, dim3((a * 2 * b + 255) / 256), dim3(256), 0, s, dj, 3, Bbar + (size_t)n * site, a, b, dc);
    HIPCHK(hipStreamSynchronize(s));
  }
  hipLaunchKernelGGL(k_scale_sites, dim3(64, N), dim3(256), 0, s, Bbar, (const int*)st->dims.p, N, dc,
                     2.0 / Z);
  HIPCHK(hipGetLastError());
}

// ============================================================================
// Host: gate adjoint over checkpoint segments
// ============================================================================
static size_t al256(size_t x) { return (x + 255) / 256 * 256; }

static GateRec rec_at(char* base, const TapeLayout& L, int k) {
  char* r = base + (size_t)k * L.rec;
  GateRec R;
  R.Bl = (zd*)(r + L.oBl);
  R.Br = (zd*)(r + L.oBr);
  R.lam = (double*)(r + L.olam);
  R.C = (zd*)(r + L.oC);
  R.A = (zd*)(r + L.oA);
  R.V = (zd*)(r + L.oV);
  R.sv = (double*)(r + L.osv);
  R.perm = (int*)(r + L.operm);
  R.meta = (int*)(r + L.ometa);
  R.dmeta = (double*)(r + L.odmeta);
  return R;
}

static void build_chain(mps_plan* p, PlanAdj& A) {
  std::vector<int> start(p->n_theta + 1, 0), list;
  std::vector<std::vector<int>> per(p->n_theta);
  for (int g = 0; g < p->C.G; ++g)
    if (p->C.kind_h[g] == 1) per[p->C.param_h[g]].push_back(g);
  for (int q = 0; q < p->n_theta; ++q) {
    start[q] = (int)list.size();
    list.insert(list.end(), per[q].begin(), per[q].end());
  }
  start[p->n_theta] = (int)list.size();
  if (list.empty()) list.push_back(0);   // no PARAM gates: a one-entry placeholder, never read
  upload(A.chain_start, start.data(), start.size(), p->ctx->stream);
  upload(A.chain_list, list.data(), list.size(), p->ctx->stream);
  A.chain_built = true;
}

// Gate sizes of a batch of lanes, gathered from the tape records into
// [lane][step][16] ints (r, -, -, -, a, m, b) and doubles (nu) for one copy.
__global__ void k_gather_meta(const GateLane* lanes, TapeLayout L, int K, int* meta, double* dmeta) {
  const GateLane& ln = lanes[blockIdx.y];
  const int step = blockIdx.x, t = threadIdx.x;
  if (step >= ln.ng || t >= 16) return;
  const char* r = ln.tape + (size_t)step * L.rec;
  const size_t o = ((size_t)blockIdx.y * K + step) * 16 + t;
  meta[o] = ((const int*)(r + L.ometa))[t];
  dmeta[o] = ((const double*)(r + L.odmeta))[t];
}

// Copies the gate sizes of nl lanes (K steps each) to the host and checks
// them: 1 <= r, a, m, b <= dc for every recorded gate.
static void read_lane_meta(const GateLane* lanes_d, const std::vector<GateLane>& lh, int nl, const TapeLayout& L,
                           int K, int dc, DevBuf& dbuf, std::vector<int>& meta, std::vector<double>& dmeta,
                           hipStream_t s) {
  const size_t cnt = (size_t)nl * K * 16;
  char* d = (char*)dbuf.ensure(cnt * (sizeof(int) + sizeof(double)));
  int* dm = (int*)d;
  double* dd = (double*)(d + cnt * sizeof(int));
  hipLaunchKernelGGL(k_gather_meta, dim3(K, nl), dim3(64), 0, s, lanes_d, L, K, dm, dd);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(meta.data(), dm, cnt * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(dmeta.data(), dd, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int l = 0; l < nl; ++l)
    for (int k = 0; k < lh[l].ng; ++k) {
      const int* mt = meta.data() + ((size_t)l * K + k) * 16;
      const bool ok = mt[0] >= 1 && mt[0] <= dc && mt[4] >= 1 && mt[4] <= dc && mt[5] >= 1 && mt[5] <= dc &&
                      mt[6] >= 1 && mt[6] <= dc;
      if (!ok) fail(MPS_EDEVICE, "gate sizes read back from the tape are out of range");
    }
}

// Workspace of one lane of the gate adjoint.
static size_t adjwork_layout(int ncap, int dc, AdjWork* W, char* w) {
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = al256(o + bytes); return r; };
  const size_t zm = (size_t)ncap * ncap * sizeof(zd);
  const size_t oW = take(zm), oK = take((size_t)ncap * dc * sizeof(zd)), oP = take(zm), oT = take(zm),
               oM = take(zm), oCb = take(zm), oTh = take(zm), oS = take(dc * sizeof(double)),
               oSc = take(8 * sizeof(double)), oD = take(1024 * sizeof(double));
  if (W) {
    W->Wbar = (zd*)(w + oW);
    W->Kt = (zd*)(w + oK);
    W->Phi = (zd*)(w + oP);
    W->T = (zd*)(w + oT);
    W->Mbar = (zd*)(w + oM);
    W->Cbar = (zd*)(w + oCb);
    W->Thb = (zd*)(w + oTh);
    W->sbar = (double*)(w + oS);
    W->scal = (double*)(w + oSc);
    W->dpart = (double*)(w + oD);
    W->ldw = ncap;
  }
  return al256(o);
}

// The adjoint of one gate (A1..A13) for nl lanes; mx holds the largest sizes
// over the lanes, which set the grids.
static void launch_gate_adjoint(const AdjLane* al, int nl, const GateDims& mx, GateStats* stats, hipStream_t s) {
  const int M = 2 * mx.a, nb = 2 * mx.b;
  hipLaunchKernelGGL(k_adj_wbar, gemm_grid(mx.r, nb, nl), dim3(256), 0, s, al);
  hipLaunchKernelGGL(k_adj_scalars, dim3(1, 1, nl), dim3(256), 0, s, al);
  hipLaunchKernelGGL(k_adj_K, gemm_grid(nb, mx.r, nl), dim3(256), 0, s, al);
  hipLaunchKernelGGL(k_adj_kscale, dim3(1, 1, nl), dim3(256), 0, s, al);
  hipLaunchKernelGGL(k_adj_phi, dim3((nb * nb + 255) / 256, 1, nl), dim3(256), 0, s, al, stats);
  hipLaunchKernelGGL(k_adj_T, gemm_grid(M, nb, nl), dim3(256), 0, s, al);
  hipLaunchKernelGGL(k_adj_Mbar, gemm_grid(M, nb, nl), dim3(256), 0, s, al);
  hipLaunchKernelGGL(k_adj_Cbar, gemm_grid(M, nb, nl), dim3(256), 0, s, al);
  hipLaunchKernelGGL(k_adj_lambar, dim3(mx.a, 1, nl), dim3(256), 0, s, al);
  const int nparts = (mx.a * mx.b + 255) / 256;
  hipLaunchKernelGGL(k_adj_theta, dim3(nparts, 1, nl), dim3(256), 0, s, al);
  hipLaunchKernelGGL(k_adj_Bl, gemm_grid(M, mx.m, nl), dim3(256), 0, s, al);
  hipLaunchKernelGGL(k_adj_Br, gemm_grid(mx.m, nb, nl), dim3(256), 0, s, al);
  hipLaunchKernelGGL(k_adj_finish, dim3(1, 1, nl), dim3(256), 0, s, al, nparts);
}

// Sizes of a recorded gate (from the tape's meta fields read back to the host).
static GateDims dims_of(const int* mt, const double* dmt, int n) {
  GateDims d;
  d.n = n;
  d.r = mt[0];
  d.a = mt[4];
  d.m = mt[5];
  d.b = mt[6];
  d.nu = dmt[0];
  return d;
}

void plan_backward(mps_plan* p, double* grad, int on_device, mps_stats* stats) {
  mps_ctx* ctx = p->ctx;
  hipStream_t s = ctx->stream;
  PlanAdj& A = adj_of(p);
  mps_state* st = p->state;
  const int N = p->N, dc = st->dcap;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  // final dims
  std::vector<int> dims(N + 1);
  HIPCHK(hipMemcpyAsync(dims.data(), st->dims.p, (N + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const size_t site = (size_t)dc * 2 * dc;
  p->Bbar.ensure((size_t)N * site * sizeof(zd));
  p->lambar.ensure((size_t)(N + 1) * dc * sizeof(double));
  HIPCHK(hipMemsetAsync(p->lambar.p, 0, p->lambar.bytes, s));
  run_sweep_adjoint(p, dims, st, (zd*)p->Bbar.p, p->E, p->Z);
  // ---- gate adjoint
  GateWork gw = ctx->gw;
  const TapeLayout L = tape_layout(dc, gw.ncap, gw.ldc, gw.ldv);
  const int K = p->opts.ckpt_gates;
  // Segments are recomputed nl at a time, each segment a lane of one
  // gate-chain launch; the adjoint then walks the batch's segments in reverse
  // order.
  const size_t seg_bytes = (size_t)K * L.rec;
  const size_t tape_budget = (size_t)64 << 30;
  int nlanes = std::min({p->n_seg, lanes_max(dc), 64, (int)std::max<size_t>(1, tape_budget / seg_bytes)});
  nlanes = std::max(1, nlanes);
  char* tape = (char*)p->tape.ensure((size_t)nlanes * seg_bytes);
  while ((int)p->replays.size() < nlanes) p->replays.push_back(plan_new_state(ctx, N, st->trunc, nullptr));
  const size_t aux_lane = 128 * sizeof(int) + 256 * sizeof(double) + sizeof(GateStats) + 64;
  char* aux = (char*)p->lane_aux.ensure((size_t)nlanes * aux_lane + 64 + (size_t)nlanes * 8);
  int* lane_err = (int*)(aux + (size_t)nlanes * aux_lane);
  unsigned long long* lane_bars = (unsigned long long*)(aux + (size_t)nlanes * aux_lane + 64);
  HIPCHK(hipMemsetAsync(lane_err, 0, sizeof(int), s));
  GateLane* lanes_d = (GateLane*)p->lanes_dev.ensure((size_t)nlanes * sizeof(GateLane));
  p->lanes_h.resize(nlanes);
  LaneConst lc;
  lc.gt = p->C.tab;
  lc.L = L;
  lc.ldc = gw.ldc;
  lc.ldv = gw.ldv;
  lc.ncap = gw.ncap;
  lc.dmax = gw.dmax;
  lc.max_sweeps = gw.max_sweeps;
  lc.nparts = ((2 * dc + ZT_M - 1) / ZT_M) * ((2 * dc + ZT_M - 1) / ZT_M);
  lc.eps = gw.eps;
  lc.tol = gw.tol;
  lc.sched = gw.sched;
  lc.ck_B = lc.ck_dims = lc.ck_lam = 0;   // no checkpoint copies in the recompute
  AdjWork W;
  adjwork_layout(gw.ncap, dc, &W, (char*)p->work.ensure(adjwork_layout(gw.ncap, dc, nullptr, nullptr)));
  double* gphi = (double*)p->gphi.ensure((size_t)std::max(1, p->C.G) * sizeof(double));
  HIPCHK(hipMemsetAsync(gphi, 0, p->gphi.bytes, s));
  zd* Bbar = (zd*)p->Bbar.p;
  double* lambar = (double*)p->lambar.p;
  const double* th = (const double*)p->theta.p;
  std::vector<int> meta((size_t)nlanes * K * 16);
  std::vector<double> dmeta((size_t)nlanes * K * 16);
  std::vector<AdjLane> rec;      // lives until the final synchronisation below
  // the adjoint records of the largest batch, allocated once for the pass
  p->adjl_dev.ensure((size_t)nlanes * K * sizeof(AdjLane));
  std::vector<GateDims> dd;
  for (int hi = p->n_seg - 1; hi >= 0; hi -= nlanes) {
    const int lo = std::max(0, hi - nlanes + 1), nl = hi - lo + 1;
    int steps = 0;
    for (int l = 0; l < nl; ++l) {
      const int sg = lo + l;
      mps_state* rp = p->replays[l];
      plan_restore(p, sg, rp);
      GateLane& ln = p->lanes_h[l];
      ln.st = view_of(rp);
      ln.g0 = sg * K;
      ln.ng = std::min(p->C.G, (sg + 1) * K) - sg * K;
      ln.rec_stride = 1;
      ln.theta = (const double*)p->theta.p;
      ln.tape = tape + (size_t)l * seg_bytes;
      char* la = aux + (size_t)l * aux_lane;
      ln.rotflag = (int*)la;
      ln.nrm_part = (double*)(la + 128 * sizeof(int));
      ln.stats = (GateStats*)(la + 128 * sizeof(int) + 256 * sizeof(double));
      ln.bar = lane_bars + l;
      ln.err = lane_err;
      ln.ckpt = nullptr;
      ln.shift_gate = -1;
      ln.shift = 0.0;
      steps = std::max(steps, ln.ng);
    }
    HIPCHK(hipMemcpyAsync(lanes_d, p->lanes_h.data(), (size_t)nl * sizeof(GateLane), hipMemcpyHostToDevice, s));
    (void)steps;
    HIPCHK(launch_chain_lanes(lanes_d, nl, lc, true, lane_bars, s));
    // sizes of the batch's gates
    read_lane_meta(lanes_d, p->lanes_h, nl, L, K, dc, p->meta_dev, meta, dmeta, s);
    int err = 0;
    HIPCHK(hipMemcpyAsync(&err, lane_err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (err) fail(MPS_EDEVICE, "a lane barrier of the batched recompute timed out");
    // adjoint lane records of the whole batch (segments in reverse, gates in
    // reverse), uploaded once; each gate is then one lane-adjoint launch set
    rec.clear();
    dd.clear();
    for (int l = nl - 1; l >= 0; --l) {
      const GateLane& ln = p->lanes_h[l];
      for (int g = ln.g0 + ln.ng - 1; g >= ln.g0; --g) {
        const size_t k = (size_t)l * K + (g - ln.g0);
        AdjLane a1;
        a1.R = rec_at(ln.tape, L, g - ln.g0);
        a1.W = W;
        a1.d = dims_of(meta.data() + k * 16, dmeta.data() + k * 16, p->C.bond_h[g]);
        const int n = a1.d.n;
        a1.Bbn = Bbar + (size_t)n * site;
        a1.Bbn1 = Bbar + (size_t)(n + 1) * site;
        a1.lb_out = lambar + (size_t)(n + 1) * dc;
        a1.lb_in = lambar + (size_t)n * dc;
        a1.gphi = gphi;
        a1.theta = th;
        a1.gt = p->C.tab;
        a1.g = g;
        a1.kind = p->C.kind_h[g];
        a1.dc = dc;
        a1.ldc = gw.ldc;
        a1.ldv = gw.ldv;
        a1.eta = p->opts.broaden;
        rec.push_back(a1);
        dd.push_back(a1.d);
      }
    }
    AdjLane* rec_d = (AdjLane*)p->adjl_dev.ensure(rec.size() * sizeof(AdjLane));
    HIPCHK(hipMemcpyAsync(rec_d, rec.data(), rec.size() * sizeof(AdjLane), hipMemcpyHostToDevice, s));
    size_t k = 0;
    for (int l = nl - 1; l >= 0; --l) {
      const GateLane& ln = p->lanes_h[l];
      for (int g = ln.g0 + ln.ng - 1; g >= ln.g0; --g, ++k)
        launch_gate_adjoint(rec_d + k, 1, dd[k], gw.stats, s);
      HIPCHK(hipGetLastError());
      if (ctx->progress) {
        HIPCHK(hipStreamSynchronize(s));
        ctx->progress(ctx->progress_user, "backward", p->n_seg - (lo + l), p->n_seg);
      }
    }
    // the next batch rewrites the host records only after its metadata copy,
    // which synchronises the stream (and with it this batch's upload)
  }
  if (!A.chain_built) build_chain(p, A);
  double* gd_dev = (double*)p->grad.ensure((size_t)std::max(1, p->n_theta) * sizeof(double));
  if (p->n_theta > 0)
    hipLaunchKernelGGL(k_chain_rule, dim3((p->n_theta + 255) / 256), dim3(256), 0, s, (const int*)A.chain_start.p,
                       (const int*)A.chain_list.p, p->C.tab, (const double*)gphi, gd_dev, p->n_theta);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(e1, s));
  if (p->n_theta > 0)
    HIPCHK(hipMemcpyAsync(grad, gd_dev, p->n_theta * sizeof(double),
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  GateStats gs;
  HIPCHK(hipMemcpyAsync(&gs, gw.stats, sizeof(GateStats), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (stats) stats->t_backward_ms = ms;
  if (gs.degen_grad > 0 && p->opts.strict_degenerate)
    fail(MPS_EDEGEN, std::to_string(gs.degen_grad) + " degenerate singular pairs carry a cotangent");
}

// ============================================================================
// Batched form: energy and gradient of nb parameter vectors of one plan.  Each
// vector is a lane of the gate-chain kernel: one cooperative launch per
// checkpoint segment takes every lane through the segment's gates, each lane
// on its own work-groups and barrier; the reverse pass recomputes one
// checkpoint segment for all lanes at a time and runs the gate adjoint of all
// lanes in one launch set per gate.
// ============================================================================
struct BatchLane {
  mps_state* st = nullptr;   // forward state
  mps_state* rp = nullptr;   // segment replay state
  DevBuf ckpt, Bbar, lambar, gphi, grad, work;
  double E = 0.0, Eim = 0.0, Z = 0.0;
  ~BatchLane() {
    delete st;
    delete rp;
  }
};

struct BatchSet {
  std::vector<BatchLane*> lanes;
  DevBuf thetas, tape, aux, lanes_dev, adj_dev, meta_dev;
  DevBuf arc, arc_off;   // compact tape records of the forward pass and their offsets
  ~BatchSet() {
    for (BatchLane* l : lanes) delete l;
  }
};

// Compact copy of one tape record: only the entries the gate adjoint reads,
// at the gate's own sizes a, m, b (nb = 2b) -- meta, dmeta, perm[0..nb), the
// singular values sv[perm[i]], lambda_{n-1}[0..a), B_n [a][2][m], B_{n+1}
// [m][2][b], C (nb columns of 2a rows), the columns perm[i] of A (2a rows
// each) and the rows perm[i] of V (nb entries each), in that order.
struct ArcLayout {
  size_t meta, dmeta, perm, sv, lam, Bl, Br, C, A, V, total;
};

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) / 16 * 16; }

__host__ __device__ inline ArcLayout arc_layout(int a, int m, int b) {
  ArcLayout o;
  const size_t nb = 2 * (size_t)b, z = sizeof(zd);
  size_t x = 0;
  o.meta = x;  x = al16(x + 16 * sizeof(int));
  o.dmeta = x; x = al16(x + 16 * sizeof(double));
  o.perm = x;  x = al16(x + nb * sizeof(int));
  o.sv = x;    x = al16(x + nb * sizeof(double));
  o.lam = x;   x = al16(x + (size_t)a * sizeof(double));
  o.Bl = x;    x += (size_t)a * 2 * m * z;
  o.Br = x;    x += (size_t)m * 2 * b * z;
  o.C = x;     x += 2 * (size_t)a * nb * z;
  o.A = x;     x += 2 * (size_t)a * nb * z;
  o.V = x;     x += nb * nb * z;
  o.total = al16(x);
  return o;
}

template <class T>
__device__ inline void arc_move(T* rec, T* arc, int dir) {
  if (dir == 0)
    *arc = *rec;
  else
    *rec = *arc;
}

// dir 0: the records of each lane's current segment (lane tape, one record
// per step) to the archive; dir 1: back from the archive into the same
// places of the records.  One block per (step, lane); off[lane * K + step] is
// the record's byte offset in the archive, -1 = not archived.  The sizes come
// from the record's meta (dir 0) or the archived meta (dir 1); perm entries
// outside [0, ncap) are skipped.
__global__ __launch_bounds__(256) void k_tape_archive(const GateLane* lanes, TapeLayout L, int K, int dc, int ldc,
                                                      int ldv, int ncap, char* arc, const long long* off, int dir) {
  const int k = blockIdx.x, l = blockIdx.y, t = threadIdx.x;
  const GateLane& ln = lanes[l];
  if (k >= ln.ng) return;
  const long long o = off[(size_t)l * K + k];
  if (o < 0) return;
  char* r = ln.tape + (size_t)k * L.rec;
  char* q = arc + o;
  const int* msrc = dir == 0 ? (const int*)(r + L.ometa) : (const int*)q;
  const int a = msrc[4], m = msrc[5], b = msrc[6], nb = 2 * b;
  const ArcLayout O = arc_layout(a, m, b);
  int* rperm = (int*)(r + L.operm);
  int* qperm = (int*)(q + O.perm);
  const int* P = dir == 0 ? rperm : qperm;
  if (t < 16) {
    arc_move((int*)(r + L.ometa) + t, (int*)(q + O.meta) + t, dir);
    arc_move((double*)(r + L.odmeta) + t, (double*)(q + O.dmeta) + t, dir);
  }
  for (int i = t; i < nb; i += 256) {
    const int pi = P[i];
    arc_move(rperm + i, qperm + i, dir);
    if (pi >= 0 && pi < ncap) arc_move((double*)(r + L.osv) + pi, (double*)(q + O.sv) + i, dir);
  }
  for (int i = t; i < a; i += 256) arc_move((double*)(r + L.olam) + i, (double*)(q + O.lam) + i, dir);
  zd* rBl = (zd*)(r + L.oBl);
  zd* rBr = (zd*)(r + L.oBr);
  zd* rC = (zd*)(r + L.oC);
  zd* rA = (zd*)(r + L.oA);
  zd* rV = (zd*)(r + L.oV);
  zd* qBl = (zd*)(q + O.Bl);
  zd* qBr = (zd*)(q + O.Br);
  zd* qC = (zd*)(q + O.C);
  zd* qA = (zd*)(q + O.A);
  zd* qV = (zd*)(q + O.V);
  for (int e = t; e < a * 2 * m; e += 256) {
    const int rowi = e / m, be = e % m;          // rowi = 2 alpha + i
    arc_move(rBl + (size_t)rowi * dc + be, qBl + e, dir);
  }
  for (int e = t; e < m * 2 * b; e += 256) {
    const int rowj = e / b, be = e % b;          // rowj = 2 gamma + j
    arc_move(rBr + (size_t)rowj * dc + be, qBr + e, dir);
  }
  const int M = 2 * a;
  for (int e = t; e < nb * M; e += 256) {
    const int c = e / M, row = e % M;
    arc_move(rC + (size_t)c * ldc + row, qC + e, dir);
    const int pc = P[c];
    if (pc >= 0 && pc < ncap) arc_move(rA + (size_t)pc * ldc + row, qA + e, dir);
  }
  for (int e = t; e < nb * nb; e += 256) {
    const int i = e / nb, c = e % nb;
    const int pi = P[i];
    if (pi >= 0 && pi < ncap) arc_move(rV + (size_t)pi * ldv + c, qV + e, dir);
  }
}

static BatchSet& batch_of(mps_plan* p) {
  PlanAdj& A = adj_of(p);
  if (!A.batch) A.batch = new BatchSet();
  return *A.batch;
}

// One group of nl <= lanes_max lanes; thetas_dev holds nl consecutive vectors.
// Lane l evaluates the energy of plan lp[l]: p itself for a batch of
// parameter vectors, or plans that share p's circuit, truncation and options
// but hold their own Hamiltonian and initial occupation (plans_compatible).
// The lanes' buffers and the gate chain's constants come from p.
static void batched_group(mps_plan* p, mps_plan* const* lp, int nl, const double* thetas_dev, double* energies,
                          double* grads_dev, GateStats* gsum, double* prof_ms, int* prof_n) {
  mps_ctx* ctx = p->ctx;
  hipStream_t s = ctx->stream;
  BatchSet& B = batch_of(p);
  const int N = p->N, G = p->C.G, K = p->opts.ckpt_gates, nth = std::max(1, p->n_theta);
  const int dc = p->state->dcap;
  ctx->ensure_gate_work(dc, p->trunc, p->opts.max_sweeps);
  const GateWork gw = ctx->gw;
  const TapeLayout L = tape_layout(dc, gw.ncap, gw.ldc, gw.ldv);
  const int n_seg = (G + K - 1) / K;
  const size_t site = (size_t)dc * 2 * dc;
  while ((int)B.lanes.size() < nl) {
    BatchLane* bl = new BatchLane();
    B.lanes.push_back(bl);
    bl->st = plan_new_state(ctx, N, p->trunc, nullptr);
    bl->rp = plan_new_state(ctx, N, p->trunc, nullptr);
  }
  // checkpoint layout: B | dims | lambda at the next 8-byte boundary
  const size_t ck_B = p->state->B.bytes, ck_dims = p->state->dims.bytes, ck_lam = p->state->lam.bytes;
  const size_t ck_lamoff = ((ck_B + ck_dims + 7) / 8) * 8;
  const size_t ckpt_stride = ((ck_lamoff + ck_lam + 255) / 256) * 256;
  const size_t aux_lane = 128 * sizeof(int) + 256 * sizeof(double) + sizeof(GateStats) + 64;
  char* aux = (char*)B.aux.ensure((size_t)nl * aux_lane + 64 + (size_t)nl * 8);
  int* lane_err = (int*)(aux + (size_t)nl * aux_lane);
  unsigned long long* lane_bars = (unsigned long long*)(aux + (size_t)nl * aux_lane + 64);
  HIPCHK(hipMemsetAsync(aux, 0, (size_t)nl * aux_lane + 64 + (size_t)nl * 8, s));
  // One tape slot holds a segment of every lane in the layout that the chain
  // kernel writes and the gate adjoint reads; the forward pass records the
  // last segment there, and the reverse pass recomputes the others into it.
  // With a tape budget every forward segment records its tape, and while the
  // rest of the budget lasts a compact copy of each record (the entries the
  // adjoint reads, at the gate's own sizes) goes to the archive; the reverse
  // pass expands an archived segment back into the slot instead of
  // recomputing it.
  const size_t seg_bytes = (size_t)nl * K * L.rec;
  char* tape = (char*)B.tape.ensure(seg_bytes);
  size_t arc_cap = 0;
  if (p->opts.tape_budget_mib != 0 && n_seg > 1) {
    size_t budget = 0;
    if (p->opts.tape_budget_mib > 0) {
      budget = (size_t)p->opts.tape_budget_mib << 20;
    } else {
      size_t free_b = 0, total_b = 0;
      HIPCHK(hipMemGetInfo(&free_b, &total_b));
      const size_t avail = free_b + B.tape.bytes + B.arc.bytes, reserve = (size_t)16 << 30;
      budget = avail > reserve ? avail - reserve : 0;
    }
    // never more than the earlier segments could need with every bond at capacity
    const size_t most = (size_t)(n_seg - 1) * nl * K * arc_layout(dc, dc, dc).total;
    arc_cap = std::min(most, budget > B.tape.bytes ? budget - B.tape.bytes : 0);
  }
  char* arc = arc_cap > 0 ? (char*)B.arc.ensure(arc_cap) : nullptr;
  long long* arc_off = arc ? (long long*)B.arc_off.ensure((size_t)n_seg * nl * K * sizeof(long long)) : nullptr;
  std::vector<char> archived(n_seg, 0);
  std::vector<long long> off_h(arc ? (size_t)nl * K : 0);
  size_t arc_used = 0;
  bool arc_open = arc != nullptr;
  auto tape_of = [&](int, int l) { return tape + (size_t)l * K * L.rec; };
  GateLane* lanes_d = (GateLane*)B.lanes_dev.ensure((size_t)nl * sizeof(GateLane));
  std::vector<GateLane> lh(nl);
  std::vector<AdjWork> W(nl);
  for (int l = 0; l < nl; ++l) {
    BatchLane* bl = B.lanes[l];
    bl->ckpt.ensure((size_t)n_seg * ckpt_stride);
    bl->Bbar.ensure((size_t)N * site * sizeof(zd));
    bl->lambar.ensure((size_t)(N + 1) * dc * sizeof(double));
    bl->gphi.ensure((size_t)std::max(1, G) * sizeof(double));
    adjwork_layout(gw.ncap, dc, &W[l], (char*)bl->work.ensure(adjwork_layout(gw.ncap, dc, nullptr, nullptr)));
    HIPCHK(hipMemsetAsync(bl->lambar.p, 0, bl->lambar.bytes, s));
    HIPCHK(hipMemsetAsync(bl->gphi.p, 0, bl->gphi.bytes, s));
    char* la = aux + (size_t)l * aux_lane;
    GateLane& ln = lh[l];
    ln.rotflag = (int*)la;
    ln.nrm_part = (double*)(la + 128 * sizeof(int));
    ln.stats = (GateStats*)(la + 128 * sizeof(int) + 256 * sizeof(double));
    ln.bar = lane_bars + l;
    ln.err = lane_err;
    ln.theta = thetas_dev + (size_t)l * nth;
    ln.shift_gate = -1;
    ln.shift = 0.0;
  }
  LaneConst lc;
  lc.gt = p->C.tab;
  lc.L = L;
  lc.ldc = gw.ldc;
  lc.ldv = gw.ldv;
  lc.ncap = gw.ncap;
  lc.dmax = gw.dmax;
  lc.max_sweeps = gw.max_sweeps;
  lc.nparts = ((2 * dc + ZT_M - 1) / ZT_M) * ((2 * dc + ZT_M - 1) / ZT_M);
  lc.eps = gw.eps;
  lc.tol = gw.tol;
  lc.sched = gw.sched;
  lc.ck_B = ck_B;
  lc.ck_dims = ck_dims;
  lc.ck_lam = ck_lam;
  // ---- forward: all lanes through the circuit, one chain launch per
  // checkpoint segment (the launch copies each lane's state to its checkpoint
  // slot before the segment's first gate)
  for (int l = 0; l < nl; ++l) init_product(B.lanes[l]->st, (const uint8_t*)lp[l]->state->occ.p);
  // with profiling on, each chain launch is bracketed by events on the stream
  const bool prof = ctx->prof_every > 0;
  std::vector<hipEvent_t> ev;
  if (prof) {
    ev.resize(2);
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  }
  std::vector<int> fmeta(arc ? (size_t)nl * K * 16 : 0);
  std::vector<double> fdmeta(arc ? (size_t)nl * K * 16 : 0);
  for (int sg = 0; sg < n_seg; ++sg) {
    // the last segment records its tape in the slot, so the reverse pass does
    // not recompute it (earlier segments use the slot's first record as their
    // workspace), unless the archive is in use: then every segment records
    const bool keep = sg == n_seg - 1 || arc_open;
    for (int l = 0; l < nl; ++l) {
      GateLane& ln = lh[l];
      ln.st = view_of(B.lanes[l]->st);
      ln.g0 = sg * K;
      ln.ng = std::min(G, (sg + 1) * K) - sg * K;
      ln.rec_stride = keep ? 1 : 0;
      ln.tape = tape_of(sg, l);
      ln.ckpt = (char*)B.lanes[l]->ckpt.p + (size_t)sg * ckpt_stride;
    }
    HIPCHK(hipMemcpyAsync(lanes_d, lh.data(), (size_t)nl * sizeof(GateLane), hipMemcpyHostToDevice, s));
    if (prof) HIPCHK(hipEventRecord(ev[0], s));
    HIPCHK(launch_chain_lanes(lanes_d, nl, lc, keep, lane_bars, s));
    if (prof) HIPCHK(hipEventRecord(ev[1], s));
    // the lane table is rewritten for the next segment only after this one
    // has been consumed
    HIPCHK(hipStreamSynchronize(s));
    if (prof) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
      *prof_ms += t;
      *prof_n += 1;
    }
    if (arc_open && sg < n_seg - 1) {
      // archive the segment if all its records fit what is left (the sizes
      // are read back and checked first); once one does not, later segments
      // are recomputed
      read_lane_meta(lanes_d, lh, nl, L, K, dc, B.meta_dev, fmeta, fdmeta, s);
      size_t o = arc_used;
      for (int l = 0; l < nl; ++l)
        for (int k = 0; k < K; ++k) {
          long long& x = off_h[(size_t)l * K + k];
          if (k >= lh[l].ng) {
            x = -1;
            continue;
          }
          const int* mt = fmeta.data() + ((size_t)l * K + k) * 16;
          x = (long long)o;
          o += arc_layout(mt[4], mt[5], mt[6]).total;
        }
      if (o > arc_cap) {
        arc_open = false;
      } else {
        long long* od = arc_off + (size_t)sg * nl * K;
        HIPCHK(hipMemcpyAsync(od, off_h.data(), off_h.size() * sizeof(long long), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_tape_archive, dim3(K, nl), dim3(256), 0, s, (const GateLane*)lanes_d, L, K, dc, gw.ldc,
                           gw.ldv, gw.ncap, arc, (const long long*)od, 0);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));   // off_h and the lane table are reused
        archived[sg] = 1;
        arc_used = o;
      }
    }
    if (ctx->progress) ctx->progress(ctx->progress_user, "forward", sg + 1, n_seg);
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  // ---- statistics of the forward pass (the recompute adds to zeroed counters)
  std::vector<GateStats> st(nl);
  for (int l = 0; l < nl; ++l)
    HIPCHK(hipMemcpyAsync(&st[l], lh[l].stats, sizeof(GateStats), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int l = 0; l < nl; ++l) HIPCHK(hipMemsetAsync(lh[l].stats, 0, sizeof(GateStats), s));
  // ---- energies and sweep adjoints, lane by lane
  std::vector<int> dims(N + 1);
  for (int l = 0; l < nl; ++l) {
    BatchLane* bl = B.lanes[l];
    run_energy(bl->st, lp[l]->H);
    double ev[3];
    HIPCHK(hipMemcpyAsync(ev, ctx->sb.energy, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(dims.data(), bl->st->dims.p, (N + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    bl->E = ev[0];
    bl->Eim = ev[1];
    bl->Z = ev[2];
    energies[l] = ev[0];
    run_sweep_adjoint(lp[l], dims, bl->st, (zd*)bl->Bbar.p, bl->E, bl->Z);
  }
  // ---- reverse pass, one segment of all lanes at a time
  std::vector<int> meta((size_t)nl * K * 16);
  std::vector<double> dmeta((size_t)nl * K * 16);
  std::vector<AdjLane> rec;
  std::vector<GateDims> mx;
  for (int sg = n_seg - 1; sg >= 0; --sg) {
    const int g0 = sg * K, ng = std::min(G, (sg + 1) * K) - g0;
    const bool expand = archived[sg] != 0;                 // compact copy in the archive
    const bool taped = sg == n_seg - 1 || expand;          // no recompute needed
    for (int l = 0; l < nl; ++l) {
      BatchLane* bl = B.lanes[l];
      mps_state* rp = bl->rp;
      if (!taped) {
        const char* base = (const char*)bl->ckpt.p + (size_t)sg * ckpt_stride;
        HIPCHK(hipMemcpyAsync(rp->B.p, base, ck_B, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(rp->dims.p, base + ck_B, ck_dims, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(rp->lam.p, base + ck_lamoff, ck_lam, hipMemcpyDeviceToDevice, s));
      }
      GateLane& ln = lh[l];
      ln.st = view_of(rp);
      ln.g0 = g0;
      ln.ng = ng;
      ln.rec_stride = 1;
      ln.tape = tape_of(sg, l);
      ln.ckpt = nullptr;
    }
    HIPCHK(hipMemcpyAsync(lanes_d, lh.data(), (size_t)nl * sizeof(GateLane), hipMemcpyHostToDevice, s));
    if (!taped) HIPCHK(launch_chain_lanes(lanes_d, nl, lc, true, lane_bars, s));
    if (expand) {
      hipLaunchKernelGGL(k_tape_archive, dim3(K, nl), dim3(256), 0, s, (const GateLane*)lanes_d, L, K, dc, gw.ldc,
                         gw.ldv, gw.ncap, arc, (const long long*)(arc_off + (size_t)sg * nl * K), 1);
      HIPCHK(hipGetLastError());
    }
    read_lane_meta(lanes_d, lh, nl, L, K, dc, B.meta_dev, meta, dmeta, s);
    int err = 0;
    HIPCHK(hipMemcpyAsync(&err, lane_err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (err) fail(MPS_EDEVICE, "a lane barrier of the batched gate chain timed out");
    rec.clear();
    mx.clear();
    for (int g = g0 + ng - 1; g >= g0; --g) {
      GateDims m{p->C.bond_h[g], 0, 0, 0, 0, 0.0};
      for (int l = 0; l < nl; ++l) {
        BatchLane* bl = B.lanes[l];
        const size_t k = (size_t)l * K + (g - g0);
        AdjLane a1;
        a1.R = rec_at(lh[l].tape, L, g - g0);
        a1.W = W[l];
        a1.d = dims_of(meta.data() + k * 16, dmeta.data() + k * 16, p->C.bond_h[g]);
        const int n = a1.d.n;
        zd* Bbar = (zd*)bl->Bbar.p;
        double* lambar = (double*)bl->lambar.p;
        a1.Bbn = Bbar + (size_t)n * site;
        a1.Bbn1 = Bbar + (size_t)(n + 1) * site;
        a1.lb_out = lambar + (size_t)(n + 1) * dc;
        a1.lb_in = lambar + (size_t)n * dc;
        a1.gphi = (double*)bl->gphi.p;
        a1.theta = lh[l].theta;
        a1.gt = p->C.tab;
        a1.g = g;
        a1.kind = p->C.kind_h[g];
        a1.dc = dc;
        a1.ldc = gw.ldc;
        a1.ldv = gw.ldv;
        a1.eta = p->opts.broaden;
        rec.push_back(a1);
        m.a = std::max(m.a, a1.d.a);
        m.m = std::max(m.m, a1.d.m);
        m.b = std::max(m.b, a1.d.b);
        m.r = std::max(m.r, a1.d.r);
      }
      mx.push_back(m);
    }
    AdjLane* rec_d = (AdjLane*)B.adj_dev.ensure(rec.size() * sizeof(AdjLane));
    HIPCHK(hipMemcpyAsync(rec_d, rec.data(), rec.size() * sizeof(AdjLane), hipMemcpyHostToDevice, s));
    size_t k = 0;
    for (int g = g0 + ng - 1; g >= g0; --g, ++k)
      launch_gate_adjoint(rec_d + k * nl, nl, mx[k], gw.stats, s);
    HIPCHK(hipGetLastError());
    if (ctx->progress) {
      HIPCHK(hipStreamSynchronize(s));
      ctx->progress(ctx->progress_user, "backward", n_seg - sg, n_seg);
    }
  }
  // ---- chain rule per lane
  PlanAdj& A = adj_of(p);
  if (!A.chain_built) build_chain(p, A);
  for (int l = 0; l < nl && p->n_theta > 0; ++l)
    hipLaunchKernelGGL(k_chain_rule, dim3((p->n_theta + 255) / 256), dim3(256), 0, s,
                       (const int*)A.chain_start.p, (const int*)A.chain_list.p, p->C.tab,
                       (const double*)B.lanes[l]->gphi.p, grads_dev + (size_t)l * nth, p->n_theta);
  HIPCHK(hipGetLastError());
  for (const GateStats& x : st) {
    gsum->disc_sum += x.disc_sum;
    gsum->disc_max = std::max(gsum->disc_max, x.disc_max);
    gsum->svd_flop += x.svd_flop;
    gsum->gemm_flop += x.gemm_flop;
    gsum->truncated += x.truncated;
    gsum->max_sweeps = std::max(gsum->max_sweeps, x.max_sweeps);
    gsum->noconv += x.noconv;
    gsum->degenerate_cuts += x.degenerate_cuts;
    gsum->max_bond = std::max(gsum->max_bond, x.max_bond);
    gsum->gates += x.gates;
  }
}

// nb evaluations in groups of lanes_max lanes: evaluation b is plan lp[b] at
// the vector th + b * nth (device); energies to the host, gradients to gdev.
static void batched_run(mps_plan* p, mps_plan* const* lp, int nb, const double* th, double* energies,
                        double* gdev, mps_stats* stats) {
  hipStream_t s = p->ctx->stream;
  const int nth = std::max(1, p->n_theta);
  const int per = lanes_max(p->state->dcap);
  GateStats gsum{};
  double prof_ms = 0.0;
  int prof_n = 0;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  for (int b0 = 0; b0 < nb; b0 += per) {
    const int nl = std::min(per, nb - b0);
    batched_group(p, lp + b0, nl, th + (size_t)b0 * nth, energies + b0, gdev + (size_t)b0 * nth, &gsum, &prof_ms,
                  &prof_n);
  }
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (gsum.noconv) fail(MPS_ENOCONV, "Jacobi SVD did not converge in " + std::to_string(p->opts.max_sweeps) + " sweeps");
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->discarded_weight_sum = gsum.disc_sum;
    stats->discarded_weight_max = gsum.disc_max;
    stats->max_bond = gsum.max_bond;
    stats->gates_truncated = gsum.truncated;
    stats->max_sweeps_used = gsum.max_sweeps;
    stats->degenerate_cuts = gsum.degenerate_cuts;
    stats->n_gates_applied = gsum.gates;
    stats->t_backward_ms = ms;
    if (prof_n > 0) {
      stats->prof_svd_ms = prof_ms;
      stats->prof_svd_flop = gsum.svd_flop;
      stats->prof_gemm_flop = gsum.gemm_flop;
      stats->prof_svd_launches = prof_n;
    }
  }
}

void plan_energy_grad_batched(mps_plan* p, int nb, const double* thetas, int n_theta, int on_device,
                              double* energies, double* grads, mps_stats* stats) {
  mps_ctx* ctx = p->ctx;
  hipStream_t s = ctx->stream;
  if (nb < 1) fail(MPS_EINVAL, "n_batch must be >= 1");
  if (n_theta != p->n_theta) fail(MPS_EINVAL, "n_theta does not match the circuit");
  BatchSet& B = batch_of(p);
  const int nth = std::max(1, n_theta);
  double* th = (double*)B.thetas.ensure((size_t)nb * nth * sizeof(double));
  if (n_theta > 0) {
    std::vector<double> host((size_t)nb * n_theta);
    if (on_device) {
      HIPCHK(hipMemcpyAsync(host.data(), thetas, host.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    } else {
      std::memcpy(host.data(), thetas, host.size() * sizeof(double));
    }
    validate_theta(host.data(), (int)host.size());
    HIPCHK(hipMemcpyAsync(th, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));   // host is released at the end of this block
  }
  double* gdev = (double*)p->grad.ensure((size_t)nb * nth * sizeof(double));
  const std::vector<mps_plan*> same(nb, p);
  batched_run(p, same.data(), nb, th, energies, gdev, stats);
  if (n_theta > 0)   // nth == n_theta here: rows are contiguous
    HIPCHK(hipMemcpyAsync(grads, gdev, (size_t)nb * n_theta * sizeof(double),
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
}

// Plans whose evaluations can share gate-chain launches: one context, the
// same circuit (gate tables equal by hash and size), qubit count, truncation,
// capacity and reverse-pass options.  The Hamiltonian and the initial
// occupation may differ.
static void plans_compatible(mps_plan* const* plans, int n) {
  const mps_plan* a = plans[0];
  for (int i = 1; i < n; ++i) {
    const mps_plan* b = plans[i];
    if (!b) fail(MPS_EINVAL, "NULL plan");
    if (b->ctx != a->ctx) fail(MPS_EINVAL, "plans belong to different contexts");
    if (b->N != a->N || b->n_theta != a->n_theta) fail(MPS_EINVAL, "plans differ in qubit or parameter count");
    if (b->C.G != a->C.G || b->C.hash != a->C.hash) fail(MPS_EINVAL, "plans hold different circuits");
    if (b->trunc.d_max != a->trunc.d_max || b->trunc.eps != a->trunc.eps ||
        b->trunc.precision != a->trunc.precision || b->state->dcap != a->state->dcap)
      fail(MPS_EINVAL, "plans differ in truncation (d_max, eps or precision)");
    if (b->opts.ckpt_gates != a->opts.ckpt_gates || b->opts.max_sweeps != a->opts.max_sweeps ||
        b->opts.broaden != a->opts.broaden)
      fail(MPS_EINVAL, "plans differ in gradient options");
  }
}

void plan_energy_grad_multi(mps_plan* const* plans, int n, const double* thetas, int n_theta, double* energies,
                            double* grads, mps_stats* stats) {
  if (n < 1) fail(MPS_EINVAL, "n_plans must be >= 1");
  mps_plan* p = plans[0];
  if (!p) fail(MPS_EINVAL, "NULL plan");
  plans_compatible(plans, n);
  if (n_theta != p->n_theta) fail(MPS_EINVAL, "n_theta does not match the circuit");
  hipStream_t s = p->ctx->stream;
  BatchSet& B = batch_of(p);
  const int nth = std::max(1, n_theta);
  double* th = (double*)B.thetas.ensure((size_t)n * nth * sizeof(double));
  if (n_theta > 0) {
    validate_theta(thetas, n * n_theta);
    HIPCHK(hipMemcpyAsync(th, thetas, (size_t)n * n_theta * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  double* gdev = (double*)p->grad.ensure((size_t)n * nth * sizeof(double));
  batched_run(p, plans, n, th, energies, gdev, stats);
  if (n_theta > 0)
    HIPCHK(hipMemcpyAsync(grads, gdev, (size_t)n * n_theta * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
}

// ============================================================================
// Parameter-shift gradient (Sec. 4, Eq. psr).  RZZ(phi) = exp(-i phi ZZ/2) has
// generator eigenvalues +-1/2, so for every PARAM gate g
//   dE/dphi_g = (E(phi_g + pi/2) - E(phi_g - pi/2)) / 2,
// and dE/dtheta_p = sum over the gates of p of coeff_g dE/dphi_g.  The 2M + 1
// evaluations (the unshifted one first, then +pi/2 and -pi/2 for each PARAM
// gate in circuit order) are lanes of the gate-chain kernel, as many per
// launch as fit; each lane's energy is then swept on its own.
// ============================================================================
void plan_energy_grad_psr(mps_plan* p, const double* theta, int n_theta, double* energy, double* grad,
                          double* gate_grad, mps_stats* stats) {
  mps_ctx* ctx = p->ctx;
  hipStream_t s = ctx->stream;
  if (n_theta != p->n_theta) fail(MPS_EINVAL, "n_theta does not match the circuit");
  if (n_theta > 0 && !theta) fail(MPS_EINVAL, "NULL theta");
  validate_theta(theta, n_theta);
  const int N = p->N, G = p->C.G, K = p->opts.ckpt_gates;
  const int dc = p->state->dcap;
  ctx->ensure_gate_work(dc, p->trunc, p->opts.max_sweeps);
  const GateWork gw = ctx->gw;
  const TapeLayout L = tape_layout(dc, gw.ncap, gw.ldc, gw.ldv);
  std::vector<int> pg;
  for (int g = 0; g < G; ++g)
    if (p->C.kind_h[g] == 1) pg.push_back(g);
  const int M = (int)pg.size(), nev = 2 * M + 1;
  BatchSet& B = batch_of(p);
  double* th = (double*)B.thetas.ensure((size_t)std::max(1, n_theta) * sizeof(double));
  if (n_theta > 0) HIPCHK(hipMemcpyAsync(th, theta, (size_t)n_theta * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  const int nmax = std::min(lanes_max(dc), nev);
  while ((int)B.lanes.size() < nmax) {
    BatchLane* bl = new BatchLane();
    B.lanes.push_back(bl);
    bl->st = plan_new_state(ctx, N, p->trunc, nullptr);
    bl->rp = plan_new_state(ctx, N, p->trunc, nullptr);
  }
  const size_t aux_lane = 128 * sizeof(int) + 256 * sizeof(double) + sizeof(GateStats) + 64;
  const size_t aux_bytes = (size_t)nmax * aux_lane + 64 + (size_t)nmax * 8;
  char* aux = (char*)B.aux.ensure(aux_bytes);
  int* lane_err = (int*)(aux + (size_t)nmax * aux_lane);
  unsigned long long* lane_bars = (unsigned long long*)(aux + (size_t)nmax * aux_lane + 64);
  char* tape = (char*)B.tape.ensure((size_t)nmax * L.rec);   // one record per lane, reused by every step
  GateLane* lanes_d = (GateLane*)B.lanes_dev.ensure((size_t)nmax * sizeof(GateLane));
  LaneConst lc;
  lc.gt = p->C.tab;
  lc.L = L;
  lc.ldc = gw.ldc;
  lc.ldv = gw.ldv;
  lc.ncap = gw.ncap;
  lc.dmax = gw.dmax;
  lc.max_sweeps = gw.max_sweeps;
  lc.nparts = ((2 * dc + ZT_M - 1) / ZT_M) * ((2 * dc + ZT_M - 1) / ZT_M);
  lc.eps = gw.eps;
  lc.tol = gw.tol;
  lc.sched = gw.sched;
  lc.ck_B = lc.ck_dims = lc.ck_lam = 0;
  std::vector<double> E(nev);
  std::vector<GateLane> lh(nmax);
  std::vector<GateStats> st(nmax);
  GateStats gsum{};
  hipEvent_t t0, t1;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  HIPCHK(hipEventRecord(t0, s));
  for (int e0 = 0; e0 < nev; e0 += nmax) {
    const int nl = std::min(nmax, nev - e0);
    HIPCHK(hipMemsetAsync(aux, 0, aux_bytes, s));
    for (int l = 0; l < nl; ++l) {
      const int ev = e0 + l;
      BatchLane* bl = B.lanes[l];
      init_product(bl->st, (const uint8_t*)p->state->occ.p);
      GateLane ln{};
      ln.st = view_of(bl->st);
      ln.rec_stride = 0;
      ln.theta = th;
      ln.ckpt = nullptr;
      ln.tape = tape + (size_t)l * L.rec;
      char* la = aux + (size_t)l * aux_lane;
      ln.rotflag = (int*)la;
      ln.nrm_part = (double*)(la + 128 * sizeof(int));
      ln.stats = (GateStats*)(la + 128 * sizeof(int) + 256 * sizeof(double));
      ln.bar = lane_bars + l;
      ln.err = lane_err;
      ln.shift_gate = ev == 0 ? -1 : pg[(ev - 1) / 2];
      ln.shift = ev == 0 ? 0.0 : ((ev - 1) % 2 == 0 ? 0.5 * M_PI : -0.5 * M_PI);
      lh[l] = ln;
    }
    for (int g0 = 0; g0 < G; g0 += K) {
      for (int l = 0; l < nl; ++l) {
        lh[l].g0 = g0;
        lh[l].ng = std::min(G, g0 + K) - g0;
      }
      HIPCHK(hipMemcpyAsync(lanes_d, lh.data(), (size_t)nl * sizeof(GateLane), hipMemcpyHostToDevice, s));
      HIPCHK(launch_chain_lanes(lanes_d, nl, lc, false, lane_bars, s));
      HIPCHK(hipStreamSynchronize(s));   // lh is rewritten for the next segment
    }
    int err = 0;
    HIPCHK(hipMemcpyAsync(&err, lane_err, sizeof(int), hipMemcpyDeviceToHost, s));
    for (int l = 0; l < nl; ++l)
      HIPCHK(hipMemcpyAsync(&st[l], lh[l].stats, sizeof(GateStats), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (err) fail(MPS_EDEVICE, "a lane barrier of the parameter-shift evaluations timed out");
    for (int l = 0; l < nl; ++l) {
      const GateStats& x = st[l];
      gsum.disc_sum += x.disc_sum;
      gsum.disc_max = std::max(gsum.disc_max, x.disc_max);
      gsum.truncated += x.truncated;
      gsum.max_sweeps = std::max(gsum.max_sweeps, x.max_sweeps);
      gsum.noconv += x.noconv;
      gsum.degenerate_cuts += x.degenerate_cuts;
      gsum.max_bond = std::max(gsum.max_bond, x.max_bond);
      gsum.gates += x.gates;
      run_energy(B.lanes[l]->st, p->H);
      double ev[3];
      HIPCHK(hipMemcpyAsync(ev, ctx->sb.energy, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      E[e0 + l] = ev[0];
    }
    if (ctx->progress) ctx->progress(ctx->progress_user, "parameter shift", std::min(nev, e0 + nl), nev);
  }
  HIPCHK(hipEventRecord(t1, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, t0, t1));
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (gsum.noconv) fail(MPS_ENOCONV, "Jacobi SVD did not converge in " + std::to_string(p->opts.max_sweeps) + " sweeps");
  std::vector<double> gg(std::max(1, G), 0.0);
  for (int i = 0; i < M; ++i) gg[pg[i]] = 0.5 * (E[1 + 2 * i] - E[2 + 2 * i]);
  for (int q = 0; q < n_theta; ++q) grad[q] = 0.0;
  for (int i = 0; i < M; ++i) grad[p->C.param_h[pg[i]]] += p->C.coeff_h[pg[i]] * gg[pg[i]];
  if (gate_grad)
    for (int g = 0; g < G; ++g) gate_grad[g] = gg[g];
  *energy = E[0];
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->discarded_weight_sum = gsum.disc_sum;
    stats->discarded_weight_max = gsum.disc_max;
    stats->max_bond = gsum.max_bond;
    stats->gates_truncated = gsum.truncated;
    stats->max_sweeps_used = gsum.max_sweeps;
    stats->degenerate_cuts = gsum.degenerate_cuts;
    stats->n_gates_applied = gsum.gates;
    stats->t_gates_ms = ms;
  }
}

// ============================================================================
// Mixed instances: plans with their own circuits, qubit counts, bond
// capacities, Hamiltonians, truncations and checkpoint intervals as lanes of
// the same cooperative launches (k_chain_mixed).  Lanes of one launch take
// their work-groups from the same XCD where the counts allow; each launch
// advances every lane by one of its own checkpoint segments, so lanes with
// shorter circuits finish early and idle.  Energies and sweep adjoints then
// run per lane with its own plan, and the reverse pass walks the segment
// index down: lanes recompute their segment (all in one launch), then the
// gate adjoints of all lanes run step by step in shared launch sets, each
// lane record carrying its own gate, capacity and leading dimensions.
// ============================================================================
struct MixLaneBufs {
  mps_state* st = nullptr;
  mps_state* rp = nullptr;
  std::vector<mps_state*> wrp;   // replay states of a reverse window's segments
  DevBuf ckpt, Bbar, lambar, gphi, grad, work, tape, wtape;   // wtape: the window's tapes, one per segment
  ~MixLaneBufs() {
    delete st;
    delete rp;
    for (mps_state* x : wrp) delete x;
  }
};

struct MixSet {
  std::vector<MixLaneBufs*> lanes;
  DevBuf thetas, aux, lanes_dev, blk_dev, adj_dev, raux, rlanes_dev, rblk_dev;
  ~MixSet() {
    for (MixLaneBufs* l : lanes) delete l;
  }
};

// Per-lane constants of a mixed launch.
struct MixInfo {
  mps_plan* p;
  int dc, W, P, ncap, ldc, ldv, K, G, n_seg;
  TapeLayout L;
  size_t ck_B, ck_dims, ck_lam, ck_lamoff, ck_stride;
  double tol;
};

static MixInfo mix_info(mps_plan* p) {
  MixInfo m;
  m.p = p;
  m.dc = p->state->dcap;
  m.W = svd_width(m.dc);
  m.P = (2 * m.dc + 2 * m.W - 1) / (2 * m.W);
  m.ncap = 2 * m.P * m.W;
  m.ldc = 2 * m.dc;
  m.ldv = m.ncap;
  m.K = std::max(1, p->opts.ckpt_gates);
  m.G = p->C.G;
  m.n_seg = std::max(1, (m.G + m.K - 1) / m.K);
  m.L = tape_layout(m.dc, m.ncap, m.ldc, m.ldv);
  m.ck_B = p->state->B.bytes;
  m.ck_dims = p->state->dims.bytes;
  m.ck_lam = p->state->lam.bytes;
  m.ck_lamoff = ((m.ck_B + m.ck_dims + 7) / 8) * 8;
  m.ck_stride = ((m.ck_lamoff + m.ck_lam + 255) / 256) * 256;
  m.tol = std::max(1e-15, 8.0 * std::sqrt((double)m.ldc) * 2.220446049250313e-16);
  return m;
}

// Work-group table of a mixed launch: lanes go to the XCD with the fewest
// work-groups so far (work-group i runs on XCD i % 8), and the work-groups of
// XCD x are blocks x, x + 8, x + 16, ...  Returns the block count.
static int mix_block_table(const std::vector<MixInfo>& info, const std::vector<int>& lanes, std::vector<int2>& blk) {
  const int X = 8;
  std::vector<std::vector<int2>> per(X);
  for (int l : lanes) {
    int x = 0;
    for (int y = 1; y < X; ++y)
      if (per[y].size() < per[x].size()) x = y;
    for (int q = 0; q < info[l].P; ++q) per[x].push_back(make_int2(l, q));
  }
  size_t depth = 0;
  for (auto& v : per) depth = std::max(depth, v.size());
  blk.assign(depth * X, make_int2(-1, 0));
  for (int x = 0; x < X; ++x)
    for (size_t k = 0; k < per[x].size(); ++k) blk[k * X + x] = per[x][k];
  return (int)blk.size();
}

static void mixed_group(mps_plan* lead, const std::vector<MixInfo>& info, const std::vector<int>& grp,
                        const std::vector<const double*>& th_dev, double* energies, std::vector<double*>& grad_dev,
                        GateStats* gsum, int cap) {
  mps_ctx* ctx = lead->ctx;
  hipStream_t s = ctx->stream;
  PlanAdj& LA = adj_of(lead);
  if (!LA.mix) LA.mix = new MixSet();
  MixSet& S = *LA.mix;
  const int nl = (int)grp.size();
  while ((int)S.lanes.size() < nl) S.lanes.push_back(new MixLaneBufs());
  size_t shm = 0;
  int max_dc = 2;
  for (int l : grp) {
    shm = std::max(shm, chain_lds_bytes(info[l].dc));
    max_dc = std::max(max_dc, info[l].dc);
  }
  // the shared Jacobi block schedules and the context's statistics block
  ctx->ensure_gate_work(max_dc, lead->trunc, lead->opts.max_sweeps);
  const GateWork gw = ctx->gw;
  const size_t aux_lane = 128 * sizeof(int) + 256 * sizeof(double) + sizeof(GateStats) + 64;
  char* aux = (char*)S.aux.ensure((size_t)nl * aux_lane + 64 + (size_t)nl * 8);
  int* lane_err = (int*)(aux + (size_t)nl * aux_lane);
  unsigned long long* bars = (unsigned long long*)(aux + (size_t)nl * aux_lane + 64);
  HIPCHK(hipMemsetAsync(aux, 0, (size_t)nl * aux_lane + 64 + (size_t)nl * 8, s));
  std::vector<MixLane> lh(nl);
  std::vector<AdjWork> W(nl);
  int S_max = 0;
  for (int j = 0; j < nl; ++j) {
    const MixInfo& m = info[grp[j]];
    mps_plan* p = m.p;
    MixLaneBufs* b = S.lanes[j];
    const int N = p->N;
    if (!b->st || b->st->N != N || b->st->dcap != m.dc || b->st->trunc.eps != p->trunc.eps ||
        b->st->trunc.d_max != p->trunc.d_max || b->st->trunc.precision != p->trunc.precision) {
      delete b->st;
      delete b->rp;
      b->st = nullptr;
      b->rp = nullptr;
      b->st = plan_new_state(ctx, N, p->trunc, nullptr);
      b->rp = plan_new_state(ctx, N, p->trunc, nullptr);
    }
    const size_t site = (size_t)m.dc * 2 * m.dc;
    b->ckpt.ensure((size_t)m.n_seg * m.ck_stride);
    b->Bbar.ensure((size_t)N * site * sizeof(zd));
    b->lambar.ensure((size_t)(N + 1) * m.dc * sizeof(double));
    b->gphi.ensure((size_t)std::max(1, m.G) * sizeof(double));
    b->tape.ensure((size_t)m.K * m.L.rec);
    adjwork_layout(m.ncap, m.dc, &W[j], (char*)b->work.ensure(adjwork_layout(m.ncap, m.dc, nullptr, nullptr)));
    HIPCHK(hipMemsetAsync(b->lambar.p, 0, b->lambar.bytes, s));
    HIPCHK(hipMemsetAsync(b->gphi.p, 0, b->gphi.bytes, s));
    MixLane& ml = lh[j];
    std::memset(&ml, 0, sizeof(ml));
    char* la = aux + (size_t)j * aux_lane;
    ml.ln.rotflag = (int*)la;
    ml.ln.nrm_part = (double*)(la + 128 * sizeof(int));
    ml.ln.stats = (GateStats*)(la + 128 * sizeof(int) + 256 * sizeof(double));
    ml.ln.bar = bars + j;
    ml.ln.err = lane_err;
    ml.ln.theta = th_dev[grp[j]];
    ml.ln.shift_gate = -1;
    ml.ln.shift = 0.0;
    ml.ln.tape = (char*)b->tape.p;
    LaneConst& c = ml.c;
    c.sched = gw.sched;
    c.gt = p->C.tab;
    c.L = m.L;
    c.ldc = m.ldc;
    c.ldv = m.ldv;
    c.ncap = m.ncap;
    c.dmax = p->trunc.d_max;
    c.max_sweeps = std::min(std::max(p->opts.max_sweeps, 1), 100);
    c.nparts = ((2 * m.dc + ZT_M - 1) / ZT_M) * ((2 * m.dc + ZT_M - 1) / ZT_M);
    c.eps = p->trunc.eps;
    c.tol = m.tol;
    c.ck_B = m.ck_B;
    c.ck_dims = m.ck_dims;
    c.ck_lam = m.ck_lam;
    ml.W = m.W;
    ml.nblk = m.P;
    S_max = std::max(S_max, m.n_seg);
    init_product(b->st, (const uint8_t*)p->state->occ.p);
  }
  std::vector<int> all(nl);
  for (int j = 0; j < nl; ++j) all[j] = j;
  std::vector<MixInfo> linfo(nl);
  for (int j = 0; j < nl; ++j) linfo[j] = info[grp[j]];
  std::vector<int2> blk;
  const int T = mix_block_table(linfo, all, blk);
  const int2* blk_d = upload(S.blk_dev, blk.data(), blk.size(), s);
  MixLane* lanes_d = (MixLane*)S.lanes_dev.ensure((size_t)nl * sizeof(MixLane));
  auto launch = [&]() {
    HIPCHK(hipMemcpyAsync(lanes_d, lh.data(), (size_t)nl * sizeof(MixLane), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(bars, 0, (size_t)nl * sizeof(unsigned long long), s));
    HIPCHK(launch_chain_mixed(lanes_d, blk_d, T, shm, s));
    // the host lane table is rewritten only after this launch has read it
    HIPCHK(hipStreamSynchronize(s));
    int err = 0;
    HIPCHK(hipMemcpy(&err, lane_err, sizeof(int), hipMemcpyDeviceToHost));
    if (err) fail(MPS_EDEVICE, "a lane barrier of the mixed gate chain timed out");
  };
  // ---- forward: segment sg of every lane that has one; a lane's last
  // segment records its tape
  for (int sg = 0; sg < S_max; ++sg) {
    for (int j = 0; j < nl; ++j) {
      const MixInfo& m = linfo[j];
      MixLane& ml = lh[j];
      ml.ln.st = view_of(S.lanes[j]->st);
      if (sg < m.n_seg) {
        ml.ln.g0 = sg * m.K;
        ml.ln.ng = std::min(m.G, (sg + 1) * m.K) - sg * m.K;
        ml.record = sg == m.n_seg - 1;
        ml.ln.rec_stride = ml.record ? 1 : 0;
        ml.ln.ckpt = (char*)S.lanes[j]->ckpt.p + (size_t)sg * m.ck_stride;
      } else {
        ml.ln.g0 = 0;
        ml.ln.ng = 0;
        ml.record = 0;
        ml.ln.ckpt = nullptr;
      }
    }
    launch();
    if (ctx->progress) ctx->progress(ctx->progress_user, "forward", sg + 1, S_max);
  }
  // ---- statistics of the forward pass
  std::vector<GateStats> st(nl);
  for (int j = 0; j < nl; ++j)
    HIPCHK(hipMemcpyAsync(&st[j], lh[j].ln.stats, sizeof(GateStats), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int j = 0; j < nl; ++j) HIPCHK(hipMemsetAsync(lh[j].ln.stats, 0, sizeof(GateStats), s));
  // ---- energies and sweep adjoints, lane by lane with each lane's plan
  for (int j = 0; j < nl; ++j) {
    mps_plan* p = linfo[j].p;
    MixLaneBufs* b = S.lanes[j];
    std::vector<int> dims(p->N + 1);
    run_energy(b->st, p->H);
    double ev[3];
    HIPCHK(hipMemcpyAsync(ev, ctx->sb.energy, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(dims.data(), b->st->dims.p, (p->N + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    energies[grp[j]] = ev[0];
    run_sweep_adjoint(p, dims, b->st, (zd*)b->Bbar.p, ev[0], ev[2]);
  }
  // ---- reverse pass in windows of segment indices [bot, top], from the top
  // down.  In a window every instance recomputes all its segments but its
  // last (recorded by the forward pass) side by side, one lane per segment,
  // into the window's tapes; then the gate adjoints of all instances run down
  // the window, segment index by segment index.  The window is as deep as the
  // launch's resident work-groups and a tape budget allow.
  const size_t wtape_budget = (size_t)64 << 30;
  auto needs = [&](int j, int sg) { return sg < linfo[j].n_seg - 1; };   // recomputed, not recorded
  std::vector<AdjLane> rec;
  int top = S_max - 1;
  while (top >= 0) {
    // deepest window that fits
    int depth = 1;
    for (int d = 2; d <= top + 1; ++d) {
      std::vector<MixInfo> ri;
      std::vector<int> idx;
      size_t tape_bytes = 0;
      for (int j = 0; j < nl; ++j)
        for (int sg = top - d + 1; sg <= top; ++sg)
          if (needs(j, sg)) {
            idx.push_back((int)ri.size());
            ri.push_back(linfo[j]);
            tape_bytes += (size_t)linfo[j].K * linfo[j].L.rec;
          }
      std::vector<int2> tb;
      if ((!ri.empty() && mix_block_table(ri, idx, tb) > cap) || tape_bytes > wtape_budget) break;
      depth = d;
    }
    const int bot = top - depth + 1;
    // lanes of the window's recompute: (instance, segment)
    std::vector<std::pair<int, int>> rl;
    for (int j = 0; j < nl; ++j)
      for (int sg = bot; sg <= top; ++sg)
        if (needs(j, sg)) rl.push_back({j, sg});
    const int nr = (int)rl.size();
    if (nr > 0) {
      char* raux = (char*)S.raux.ensure((size_t)nr * aux_lane + 64 + (size_t)nr * 8);
      int* rerr = (int*)(raux + (size_t)nr * aux_lane);
      unsigned long long* rbars = (unsigned long long*)(raux + (size_t)nr * aux_lane + 64);
      HIPCHK(hipMemsetAsync(raux, 0, (size_t)nr * aux_lane + 64 + (size_t)nr * 8, s));
      std::vector<MixLane> rh(nr);
      std::vector<MixInfo> ri(nr);
      std::vector<int> idx(nr);
      for (int q = 0; q < nr; ++q) {
        const int j = rl[q].first, sg = rl[q].second, slot = sg - bot;
        const MixInfo& m = linfo[j];
        mps_plan* p = m.p;
        MixLaneBufs* b = S.lanes[j];
        while ((int)b->wrp.size() < depth) b->wrp.push_back(plan_new_state(ctx, p->N, p->trunc, nullptr));
        mps_state* rp = b->wrp[slot];
        if (rp->N != p->N || rp->dcap != m.dc) {
          delete rp;
          rp = b->wrp[slot] = plan_new_state(ctx, p->N, p->trunc, nullptr);
        }
        const char* base = (const char*)b->ckpt.p + (size_t)sg * m.ck_stride;
        HIPCHK(hipMemcpyAsync(rp->B.p, base, m.ck_B, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(rp->dims.p, base + m.ck_B, m.ck_dims, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(rp->lam.p, base + m.ck_lamoff, m.ck_lam, hipMemcpyDeviceToDevice, s));
        MixLane& ml = rh[q];
        ml = lh[j];   // the instance's constants, width and work-group count
        char* la = raux + (size_t)q * aux_lane;
        ml.ln.rotflag = (int*)la;
        ml.ln.nrm_part = (double*)(la + 128 * sizeof(int));
        ml.ln.stats = (GateStats*)(la + 128 * sizeof(int) + 256 * sizeof(double));
        ml.ln.bar = rbars + q;
        ml.ln.err = rerr;
        ml.ln.st = view_of(rp);
        ml.ln.g0 = sg * m.K;
        ml.ln.ng = std::min(m.G, (sg + 1) * m.K) - sg * m.K;
        ml.ln.rec_stride = 1;
        ml.ln.ckpt = nullptr;
        ml.record = 1;
        ri[q] = m;
        idx[q] = q;
      }
      // each instance's window tapes, as many as its highest slot needs
      std::vector<int> slots(nl, 0);
      for (const auto& r : rl) slots[r.first] = std::max(slots[r.first], r.second - bot + 1);
      for (int j = 0; j < nl; ++j)
        if (slots[j] > 0) S.lanes[j]->wtape.ensure((size_t)slots[j] * linfo[j].K * linfo[j].L.rec);
      for (int q = 0; q < nr; ++q) {
        const int j = rl[q].first, slot = rl[q].second - bot;
        rh[q].ln.tape = (char*)S.lanes[j]->wtape.p + (size_t)slot * linfo[j].K * linfo[j].L.rec;
      }
      std::vector<int2> rblk;
      const int RT = mix_block_table(ri, idx, rblk);
      const int2* rblk_d = upload(S.rblk_dev, rblk.data(), rblk.size(), s);
      MixLane* rlanes_d = (MixLane*)S.rlanes_dev.ensure((size_t)nr * sizeof(MixLane));
      HIPCHK(hipMemcpyAsync(rlanes_d, rh.data(), (size_t)nr * sizeof(MixLane), hipMemcpyHostToDevice, s));
      HIPCHK(launch_chain_mixed(rlanes_d, rblk_d, RT, shm, s));
      HIPCHK(hipStreamSynchronize(s));   // rh and rblk are released at the end of this block
      int err = 0;
      HIPCHK(hipMemcpy(&err, rerr, sizeof(int), hipMemcpyDeviceToHost));
      if (err) fail(MPS_EDEVICE, "a lane barrier of the mixed gate chain timed out");
    }
    // the tape of instance j's segment sg in this window
    auto tape_of = [&](int j, int sg) -> char* {
      const MixInfo& m = linfo[j];
      if (sg == m.n_seg - 1) return (char*)S.lanes[j]->tape.p;
      return (char*)S.lanes[j]->wtape.p + (size_t)(sg - bot) * m.K * m.L.rec;
    };
    for (int sg = top; sg >= bot; --sg) {
      // gate sizes of every lane's segment, read back from the tape records
      std::vector<int> ng(nl, 0), g0(nl, 0);
      std::vector<std::vector<int>> meta(nl);
      std::vector<std::vector<double>> dmeta(nl);
      for (int j = 0; j < nl; ++j) {
        const MixInfo& m = linfo[j];
        if (sg >= m.n_seg) continue;
        g0[j] = sg * m.K;
        ng[j] = std::min(m.G, (sg + 1) * m.K) - g0[j];
        meta[j].resize((size_t)ng[j] * 16);
        dmeta[j].resize((size_t)ng[j] * 16);
        const char* tb = tape_of(j, sg);
        HIPCHK(hipMemcpy2DAsync(meta[j].data(), 16 * sizeof(int), tb + m.L.ometa, m.L.rec, 16 * sizeof(int), ng[j],
                                hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpy2DAsync(dmeta[j].data(), 16 * sizeof(double), tb + m.L.odmeta, m.L.rec, 16 * sizeof(double),
                                ng[j], hipMemcpyDeviceToHost, s));
      }
      HIPCHK(hipStreamSynchronize(s));
      // lanes in order of decreasing segment length, so that the lanes still
      // active at step k are a prefix of each step's records
      std::vector<int> order;
      for (int j = 0; j < nl; ++j)
        if (ng[j] > 0) order.push_back(j);
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return ng[x] > ng[y]; });
      if (order.empty()) continue;
      const int steps = ng[order[0]];
      rec.clear();
      std::vector<std::pair<int, GateDims>> step_launch;   // (active lanes, largest sizes)
      for (int k = 0; k < steps; ++k) {
        GateDims mx{0, 0, 0, 0, 0, 0.0};
        int act = 0;
        for (int j : order) {
          if (k >= ng[j]) break;
          const MixInfo& m = linfo[j];
          mps_plan* p = m.p;
          MixLaneBufs* b = S.lanes[j];
          const int g = g0[j] + ng[j] - 1 - k, q = ng[j] - 1 - k;
          const int* mt = meta[j].data() + (size_t)q * 16;
          if (!(mt[0] >= 1 && mt[0] <= m.dc && mt[4] >= 1 && mt[4] <= m.dc && mt[5] >= 1 && mt[5] <= m.dc &&
                mt[6] >= 1 && mt[6] <= m.dc))
            fail(MPS_EDEVICE, "gate sizes read back from the tape are out of range");
          AdjLane a1;
          a1.R = rec_at(tape_of(j, sg), m.L, q);
          a1.W = W[j];
          a1.d = dims_of(mt, dmeta[j].data() + (size_t)q * 16, p->C.bond_h[g]);
          const int n = a1.d.n;
          const size_t site = (size_t)m.dc * 2 * m.dc;
          zd* Bbar = (zd*)b->Bbar.p;
          double* lambar = (double*)b->lambar.p;
          a1.Bbn = Bbar + (size_t)n * site;
          a1.Bbn1 = Bbar + (size_t)(n + 1) * site;
          a1.lb_out = lambar + (size_t)(n + 1) * m.dc;
          a1.lb_in = lambar + (size_t)n * m.dc;
          a1.gphi = (double*)b->gphi.p;
          a1.theta = th_dev[grp[j]];
          a1.gt = p->C.tab;
          a1.g = g;
          a1.kind = p->C.kind_h[g];
          a1.dc = m.dc;
          a1.ldc = m.ldc;
          a1.ldv = m.ldv;
          a1.eta = p->opts.broaden;
          rec.push_back(a1);
          mx.a = std::max(mx.a, a1.d.a);
          mx.m = std::max(mx.m, a1.d.m);
          mx.b = std::max(mx.b, a1.d.b);
          mx.r = std::max(mx.r, a1.d.r);
          ++act;
        }
        step_launch.push_back({act, mx});
      }
      AdjLane* rec_d = (AdjLane*)S.adj_dev.ensure(rec.size() * sizeof(AdjLane));
      HIPCHK(hipMemcpyAsync(rec_d, rec.data(), rec.size() * sizeof(AdjLane), hipMemcpyHostToDevice, s));
      size_t off = 0;
      for (const auto& sl : step_launch) {
        launch_gate_adjoint(rec_d + off, sl.first, sl.second, gw.stats, s);
        off += sl.first;
      }
      HIPCHK(hipGetLastError());
      // rec is rewritten for the next segment index only after this upload
      HIPCHK(hipStreamSynchronize(s));
      if (ctx->progress) ctx->progress(ctx->progress_user, "backward", S_max - sg, S_max);
    }
    top = bot - 1;
  }
  // ---- chain rule per lane
  for (int j = 0; j < nl; ++j) {
    mps_plan* p = linfo[j].p;
    PlanAdj& A = adj_of(p);
    if (!A.chain_built) build_chain(p, A);
    if (p->n_theta > 0)
      hipLaunchKernelGGL(k_chain_rule, dim3((p->n_theta + 255) / 256), dim3(256), 0, s, (const int*)A.chain_start.p,
                         (const int*)A.chain_list.p, p->C.tab, (const double*)S.lanes[j]->gphi.p, grad_dev[grp[j]],
                         p->n_theta);
  }
  HIPCHK(hipGetLastError());
  for (const GateStats& x : st) {
    gsum->disc_sum += x.disc_sum;
    gsum->disc_max = std::max(gsum->disc_max, x.disc_max);
    gsum->svd_flop += x.svd_flop;
    gsum->gemm_flop += x.gemm_flop;
    gsum->truncated += x.truncated;
    gsum->max_sweeps = std::max(gsum->max_sweeps, x.max_sweeps);
    gsum->noconv += x.noconv;
    gsum->degenerate_cuts += x.degenerate_cuts;
    gsum->max_bond = std::max(gsum->max_bond, x.max_bond);
    gsum->gates += x.gates;
  }
}

void plan_energy_grad_plans(mps_plan* const* plans, int n, const double* const* thetas, double* energies,
                            double* const* grads, mps_stats* stats) {
  if (n < 1) fail(MPS_EINVAL, "n_plans must be >= 1");
  if (!plans || !thetas || !energies || !grads) fail(MPS_EINVAL, "NULL argument");
  mps_plan* lead = plans[0];
  if (!lead) fail(MPS_EINVAL, "NULL plan");
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) fail(MPS_EINVAL, "NULL plan");
    if (plans[i]->ctx != lead->ctx) fail(MPS_EINVAL, "plans belong to different contexts");
    if (plans[i]->n_theta > 0 && (!thetas[i] || !grads[i])) fail(MPS_EINVAL, "NULL theta or gradient array");
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) fail(MPS_EINVAL, "a plan appears twice (use mps_energy_grad_batched)");
    validate_theta(thetas[i], plans[i]->n_theta);
  }
  mps_ctx* ctx = lead->ctx;
  hipStream_t s = ctx->stream;
  // parameters and gradients on the device, one row per plan
  std::vector<MixInfo> info(n);
  std::vector<size_t> off(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    info[i] = mix_info(plans[i]);
    off[i + 1] = off[i] + (size_t)std::max(1, plans[i]->n_theta);
  }
  PlanAdj& LA = adj_of(lead);
  if (!LA.mix) LA.mix = new MixSet();
  double* th = (double*)LA.mix->thetas.ensure(2 * off[n] * sizeof(double));
  double* gd = th + off[n];
  std::vector<const double*> th_dev(n);
  std::vector<double*> g_dev(n);
  for (int i = 0; i < n; ++i) {
    th_dev[i] = th + off[i];
    g_dev[i] = gd + off[i];
    if (plans[i]->n_theta > 0)
      HIPCHK(hipMemcpyAsync(th + off[i], thetas[i], plans[i]->n_theta * sizeof(double), hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  // groups of lanes that one cooperative launch holds
  size_t shm = 0;
  int max_dc = 2;
  for (auto& m : info) {
    shm = std::max(shm, chain_lds_bytes(m.dc));
    max_dc = std::max(max_dc, m.dc);
  }
  const int cap = mixed_blocks_max(shm);
  if (cap <= 0) fail(MPS_EDEVICE, "the mixed gate-chain kernel cannot be resident");
  ctx->ensure_gate_work(max_dc, lead->trunc, lead->opts.max_sweeps);
  ctx->reset_stats();   // degenerate pairs of the reverse pass are counted here
  GateStats gsum{};
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  std::vector<int> grp;
  auto flush = [&]() {
    if (grp.empty()) return;
    mixed_group(lead, info, grp, th_dev, energies, g_dev, &gsum, cap);
    grp.clear();
  };
  std::vector<int2> blk;
  for (int i = 0; i < n; ++i) {
    std::vector<int> trial(grp);
    trial.push_back(i);
    if (mix_block_table(info, trial, blk) > cap) {
      flush();
      trial.assign(1, i);
      if (mix_block_table(info, trial, blk) > cap)
        fail(MPS_EDEVICE, "a lane needs more work-groups than the device holds at once");
    }
    grp = trial;
  }
  flush();
  HIPCHK(hipEventRecord(e1, s));
  for (int i = 0; i < n; ++i)
    if (plans[i]->n_theta > 0)
      HIPCHK(hipMemcpyAsync(grads[i], g_dev[i], plans[i]->n_theta * sizeof(double), hipMemcpyDeviceToHost, s));
  GateStats gs;
  HIPCHK(hipMemcpyAsync(&gs, ctx->gw.stats, sizeof(GateStats), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (gsum.noconv) fail(MPS_ENOCONV, "a Jacobi SVD did not converge");
  bool strict = false;
  for (int i = 0; i < n; ++i) strict = strict || plans[i]->opts.strict_degenerate;
  if (gs.degen_grad > 0 && strict)
    fail(MPS_EDEGEN, std::to_string(gs.degen_grad) + " degenerate singular pairs carry a cotangent");
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->discarded_weight_sum = gsum.disc_sum;
    stats->discarded_weight_max = gsum.disc_max;
    stats->max_bond = gsum.max_bond;
    stats->gates_truncated = gsum.truncated;
    stats->max_sweeps_used = gsum.max_sweeps;
    stats->degenerate_cuts = gsum.degenerate_cuts;
    stats->n_gates_applied = gsum.gates;
    stats->t_backward_ms = ms;
  }
}

PlanAdj::~PlanAdj() {
  delete batch;
  delete mix;
}
