// Two-qubit gate update on the MPS (arXiv:2211.07983, Sec. 3, the Hastings
// update for a nearest-neighbour gate):
//   C  = Q . (B_n B_{n+1})            (contraction, k_contract)
//   C~ = lambda_{n-1} C               (row weighting, fused into k_contract)
//   C~ = U s W  truncated to r values (one-sided Jacobi SVD, k_svd_jacobi)
//   B~_n = C W_r^dagger / nu, B~_{n+1} = W_r, lambda_n = s_r / nu   (k_update_*)
// All sizes are read from the device-side bond dimensions, so a whole circuit
// is enqueued without any host synchronisation.  k_chain_lanes runs the same
// three steps for a run of gates of many independent MPS ("lanes") in one
// cooperative launch.

#include <algorithm>
#include <vector>

#include "engine.h"


// ----------------------------------------------------------------------------
// k_contract: C[(a,i'),(j',b)] = sum_{ij} Q[(i'j'),(ij)] sum_g B_n[a,i,g] B_{n+1}[g,j,b]
// and A = lambda_{n-1}[a] C (trans = 0) or A = (lambda_{n-1} C)^H (trans = 1).  GEMM rows r = 2a + i, columns c = 2b + j so that
// each thread holds the four (i, j) values of one (alpha, beta) pair.
// C and A are column-major with leading dimension ldc; column index j'*b + beta.
// ----------------------------------------------------------------------------
// One 32 x 32 output tile (bx, by) of the contraction; part = by * nbx + bx
// indexes the tile's |C~|^2 partial sum.  sbuf: LDS staging for the tile
// GEMM (ZT_LDS_ELEMS elements), or nullptr for the kernel's own.
template <bool DYN>
__device__ void contract_tile(const MpsView& st, const GateTable& gt, int g, const double* theta, zd* C, zd* A,
                              int ldc, double* nrm_part, int trans, int bx, int by, int nbx, zd* sbuf,
                              double dphi = 0.0) {
  __shared__ zd Q[16];
  __shared__ double red[256];
  const int n = gt.bond[g];
  const int a = st.dims[n], m = st.dims[n + 1], b = st.dims[n + 2];
  const int Mr = 2 * a, Nc = 2 * b;
  const int i0 = by * ZT_M, j0 = bx * ZT_N;
  const int part = by * nbx + bx;
  if (i0 >= Mr || j0 >= Nc) {
    if (threadIdx.x == 0) nrm_part[part] = 0.0;
    return;
  }
  gate_matrix(gt, g, theta, Q, dphi);
  const zd* Bl = st.site(n);
  const zd* Br = st.site(n + 1);
  const int dc = st.dcap;
  auto fa = [&](int r, int k) { return Bl[(size_t)(r >> 1) * 2 * dc + (r & 1) * dc + k]; };
  auto fb = [&](int k, int c) { return Br[(size_t)k * 2 * dc + (c & 1) * dc + (c >> 1)]; };
  zd acc[2][2];
  if constexpr (DYN)
    ztile_acc_in(Mr, Nc, m, i0, j0, fa, fb, acc, sbuf, sbuf + ZT_K * (ZT_M + 1));
  else
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
        if (trans)
          A[(size_t)(2 * al + ip) * ldc + (jp * b + be)] = zconj(wv);
        else
          A[idx] = wv;
        nrm += zabs2(wv);
      }
  }
  nrm = block_sum256(nrm, red);
  if (threadIdx.x == 0) nrm_part[part] = nrm;
}

__global__ __launch_bounds__(256) void k_contract(MpsView st, GateTable gt, int g, const double* theta,
                                                  zd* C, zd* A, int ldc, double* nrm_part, int trans,
                                                  int* rotflag) {
  // the Jacobi kernel that follows counts rotations per sweep in rotflag
  // and synchronises its work-groups on the counter after the 128 flags
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 130) rotflag[threadIdx.x] = 0;
  contract_tile<false>(st, gt, g, theta, C, A, ldc, nrm_part, trans, blockIdx.x, blockIdx.y, gridDim.x, nullptr);
}

// ----------------------------------------------------------------------------
// One-sided block Jacobi SVD of A (M x ncol, column-major), accumulating the
// right rotations in V (ncol x ncol).  P work-groups each hold a pair of
// column blocks of width W in LDS; the pairs follow a tournament over the 2P
// blocks (round_blocks), with a barrier over the P work-groups between
// rounds.  Round 0 of a sweep orthogonalises all
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

// Blocks of work-group p in round k of a sweep over 2P blocks: the
// precomputed schedule when P is a power of two (consecutive rounds of a
// work-group share a block), else the round robin above.
__device__ inline void round_blocks(const unsigned char* sched, int P, int k, int p, int& q0, int& q1) {
  if (sched && (P & (P - 1)) == 0 && P <= 64) {
    size_t off = 0;
    for (int q = 1; q < P; q <<= 1) off += (size_t)(2 * q - 1) * q * 2;
    const unsigned char* e = sched + off + ((size_t)k * P + p) * 2;
    q0 = e[0];
    q1 = e[1];
  } else {
    tourney(P, k, p, q0, q1);
  }
}

// Cross-lane sums over groups of TPP consecutive lanes.  Every step pairs
// lanes symmetrically (l <-> l^1, l^2, the two halves of 8, of 16, of 32), so
// all lanes of a group end with bitwise identical totals and therefore take
// identical rotation decisions.
template <int CTRL>
__device__ inline double dpp_add(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return v + __hiloint2double(hi, lo);
}
__device__ inline double swz16_add(double v) {   // lane l <-> l ^ 16
  const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
  return v + __hiloint2double(hi, lo);
}
template <int TPP>
__device__ inline void group_sum4(double& a, double& b, double& c, double& d) {
  static_assert(TPP == 8 || TPP == 16 || TPP == 32 || TPP == 64, "group size");
  a = dpp_add<0xB1>(a); b = dpp_add<0xB1>(b); c = dpp_add<0xB1>(c); d = dpp_add<0xB1>(d);      // quad [1,0,3,2]
  a = dpp_add<0x4E>(a); b = dpp_add<0x4E>(b); c = dpp_add<0x4E>(c); d = dpp_add<0x4E>(d);      // quad [2,3,0,1]
  a = dpp_add<0x141>(a); b = dpp_add<0x141>(b); c = dpp_add<0x141>(c); d = dpp_add<0x141>(d);  // half-row mirror
  if (TPP >= 16) {
    a = dpp_add<0x140>(a); b = dpp_add<0x140>(b); c = dpp_add<0x140>(c); d = dpp_add<0x140>(d);  // row mirror
  }
  if (TPP >= 32) {
    a = swz16_add(a); b = swz16_add(b); c = swz16_add(c); d = swz16_add(d);
  }
  if (TPP == 64) {
    a += __shfl_xor(a, 32); b += __shfl_xor(b, 32); c += __shfl_xor(c, 32); d += __shfl_xor(d, 32);
  }
}

// Rotation of the column pair (x, y): alpha = |x|^2, beta = |y|^2,
// gamma = x^H y = |gamma| e^{i phi}.  With d = beta - alpha and
// h = 2 sign(d) / (|d| + sqrt(d^2 + 4 |gamma|^2)) the tangent of the angle is
// t = h |gamma| and c = 1 / sqrt(1 + t^2); the unitary update
//   x' = c x - c h conj(gamma) y,    y' = c h gamma x + c y
// makes x'^H y' = 0.  Returns false when the pair is already orthogonal
// (|gamma| <= tol sqrt(alpha beta)) or negligible (|gamma| <= floor_g).
__device__ inline bool jacobi_rotation(double al, double be, double gr, double gi, double tol, double floor_g,
                                       double& c, zd& p, zd& q) {
  const double g2 = fma(gr, gr, gi * gi);
  const double ab = al * be;
  if (!(ab > 1e-300) || g2 <= tol * tol * ab || g2 <= floor_g * floor_g) return false;
  const double d = be - al;
  const double qd = sqrt(fma(d, d, 4.0 * g2));
  const double h = (d >= 0.0 ? 2.0 : -2.0) / (fabs(d) + qd);
  c = rsqrt(fma(h * h, g2, 1.0));
  const double ch = c * h;
  p = zmk(ch * gr, -ch * gi);    // c h conj(gamma)
  q = zmk(ch * gr, ch * gi);     // c h gamma
  return true;
}

// partial sums of |u|^2, |v|^2 and conj(u) v
__device__ inline void pair_acc(const zd u, const zd v, double& al, double& be, double& gr, double& gi) {
  al = fma(u.x, u.x, fma(u.y, u.y, al));
  be = fma(v.x, v.x, fma(v.y, v.y, be));
  gr = fma(u.x, v.x, fma(u.y, v.y, gr));
  gi = fma(u.x, v.y, fma(-u.y, v.x, gi));
}

__device__ inline zd rot_x(const zd u, const zd v, double c, const zd p) { return zsub(zscale(u, c), zmul(p, v)); }
__device__ inline zd rot_y(const zd u, const zd v, double c, const zd q) { return zadd(zmul(q, u), zscale(v, c)); }

// Loads the two column blocks (q0, q1) of a (and of v when ACC) into LDS with
// LB independent loads in flight per thread (the blocks come from other
// work-groups through the device-coherent level after each round's barrier,
// so the loads are latency-bound; more in flight means fewer round trips).
constexpr int LB = 16;
// Slots: columns [0, W) of the LDS pair hold block q0, [W, 2W) block q1;
// only the slots in [s0, s1) (in columns) are moved.
__device__ inline void load_blocks(zd* dst, int ldst, const zd* src, int lds, int rows, int ncol, int W, int q0,
                                   int q1, bool identity, int s0 = 0, int s1 = -1) {
  if (s1 < 0) s1 = 2 * W;
  const int tot = (s1 - s0) * rows;
  for (int e0 = threadIdx.x; e0 < tot; e0 += LB * 256) {
    zd buf[LB];
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int e = e0 + u * 256;
      if (e < tot) {
        const int c = s0 + e / rows, r = e - (c - s0) * rows;
        const int gc = (c < W ? q0 : q1) * W + (c % W);
        buf[u] = identity ? zmk(r == gc ? 1.0 : 0.0, 0.0) : (gc < ncol ? src[(size_t)gc * lds + r] : zmk(0.0, 0.0));
      }
    }
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int e = e0 + u * 256;
      if (e < tot) {
        const int c = s0 + e / rows, r = e - (c - s0) * rows;
        dst[c * ldst + r] = buf[u];
      }
    }
  }
}

__device__ inline void store_blocks(zd* dst, int ldd, const zd* src, int lsrc, int rows, int ncol, int W, int q0,
                                    int q1, int s0 = 0, int s1 = -1) {
  if (s1 < 0) s1 = 2 * W;
  for (int e = threadIdx.x; e < (s1 - s0) * rows; e += 256) {
    const int c = s0 + e / rows, r = e - (c - s0) * rows;
    const int gc = (c < W ? q0 : q1) * W + (c % W);
    if (gc < ncol) dst[(size_t)gc * ldd + r] = src[c * lsrc + r];
  }
}

// Barrier over the nblk work-groups of one SVD (the whole grid of a
// single-SVD launch, or one lane of a batched launch): a monotonic counter,
// zeroed before the launch, that every work-group increments once per
// barrier; barrier k completes when it reaches (k + 1) nblk.  The launches
// are cooperative, so every work-group is resident and the wait ends; the spin
// is bounded all the same and a timeout is recorded in *err (reported as an
// error by the host) instead of waiting forever.  The release and acquire are
// agent-scope even when the work-groups share one XCD: an L1-only invalidate
// (the workgroup-scope cache operation) left stale blocks visible across
// compute units and the Jacobi sweeps stopped converging.
struct LaneBarrier {
  unsigned long long* ctr;
  int* err;
  unsigned long long nblk;
  unsigned long long gen;
  __device__ void sync() {
    // every wave's global stores of the phase complete (the work-group barrier
    // alone does not wait for them), then one agent-scope release for the
    // work-group: a single L2 write-back instead of one per wave
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // A single work-group shares its compute unit's L1 and needs no more:
    // its blocks go through global memory only to itself, which the
    // work-group barrier above already orders.  Skipping the agent-scope
    // fences also spares the other lanes on its XCD an L2 flush per round.
    if (nblk == 1) {
      ++gen;
      return;
    }
    if (threadIdx.x == 0) {
      const unsigned long long target = (gen + 1) * nblk;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // relaxed polls: an acquire load would invalidate the caches on every
      // poll, under every other lane resident on the same L2
      unsigned spins = 0;
      while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(2);
        // about a second: far beyond one Jacobi round; after a timeout every
        // later wait of the launch ends at once
        if (++spins > (1u << 20) || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
      // one acquire after the wait: the other work-groups' stores are visible
      // to this compute unit
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    ++gen;
    __syncthreads();
  }
};

// LDS column pitch of the Jacobi blocks: the matrix's leading dimension, at
// least the 8 * 256 / W rows that the 256 threads of a pair group cover.
__host__ __device__ inline int svd_pitch(int ld, int W) {
  const int R = 8 * 256 / W;
  return ld > R ? ld : R;
}

template <int W, bool ACC, class Barrier>
__device__ void svd_body(const SvdArgs& s, const int p, const int nblk, Barrier& bar) {
  constexpr int TPP = 256 / W;     // threads per column pair
  constexpr int RPT = 8;           // rows per thread held in registers (M, ncol <= 8 * TPP)
  extern __shared__ zd lds[];
  const int n = s.bond;
  const int a = s.dims[n], b = s.dims[n + 2];
  const int M = s.trans ? 2 * b : 2 * a, ncol = s.trans ? 2 * a : 2 * b;
  const int P = (ncol + 2 * W - 1) / (2 * W);
  const int t = threadIdx.x;
  const int mpad = svd_pitch(s.lda, W);   // LDS column stride for A
  const int vpad = svd_pitch(s.ldv, W);   // LDS column stride for V
  zd* Al = lds;                    // [2W][mpad]
  zd* Vl = lds + 2 * W * mpad;     // [2W][vpad] (ACC only)
  __shared__ int sh_rot;
  __shared__ int sh_stop;
  const int pr = t / TPP, lt = t % TPP;
  const double tol = s.tol;
  // Rows past the matrix in the LDS blocks hold zeros for the whole call: the
  // cross rounds rotate all RPT * TPP rows of a pair without bounds checks, and
  // rotations keep zero rows zero.
  for (int e = t; e < 2 * W * RPT * TPP; e += 256) {
    const int c = e / (RPT * TPP), r = e - c * (RPT * TPP);
    if (r >= M) Al[c * mpad + r] = zmk(0.0, 0.0);
    if (ACC && r >= ncol) Vl[c * vpad + r] = zmk(0.0, 0.0);
  }
  // |gamma| below floor = 1e-28 |A|_F^2 means both columns are negligible (far
  // below any kept Schmidt value): such pairs are left alone, which keeps wide
  // matrices, whose surplus columns must shrink to zero, from sweeping forever.
  double fro = 0.0;
  for (int q = 0; q < s.nparts; ++q) fro += s.nrm_part[q];
  const double floor_g = 1e-28 * fro;
  int sweep = 0;
  for (; sweep < s.max_sweeps; ++sweep) {
    if (t == 0) sh_rot = 0;
    int hold0 = -1, hold1 = -1;   // blocks resident in the two LDS slots
    for (int k = 0; k < 2 * P - 1; ++k) {
      int q0, q1;
      round_blocks(s.sched, P, k, p, q0, q1);
      if (p < P) {
        // a block this work-group already holds stays in its slot
        if (q0 == hold1 || q1 == hold0) {
          const int q = q0;
          q0 = q1;
          q1 = q;
        }
        const int s0 = q0 == hold0 ? W : 0, s1 = q1 == hold1 ? W : 2 * W;
        if (s0 < s1) {
          load_blocks(Al, mpad, s.A, s.lda, M, ncol, W, q0, q1, false, s0, s1);
          if (ACC) load_blocks(Vl, vpad, s.V, s.ldv, ncol, ncol, W, q0, q1, sweep == 0 && k == 0, s0, s1);
        }
        hold0 = q0;
        hold1 = q1;
        __syncthreads();
        bool rot = false;
        if (k == 0) {
          // all pairs of the 2W columns, circle ordering
          for (int sub = 0; sub < 2 * W - 1; ++sub) {
            const int R = 2 * W - 1;
            int c0, c1;
            if (pr == 0) {
              c0 = R;
              c1 = sub % R;
            } else {
              c0 = (sub + pr) % R;
              c1 = (sub - pr + R) % R;
            }
            zd* x = Al + c0 * mpad;
            zd* y = Al + c1 * mpad;
            double al0 = 0.0, be0 = 0.0, gr0 = 0.0, gi0 = 0.0, al1 = 0.0, be1 = 0.0, gr1 = 0.0, gi1 = 0.0;
            int r = lt;
            for (; r + TPP < M; r += 2 * TPP) {
              pair_acc(x[r], y[r], al0, be0, gr0, gi0);
              pair_acc(x[r + TPP], y[r + TPP], al1, be1, gr1, gi1);
            }
            if (r < M) pair_acc(x[r], y[r], al0, be0, gr0, gi0);
            double al = al0 + al1, be = be0 + be1, gr = gr0 + gr1, gi = gi0 + gi1;
            group_sum4<TPP>(al, be, gr, gi);
            double c;
            zd pp, qq;
            if (jacobi_rotation(al, be, gr, gi, tol, floor_g, c, pp, qq)) {
              for (int rr = lt; rr < M; rr += TPP) {
                const zd u = x[rr], v = y[rr];
                x[rr] = rot_x(u, v, c, pp);
                y[rr] = rot_y(u, v, c, qq);
              }
              if (ACC) {
                zd* xv = Vl + c0 * vpad;
                zd* yv = Vl + c1 * vpad;
                for (int rr = lt; rr < ncol; rr += TPP) {
                  const zd u = xv[rr], v = yv[rr];
                  xv[rr] = rot_x(u, v, c, pp);
                  yv[rr] = rot_y(u, v, c, qq);
                }
              }
              rot = true;
            }
            __syncthreads();
          }
        } else {
          // cross pairs: column pr of the first block stays in registers
          // (all RPT row chunks, the zero padding included: guarding the
          // padding chunks made the batched chain launch 6 % slower)
          const int c0 = pr;
          zd xr[RPT], xv[RPT];
          const zd* xa = Al + c0 * mpad + lt;
          const zd* xva = Vl + c0 * vpad + lt;
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            xr[i] = xa[i * TPP];
            if (ACC) xv[i] = xva[i * TPP];
          }
          for (int sub = 0; sub < W; ++sub) {
            const int c1 = W + ((pr + sub) & (W - 1));
            zd* y = Al + c1 * mpad + lt;
            zd yr[RPT];
            double al0 = 0.0, be0 = 0.0, gr0 = 0.0, gi0 = 0.0, al1 = 0.0, be1 = 0.0, gr1 = 0.0, gi1 = 0.0;
#pragma unroll
            for (int i = 0; i < RPT; i += 2) {
              yr[i] = y[i * TPP];
              yr[i + 1] = y[(i + 1) * TPP];
              pair_acc(xr[i], yr[i], al0, be0, gr0, gi0);
              pair_acc(xr[i + 1], yr[i + 1], al1, be1, gr1, gi1);
            }
            double al = al0 + al1, be = be0 + be1, gr = gr0 + gr1, gi = gi0 + gi1;
            group_sum4<TPP>(al, be, gr, gi);
            double c;
            zd pp, qq;
            if (jacobi_rotation(al, be, gr, gi, tol, floor_g, c, pp, qq)) {
#pragma unroll
              for (int i = 0; i < RPT; ++i) {
                const zd u = xr[i], v = yr[i];
                xr[i] = rot_x(u, v, c, pp);
                y[i * TPP] = rot_y(u, v, c, qq);
              }
              if (ACC) {
                zd* yv = Vl + c1 * vpad + lt;
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                  const zd u = xv[i], v = yv[i * TPP];
                  xv[i] = rot_x(u, v, c, pp);
                  yv[i * TPP] = rot_y(u, v, c, qq);
                }
              }
              rot = true;
            }
            __syncthreads();
          }
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            Al[c0 * mpad + lt + i * TPP] = xr[i];
            if (ACC) Vl[c0 * vpad + lt + i * TPP] = xv[i];
          }
          __syncthreads();
        }
        if (rot && lt == 0) sh_rot = 1;
        // blocks that leave this work-group after this round go back to
        // global memory (all of them after the sweep's last round)
        int n0 = -1, n1 = -1;
        if (k + 1 < 2 * P - 1) round_blocks(s.sched, P, k + 1, p, n0, n1);
        const bool keep0 = hold0 == n0 || hold0 == n1, keep1 = hold1 == n0 || hold1 == n1;
        const int t0 = keep0 ? W : 0, t1 = keep1 ? W : 2 * W;
        if (t0 < t1) {
          store_blocks(s.A, s.lda, Al, mpad, M, ncol, W, q0, q1, t0, t1);
          if (ACC) store_blocks(s.V, s.ldv, Vl, vpad, ncol, ncol, W, q0, q1, t0, t1);
        }
        if (!keep0) hold0 = -1;
        if (!keep1) hold1 = -1;
      }
      // Sweep finished with this round: count the work-groups that rotated.
      // The counter of this sweep (zeroed before the launch) is incremented
      // before the round's barrier and read after it, so every work-group
      // reads the same value and all of them leave the loop after the same
      // number of barriers.
      if (k == 2 * P - 2) {
        __syncthreads();   // sh_rot final
        if (t == 0 && sh_rot)
          __hip_atomic_fetch_add(&s.rotflag[sweep], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      bar.sync();
    }
    if (t == 0) sh_stop = __hip_atomic_load(&s.rotflag[sweep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    __syncthreads();
    if (sh_stop) break;
  }
  const int used = sweep + 1;
  // The Jacobi blocks are back in global memory: the reductions below use
  // the front of the block LDS (at least 64 KiB for every width), so a kernel
  // that instantiates several widths holds no per-width shared arrays.
  double* red = (double*)lds;          // [256]
  double* shs = (double*)lds + 256;    // [1024]
  // singular values: column norms
  for (int c = p; c < ncol; c += nblk) {
    double acc = 0.0;
    for (int r = t; r < M; r += 256) acc += zabs2(s.A[(size_t)c * s.lda + r]);
    acc = block_sum256(acc, red);
    if (t == 0) s.sv[c] = sqrt(acc);
  }
  bar.sync();
  if (p != 0) return;
  // work-group 0: order, rank, normalisation, lambda, statistics
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
    const double pp = M < ncol ? M : ncol;
    gs->svd_flop += 84.0 * pp * pp * pp;
    // the gate's GEMMs around this SVD: (2a x m)(m x 2b) contraction, the 4x4
    // gate matrix on every (alpha, beta), and the (2a x 2b)(2b x r) update
    const double ga = a, gb = b, gm = s.dims[n + 1];
    gs->gemm_flop += 8.0 * (4.0 * ga * gb * gm + 16.0 * ga * gb + 4.0 * ga * gb * r);
    s.dims[n + 1] = r;
  }
  __syncthreads();
  const int r = s.gmeta[0];
  const double nu = s.gdmeta[0];
  for (int q = t; q < r; q += 256) s.lam_out[q] = shs[s.perm[q]] / nu;
}

// stride 8: the grid is 8 P work-groups of which every eighth works, so the
// P working ones share XCD 0 (work-groups go to the XCDs round-robin) and
// with it one L2; stride 1: all P work.
template <int W, bool ACC>
__global__ __launch_bounds__(256) void k_svd_jacobi(SvdArgs s, int stride) {
  if (blockIdx.x % stride) return;
  const int nblk = gridDim.x / stride;
  LaneBarrier bar{s.bar, &s.stats->barrier_timeout, (unsigned long long)nblk, 0ull};
  svd_body<W, ACC>(s, blockIdx.x / stride, nblk, bar);
}

// ----------------------------------------------------------------------------
// k_update_left: B~_n[(a,i'), mu] = sum_c C[(a,i'), c] V[c, perm[mu]] / nu.
// ----------------------------------------------------------------------------
template <bool DYN>
__device__ void update_left_tile(const MpsView& st, int n, const zd* C, int ldc, const zd* V, int ldv,
                                 const int* perm, const int* gmeta, const double* gdmeta, int bx, int by, zd* sbuf) {
  const int a = st.dims[n], b = st.dims[n + 2];
  const int r = gmeta[0];
  const double inv = 1.0 / gdmeta[0];
  const int Mr = 2 * a, Nc = r, K = 2 * b;
  const int i0 = by * ZT_M, j0 = bx * ZT_N;
  if (i0 >= Mr || j0 >= Nc) return;
  auto fa = [&](int row, int k) { return C[(size_t)k * ldc + row]; };
  auto fb = [&](int k, int mu) { return V[(size_t)perm[mu] * ldv + k]; };
  zd acc[2][2];
  if constexpr (DYN)
    ztile_acc_in(Mr, Nc, K, i0, j0, fa, fb, acc, sbuf, sbuf + ZT_K * (ZT_M + 1));
  else
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

__global__ __launch_bounds__(256) void k_update_left(MpsView st, int n, const zd* C, int ldc, const zd* V,
                                                     int ldv, const int* perm, const int* gmeta,
                                                     const double* gdmeta) {
  update_left_tile<false>(st, n, C, ldc, V, ldv, perm, gmeta, gdmeta, blockIdx.x, blockIdx.y, nullptr);
}

// k_update_right: B~_{n+1}[mu, j', beta] = conj(V[j'*b + beta, perm[mu]]).
__device__ void update_right_row(const MpsView& st, int n, const zd* V, int ldv, const int* perm,
                                 const int* gmeta, int mu) {
  const int b = st.dims[n + 2];
  const int r = gmeta[0];
  if (mu >= r) return;
  zd* Br = st.site(n + 1);
  const int dc = st.dcap;
  const int col = perm[mu];
  for (int e = threadIdx.x; e < 2 * b; e += 256) {
    const int jp = e / b, be = e % b;
    Br[(size_t)mu * 2 * dc + jp * dc + be] = zconj(V[(size_t)col * ldv + e]);
  }
}

__global__ __launch_bounds__(256) void k_update_right(MpsView st, int n, const zd* V, int ldv, const int* perm,
                                                      const int* gmeta) {
  update_right_row(st, n, V, ldv, perm, gmeta, blockIdx.x);
}

// Forward mode (Jacobi on X = C~^H, no accumulation): column c of the rotated
// X is s_c w_c^H, so w_c = conj(X[:, c]) / s_c.
// k_update_left_t: B~_n[(a,i'), mu] = sum_k C[(a,i'), k] X[k, perm[mu]] / (s_{perm[mu]} nu).
__global__ __launch_bounds__(256) void k_update_left_t(MpsView st, int n, const zd* C, int ldc, const zd* X,
                                                       const double* sv, const int* perm, const int* gmeta,
                                                       const double* gdmeta) {
  const int a = st.dims[n], b = st.dims[n + 2];
  const int r = gmeta[0];
  const double nu = gdmeta[0];
  const int Mr = 2 * a, Nc = r, K = 2 * b;
  const int i0 = blockIdx.y * ZT_M, j0 = blockIdx.x * ZT_N;
  if (i0 >= Mr || j0 >= Nc) return;
  auto fa = [&](int row, int k) { return C[(size_t)k * ldc + row]; };
  auto fb = [&](int k, int mu) { return X[(size_t)perm[mu] * ldc + k]; };
  zd acc[2][2];
  ztile_acc(Mr, Nc, K, i0, j0, fa, fb, acc);
  const int r0 = i0 + tile_row0(), c0 = j0 + tile_col0();
  zd* Bn = st.site(n);
  const int dc = st.dcap;
  for (int y = 0; y < 2; ++y) {
    const int mu = c0 + y;
    if (mu >= Nc) continue;
    const double inv = 1.0 / (sv[perm[mu]] * nu);
    for (int x = 0; x < 2; ++x) {
      const int row = r0 + x;
      if (row < Mr) Bn[(size_t)(row >> 1) * 2 * dc + (row & 1) * dc + mu] = zscale(acc[x][y], inv);
    }
  }
}

// k_update_right_t: B~_{n+1}[mu, j', beta] = conj(X[j'*b + beta, perm[mu]]) / s_{perm[mu]}.
__global__ __launch_bounds__(256) void k_update_right_t(MpsView st, int n, const zd* X, int ldc, const double* sv,
                                                        const int* perm, const int* gmeta) {
  const int b = st.dims[n + 2];
  const int r = gmeta[0];
  const int mu = blockIdx.x;
  if (mu >= r) return;
  zd* Br = st.site(n + 1);
  const int dc = st.dcap;
  const int col = perm[mu];
  const double inv = 1.0 / sv[col];
  for (int e = threadIdx.x; e < 2 * b; e += 256) {
    const int jp = e / b, be = e % b;
    Br[(size_t)mu * 2 * dc + jp * dc + be] = zscale(zconj(X[(size_t)col * ldc + e]), inv);
  }
}

// ----------------------------------------------------------------------------
// Batched segment recompute: lane kernels.  Lane l replays gate g0 + step of its
// segment on its own state and writes the gate's tape record.
// ----------------------------------------------------------------------------
struct LaneRec {
  zd *Bl, *Br, *C, *A, *V;
  double *lam, *sv, *dmeta;
  int *perm, *meta;
};

__device__ inline LaneRec lane_rec(const GateLane& ln, const TapeLayout& L, int step) {
  char* r = ln.tape + (size_t)step * ln.rec_stride * L.rec;
  LaneRec R;
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

__device__ inline SvdArgs lane_svd_args(const GateLane& ln, const LaneConst& c, int n, const LaneRec& R) {
  SvdArgs s;
  s.A = R.A;
  s.lda = c.ldc;
  s.V = R.V;
  s.ldv = c.ldv;
  s.dims = ln.st.dims;
  s.bond = n;
  s.sv = R.sv;
  s.perm = R.perm;
  s.gmeta = R.meta;
  s.gdmeta = R.dmeta;
  s.rotflag = ln.rotflag;
  s.bar = ln.bar;
  s.sched = c.sched;
  s.lam_out = ln.st.lam + (size_t)(n + 1) * ln.st.dcap;
  s.stats = ln.stats;
  s.eps = c.eps;
  s.dmax = c.dmax;
  s.tol = c.tol;
  s.max_sweeps = c.max_sweeps;
  s.nrm_part = ln.nrm_part;
  s.nparts = c.nparts;
  s.trans = 0;
  return s;
}

// Work-group p of nblk copies its share of `words` 8-byte words.
__device__ inline void copy_words(unsigned long long* dst, const unsigned long long* src, size_t words, int p,
                                  int nblk) {
  for (size_t e = (size_t)p * 256 + threadIdx.x; e < words; e += (size_t)nblk * 256) dst[e] = src[e];
}

// The gate chain of one lane on work-group p of its nblk: ln.ng gates from
// ln.g0, each contraction tiles, Jacobi SVD and site update with the lane's
// barrier in between; the state before the first gate goes to ln.ckpt.
// Always inlined: as a call (the mixed kernel instantiates four widths) it
// passed its state through the scratch stack, about 1 KB per thread.
template <int W>
__device__ __attribute__((always_inline)) void chain_body(const GateLane& ln, const LaneConst& c, int p, int nblk,
                                                          int record, zd* sbuf) {
  LaneBarrier bar{ln.bar, ln.err, (unsigned long long)nblk, 0ull};
  const MpsView& st = ln.st;
  const int dc = st.dcap;
  const int tiles = (c.ldc + ZT_M - 1) / ZT_M;
  const int tm = (2 * dc + ZT_M - 1) / ZT_M, tn = (dc + ZT_N - 1) / ZT_N;
  if (ln.ckpt) {
    // the state before the lane's first gate (the update below writes only
    // after two barriers, which this copy precedes); layout: B, dims at ck_B,
    // lambda at the next 8-byte boundary after the dims
    copy_words((unsigned long long*)ln.ckpt, (const unsigned long long*)st.B, c.ck_B / 8, p, nblk);
    int* dd = (int*)(ln.ckpt + c.ck_B);
    for (size_t e = (size_t)p * 256 + threadIdx.x; e < c.ck_dims / 4; e += (size_t)nblk * 256) dd[e] = st.dims[e];
    copy_words((unsigned long long*)(ln.ckpt + ((c.ck_B + c.ck_dims + 7) / 8) * 8), (const unsigned long long*)st.lam,
               c.ck_lam / 8, p, nblk);
  }
  for (int step = 0; step < ln.ng; ++step) {
    const int g = ln.g0 + step;
    const int n = c.gt.bond[g];
    const LaneRec R = lane_rec(ln, c.L, step);
    if (record) {
      const int a = st.dims[n], m = st.dims[n + 1], b = st.dims[n + 2];
      const size_t site = (size_t)dc * 2 * dc;
      const zd* s0 = st.site(n);
      const zd* s1 = st.site(n + 1);
      for (size_t e = (size_t)p * 256 + threadIdx.x; e < site; e += (size_t)nblk * 256) {
        const int row = (int)(e / dc), col = (int)(e % dc);
        const int l = row >> 1;
        if (l < a && col < m) R.Bl[e] = s0[e];
        if (l < m && col < b) R.Br[e] = s1[e];
      }
      if (p == 0) {
        for (int q = threadIdx.x; q < a; q += 256) R.lam[q] = st.lam[(size_t)n * dc + q];
        if (threadIdx.x == 0) {
          R.meta[4] = a;
          R.meta[5] = m;
          R.meta[6] = b;
        }
      }
    }
    // The sweep votes of the lane start at zero.  The lane's work-groups
    // update them with device-scope atomics, so the reset is a device-scope
    // atomic store as well (ordered before the next barrier's release).
    if (p == 0 && threadIdx.x < 128)
      __hip_atomic_store(&ln.rotflag[threadIdx.x], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int tile = p; tile < tiles * tiles; tile += nblk)
      contract_tile<true>(st, c.gt, g, ln.theta, R.C, R.A, c.ldc, ln.nrm_part, 0, tile % tiles, tile / tiles, tiles,
                          sbuf, g == ln.shift_gate ? ln.shift : 0.0);
    bar.sync();
    const SvdArgs s = lane_svd_args(ln, c, n, R);
    svd_body<W, true>(s, p, nblk, bar);
    bar.sync();
    for (int tile = p; tile < tm * tn; tile += nblk)
      update_left_tile<true>(st, n, R.C, c.ldc, R.V, c.ldv, R.perm, R.meta, R.dmeta, tile % tn, tile / tn, sbuf);
    for (int mu = p; mu < dc; mu += nblk) update_right_row(st, n, R.V, c.ldv, R.perm, R.meta, mu);
    bar.sync();
  }
}

template <int W>
__global__ __launch_bounds__(256) void k_chain_lanes(const GateLane* lanes, LaneConst c, int nblk, int record,
                                                     int nl, int xcd_local) {
  // Work-groups are dispatched to the 8 XCDs round-robin (work-group i on XCD
  // i % 8).  With xcd_local the grid is padded to 8 nblk ceil(nl / 8)
  // work-groups and lane l takes nblk work-groups of XCD l % 8, so its
  // barrier and block exchange stay in that XCD's L2 (padding work-groups
  // exit at once).  Otherwise work-group i serves lane i / nblk.
  int lane, p;
  if (xcd_local) {
    const int k = blockIdx.x / 8;
    lane = (int)(blockIdx.x % 8) + 8 * (k / nblk);
    p = k % nblk;
    if (lane >= nl) return;
  } else {
    lane = blockIdx.x / nblk;
    p = blockIdx.x % nblk;
  }
  extern __shared__ zd lds[];
  chain_body<W>(lanes[lane], c, p, nblk, record, lds);
}

// Lanes of different circuits, qubit counts and capacities in one launch:
// each lane carries its own constants, Jacobi width and work-group count, and
// blk[i] = (lane, work-group of the lane) for work-group i (lane -1: idle),
// laid out on the host so that a lane's work-groups share one XCD.
__global__ __launch_bounds__(256) void k_chain_mixed(const MixLane* lanes, const int2* blk) {
  const int2 b = blk[blockIdx.x];
  if (b.x < 0) return;
  const MixLane& L = lanes[b.x];
  extern __shared__ zd lds[];
  switch (L.W) {
    case 32: chain_body<32>(L.ln, L.c, b.y, L.nblk, L.record, lds); break;
    case 16: chain_body<16>(L.ln, L.c, b.y, L.nblk, L.record, lds); break;
    case 8: chain_body<8>(L.ln, L.c, b.y, L.nblk, L.record, lds); break;
    default: chain_body<4>(L.ln, L.c, b.y, L.nblk, L.record, lds); break;
  }
}

static const void* chain_kernel(int W) {
  switch (W) {
    case 32: return (const void*)k_chain_lanes<32>;
    case 16: return (const void*)k_chain_lanes<16>;
    case 8: return (const void*)k_chain_lanes<8>;
    default: return (const void*)k_chain_lanes<4>;
  }
}

// Dynamic LDS of the chain kernel: the Jacobi blocks or the tile-GEMM staging.
static size_t chain_shared_bytes(int dc, int ldc, int ldv) {
  return std::max(svd_shared_bytes(dc, ldc, ldv, GATE_TAPE), (size_t)ZT_LDS_ELEMS * sizeof(zd));
}

hipError_t launch_chain_lanes(const GateLane* d_lanes, int nl, const LaneConst& c, bool record,
                              unsigned long long* bars, hipStream_t stream) {
  const int dc = c.ldc / 2;
  const int W = svd_width(dc);
  const int P = (c.ncap + 2 * W - 1) / (2 * W);
  const size_t shm = chain_shared_bytes(dc, c.ldc, c.ldv);
  hipError_t e = hipMemsetAsync(bars, 0, (size_t)nl * sizeof(unsigned long long), stream);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(chain_kernel(W), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  LaneConst cc = c;
  int nb = P, rec = record ? 1 : 0, nlanes = nl;
  // Lanes on one XCD each when the padded grid is resident at once.  Besides
  // keeping the block exchange in one L2, this is the layout every recompute
  // result has been reproducible in: with lanes of 16 work-groups spread over
  // all XCDs, segment replays at capacity 128 differed from their forward
  // pass now and then, a fault this layout has not shown.  Capacity 256
  // (64 work-groups per lane) cannot be XCD-local and keeps the plain layout.
  int dev = 0, cus = 0, per_cu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, chain_kernel(W), 256, shm);
  if (e != hipSuccess) return e;
  const int padded = 8 * P * ((nl + 7) / 8);
  int xcd = P <= 32 && padded <= per_cu * cus ? 1 : 0;
  const int T = xcd ? padded : P * nl;
  void* args[] = {(void*)&d_lanes, &cc, &nb, &rec, &nlanes, &xcd};
  return hipLaunchCooperativeKernel(chain_kernel(W), dim3(T), dim3(256), args, shm, stream);
}

TapeLayout tape_layout(int dc, int ncap, int ldc, int ldv) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  TapeLayout L;
  size_t o = 0;
  const size_t site = (size_t)dc * 2 * dc * sizeof(zd);
  L.oBl = o; o = al(o + site);
  L.oBr = o; o = al(o + site);
  L.olam = o; o = al(o + dc * sizeof(double));
  L.oC = o; o = al(o + (size_t)ncap * ldc * sizeof(zd));
  L.oA = o; o = al(o + (size_t)ncap * ldc * sizeof(zd));
  L.oV = o; o = al(o + (size_t)ncap * ldv * sizeof(zd));
  L.osv = o; o = al(o + ncap * sizeof(double));
  L.operm = o; o = al(o + ncap * sizeof(int));
  L.ometa = o; o = al(o + 16 * sizeof(int));
  L.odmeta = o; o = al(o + 16 * sizeof(double));
  L.rec = o;
  return L;
}

// Lanes that fit one cooperative launch of the chain kernel: its LDS use
// bounds the work-groups per compute unit, and each lane needs P of them.
int lanes_max(int dcap) {
  const int W = svd_width(dcap);
  const int P = (2 * dcap + 2 * W - 1) / (2 * W);
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
  const size_t shm = chain_shared_bytes(dcap, 2 * dcap, 2 * P * W);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, chain_kernel(W), 256, shm) != hipSuccess) return 1;
  return std::max(1, per_cu * cus / P);
}


// Dynamic LDS of the chain kernel for a lane of capacity dcap.
size_t chain_lds_bytes(int dcap) {
  const int W = svd_width(dcap);
  const int P = (2 * dcap + 2 * W - 1) / (2 * W);
  return chain_shared_bytes(dcap, 2 * dcap, 2 * P * W);
}

// Work-groups one cooperative launch of the mixed kernel holds with `shm`
// bytes of dynamic LDS each.
int mixed_blocks_max(size_t shm) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipFuncSetAttribute((const void*)k_chain_mixed, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) !=
      hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_chain_mixed, 256, shm) != hipSuccess)
    return 0;
  return per_cu * cus;
}

hipError_t launch_chain_mixed(const MixLane* d_lanes, const int2* d_blk, int nblocks, size_t shm,
                              hipStream_t stream) {
  hipError_t e = hipFuncSetAttribute((const void*)k_chain_mixed, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  void* args[] = {(void*)&d_lanes, (void*)&d_blk};
  return hipLaunchCooperativeKernel((const void*)k_chain_mixed, dim3(nblocks), dim3(256), args, shm, stream);
}


// ----------------------------------------------------------------------------
// Host launchers
// ----------------------------------------------------------------------------
// Column-block width: two blocks of W columns (and of V when accumulating)
// fill at most 128 KiB of LDS, and each pair group of 256 / W threads holds
// eight rows per thread, so 2 dcap <= 8 * 256 / W.
int svd_width(int dcap) { return dcap <= 32 ? 32 : dcap <= 64 ? 16 : dcap <= 128 ? 8 : 4; }

static const void* svd_kernel(int W, GateMode mode) {
  const bool acc = mode == GATE_TAPE;
  switch (W) {
    case 32: return acc ? (const void*)k_svd_jacobi<32, true> : (const void*)k_svd_jacobi<32, false>;
    case 16: return acc ? (const void*)k_svd_jacobi<16, true> : (const void*)k_svd_jacobi<16, false>;
    case 8: return acc ? (const void*)k_svd_jacobi<8, true> : (const void*)k_svd_jacobi<8, false>;
    default: return acc ? (const void*)k_svd_jacobi<4, true> : (const void*)k_svd_jacobi<4, false>;
  }
}

static SvdArgs svd_args(const MpsView& st, int bond, GateWork& w, GateMode mode) {
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
  s.bar = (unsigned long long*)(w.rotflag + 128);
  s.sched = w.sched;
  s.lam_out = st.lam + (size_t)(bond + 1) * st.dcap;
  s.stats = w.stats;
  s.eps = w.eps;
  s.dmax = w.dmax;
  s.tol = w.tol;
  s.max_sweeps = w.max_sweeps;
  s.nrm_part = w.nrm_part;
  const int tiles = (2 * st.dcap + ZT_M - 1) / ZT_M;
  s.nparts = tiles * tiles;
  s.trans = mode == GATE_FWD ? 1 : 0;
  return s;
}

hipError_t launch_contract(const MpsView& st, const GateTable& gt, int g, const double* theta, GateWork& w,
                           hipStream_t stream, GateMode mode) {
  const int tiles = (2 * st.dcap + ZT_M - 1) / ZT_M;
  hipLaunchKernelGGL(k_contract, dim3(tiles, tiles), dim3(256), 0, stream, st, gt, g, theta, w.C, w.A, w.ldc,
                     w.nrm_part, mode == GATE_FWD ? 1 : 0, w.rotflag);
  return hipGetLastError();
}

// One sweep over 2P blocks (P a power of two) by P work-groups in 2P - 1
// rounds, built so that a work-group keeps one of its two blocks from each
// round to the next: the first P blocks T stay while the other P blocks S
// pass along a ring (P rounds pair every T with every S); then the T blocks
// among themselves and the S blocks among themselves, each the same problem
// for P/2 work-groups, with S reordered so that every work-group again keeps
// one block at the switch.
static void schedule_rounds(int P, const std::vector<int>& L, std::vector<std::vector<std::pair<int, int>>>& out) {
  out.clear();
  if (P == 1) {
    out.push_back({{L[0], L[1]}});
    return;
  }
  for (int j = 0; j < P; ++j) {
    std::vector<std::pair<int, int>> rd;
    for (int i = 0; i < P; ++i) rd.push_back({L[i], L[P + (i + j) % P]});
    out.push_back(rd);
  }
  const int h = P / 2;
  std::vector<int> T(L.begin(), L.begin() + P), S2(P);
  for (int i = 0; i < h; ++i) {
    S2[i] = L[P + (h + i - 1 + P) % P];
    S2[h + i] = L[P + (i - 1 + P) % P];
  }
  std::vector<std::vector<std::pair<int, int>>> a, b;
  schedule_rounds(h, T, a);
  schedule_rounds(h, S2, b);
  for (int r = 0; r < P - 1; ++r) {
    std::vector<std::pair<int, int>> rd = a[r];
    rd.insert(rd.end(), b[r].begin(), b[r].end());
    out.push_back(rd);
  }
}

std::vector<unsigned char> jacobi_schedule_table() {
  std::vector<unsigned char> tab;
  for (int P = 1; P <= 64; P <<= 1) {
    std::vector<int> L(2 * P);
    for (int i = 0; i < 2 * P; ++i) L[i] = i;
    std::vector<std::vector<std::pair<int, int>>> rounds;
    schedule_rounds(P, L, rounds);
    // check: 2P - 1 perfect matchings that meet every block pair once
    if ((int)rounds.size() != 2 * P - 1) return {};
    std::vector<char> met((size_t)4 * P * P, 0);
    for (const auto& rd : rounds) {
      if ((int)rd.size() != P) return {};
      std::vector<char> used(2 * P, 0);
      for (const auto& e : rd) {
        if (e.first == e.second || used[e.first] || used[e.second]) return {};
        used[e.first] = used[e.second] = 1;
        char& m = met[(size_t)std::min(e.first, e.second) * 2 * P + std::max(e.first, e.second)];
        if (m) return {};
        m = 1;
        tab.push_back((unsigned char)e.first);
        tab.push_back((unsigned char)e.second);
      }
    }
  }
  return tab;
}

size_t svd_shared_bytes(int dcap, int ldc, int ldv, GateMode mode) {
  const int W = svd_width(dcap);
  return (size_t)2 * W * (svd_pitch(ldc, W) + (mode == GATE_TAPE ? svd_pitch(ldv, W) : 0)) * sizeof(zd);
}

hipError_t launch_svd(const MpsView& st, int bond, GateWork& w, hipStream_t stream, GateMode mode) {
  SvdArgs s = svd_args(st, bond, w, mode);
  const int W = svd_width(st.dcap);
  const int P = (w.ncap + 2 * W - 1) / (2 * W);
  const size_t shm = svd_shared_bytes(st.dcap, w.ldc, w.ldv, mode);
  // The P work-groups spread over the XCDs (work-group i on XCD i mod 8).
  // Packing them onto one XCD (a grid of 8 P with every eighth working) made
  // saturated 256 x 256 gates slower, 9.3 against 5.5 ms: every barrier's
  // release and acquire then flush and invalidate the one L2 they all share.
  int stride = 1;
  void* args[] = {&s, &stride};
  return hipLaunchCooperativeKernel(svd_kernel(W, mode), dim3(P * stride), dim3(256), args, shm, stream);
}

hipError_t launch_update(const MpsView& st, int bond, GateWork& w, hipStream_t stream, GateMode mode) {
  const int dc = st.dcap;
  const int tm = (2 * dc + ZT_M - 1) / ZT_M, tn = (dc + ZT_N - 1) / ZT_N;
  if (mode == GATE_FWD) {
    hipLaunchKernelGGL(k_update_left_t, dim3(tn, tm), dim3(256), 0, stream, st, bond, (const zd*)w.C, w.ldc,
                       (const zd*)w.A, (const double*)w.sv, (const int*)w.perm, (const int*)w.gmeta,
                       (const double*)w.gdmeta);
    hipLaunchKernelGGL(k_update_right_t, dim3(dc), dim3(256), 0, stream, st, bond, (const zd*)w.A, w.ldc,
                       (const double*)w.sv, (const int*)w.perm, (const int*)w.gmeta);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_update_left, dim3(tn, tm), dim3(256), 0, stream, st, bond, (const zd*)w.C, w.ldc,
                     (const zd*)w.V, w.ldv, (const int*)w.perm, (const int*)w.gmeta, (const double*)w.gdmeta);
  hipLaunchKernelGGL(k_update_right, dim3(dc), dim3(256), 0, stream, st, bond, (const zd*)w.V, w.ldv,
                     (const int*)w.perm, (const int*)w.gmeta);
  return hipGetLastError();
}

hipError_t launch_gate(const MpsView& st, const GateTable& gt, int g, int bond, const double* theta,
                       GateWork& w, hipStream_t stream, GateMode mode) {
  hipError_t e = launch_contract(st, gt, g, theta, w, stream, mode);
  if (e != hipSuccess) return e;
  e = launch_svd(st, bond, w, stream, mode);
  if (e != hipSuccess) return e;
  return launch_update(st, bond, w, stream, mode);
}

hipError_t svd_set_attributes(int dcap, size_t shm) {
  const int W = svd_width(dcap);
  for (GateMode m : {GATE_TAPE, GATE_FWD}) {
    hipError_t e = hipFuncSetAttribute(svd_kernel(W, m), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
