// Internal declarations shared by the engine's translation units.
#pragma once
#include <vector>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

// Device copy of a compiled gate list.
struct GateTable {
  const int* bond;
  const int* kind;
  const zd* pre;     // [G][16]
  const zd* post;    // [G][16]
  const int* param;
  const double* coeff;
  int G;
};

// Accumulated per-call statistics (device).
struct GateStats {
  double disc_sum;
  double disc_max;
  double svd_flop;   // algorithmic SVD work, 84 p^3 per gate (p = min(rows, cols))
  double gemm_flop;  // gate GEMM work: 8 flops per complex MAC of the contraction, gate matrix and left update
  int truncated;
  int max_sweeps;
  int noconv;
  int degenerate_cuts;
  int max_bond;
  int gates;
  int degen_grad;    // degenerate pairs that carried a cotangent (backward)
  int barrier_timeout;  // a work-group barrier of the SVD timed out (results invalid)
};

// Workspace of one gate update.
struct GateWork {
  zd* C;          // [ncap][ldc] column-major, unweighted C
  zd* A;          // [ncap][ldc] weighted C, orthogonalised in place
  zd* V;          // [ncap][ldv]
  double* sv;     // [ncap]
  int* perm;      // [ncap]
  int* gmeta;     // [4]
  double* gdmeta; // [4]
  int* rotflag;   // [128]
  double* nrm_part; // [256] per-tile |A|^2 partial sums of k_contract
  const unsigned char* sched;   // Jacobi block schedules (jacobi_schedule_table)
  GateStats* stats;
  int ldc, ldv, ncap;
  double eps, tol;
  int dmax, max_sweeps;
};

struct SvdArgs {
  zd* A;
  int lda;
  zd* V;
  int ldv;
  int* dims;
  int bond;
  double* sv;
  int* perm;
  int* gmeta;
  double* gdmeta;
  int* rotflag;
  const unsigned char* sched;   // Jacobi block schedules (nullable: round robin only)
  unsigned long long* bar;  // work-group barrier counter (zeroed before the launch)
  double* lam_out;
  GateStats* stats;
  double eps;
  int dmax;
  double tol;
  int max_sweeps;
  const double* nrm_part;
  int nparts;
  int trans;         // 1: the matrix is C~^H (columns = rows of C~)
};

// ----------------------------------------------------------------------------
// Gate matrix Q (4x4) of gate g, evaluated on the device from theta.
// ----------------------------------------------------------------------------
// dphi is added to a PARAM gate's angle (the parameter-shift evaluations).
__device__ inline void gate_matrix(const GateTable& gt, int g, const double* theta, zd* Q, double dphi = 0.0) {
  // called by threads 0..15 of a block, Q in shared memory
  const int t = threadIdx.x;
  const zd* pre = gt.pre + (size_t)g * 16;
  if (gt.kind[g] == 0) {
    if (t < 16) Q[t] = pre[t];
    return;
  }
  const zd* post = gt.post + (size_t)g * 16;
  const double phi = gt.coeff[g] * theta[gt.param[g]] + dphi;
  double sn, cs;
  sincos(0.5 * phi, &sn, &cs);
  // RZZ diagonal: e^{-i phi/2}, e^{+i phi/2}, e^{+i phi/2}, e^{-i phi/2}
  if (t < 16) {
    const int r = t >> 2, c = t & 3;
    zd acc = zmk(0.0, 0.0);
    for (int k = 0; k < 4; ++k) {
      const double sg = (k == 0 || k == 3) ? -1.0 : 1.0;
      const zd d = zmk(cs, sg * sn);
      acc = zfma(zmul(post[r * 4 + k], d), pre[k * 4 + c], acc);
    }
    Q[t] = acc;
  }
}


// Byte offsets of one gate record of the reverse-pass tape: the gate's inputs
// (B_n, B_{n+1}, lambda_{n-1}), C, the orthogonalised A = C~ V, V, the singular
// values, their order and the sizes (meta[0] = r, meta[4..6] = a, m, b;
// dmeta[0] = nu).
struct TapeLayout {
  size_t oBl, oBr, olam, oC, oA, oV, osv, operm, ometa, odmeta, rec;
};
TapeLayout tape_layout(int dc, int ncap, int ldc, int ldv);

// One lane of a batched gate chain: gates [g0, g0 + ng) applied to the lane's
// own state with the lane's parameters: a segment recompute (one tape record
// per gate) or a whole forward pass (one reused record).
struct GateLane {
  MpsView st;
  int g0, ng;
  int rec_stride;     // tape records per step (0: every step reuses record 0)
  const double* theta;
  char* ckpt;         // chain launches: the state before the first gate is copied here (nullable)
  char* tape;
  GateStats* stats;
  int* rotflag;       // [128] Jacobi sweep counters
  double* nrm_part;   // [256] |C~|^2 partial sums
  unsigned long long* bar;   // lane barrier counter
  int* err;           // set when a lane barrier timed out
  int shift_gate;     // gate whose angle is shifted by `shift` (-1: none)
  double shift;
};

// Launch constants shared by all lanes.
struct LaneConst {
  const unsigned char* sched;   // Jacobi block schedules (jacobi_schedule_table)
  GateTable gt;
  TapeLayout L;
  int ldc, ldv, ncap, dmax, max_sweeps, nparts;
  double eps, tol;
  size_t ck_B, ck_dims, ck_lam;   // byte sizes of a checkpoint's parts (B, dims, lambda)
};
int lanes_max(int dcap);

// All ng gates of every lane in one cooperative launch: per gate the lane's
// work-groups share the contraction tiles, run the Jacobi SVD and share the
// site update, separated by the lane's barrier, so each lane advances at its
// own pace.  record: write the tape inputs; the barrier words bars[nl] are
// zeroed here before the launch.
hipError_t launch_chain_lanes(const GateLane* d_lanes, int nl, const LaneConst& c, bool record,
                              unsigned long long* bars, hipStream_t stream);

// A lane of a mixed launch: its own constants (circuit, tape layout,
// capacities, truncation), Jacobi width W (svd_width of its capacity) and
// work-group count nblk; record: write the tape of this launch's gates.
struct MixLane {
  GateLane ln;
  LaneConst c;
  int W, nblk, record, pad;
};
// Dynamic LDS of a lane of capacity dcap; work-groups that one cooperative
// launch of the mixed kernel holds with shm bytes each (0 on error).
size_t chain_lds_bytes(int dcap);
int mixed_blocks_max(size_t shm);
// One cooperative launch of every lane in d_lanes: d_blk[i] = (lane, work-
// group of that lane) for work-group i < nblocks, lane -1 for an idle one.
// The lanes' barrier words must be zero.
hipError_t launch_chain_mixed(const MixLane* d_lanes, const int2* d_blk, int nblocks, size_t shm,
                              hipStream_t stream);

// GATE_TAPE: Jacobi on C~ with the right rotations accumulated in V (the full
// decomposition the reverse pass needs).  GATE_FWD: Jacobi on C~^H without
// accumulation; the normalised columns are the right singular vectors.
enum GateMode { GATE_TAPE = 0, GATE_FWD = 1 };

int svd_width(int dcap);
hipError_t launch_gate(const MpsView& st, const GateTable& gt, int g, int bond, const double* theta,
                       GateWork& w, hipStream_t stream, GateMode mode = GATE_TAPE);
hipError_t launch_contract(const MpsView& st, const GateTable& gt, int g, const double* theta, GateWork& w,
                           hipStream_t stream, GateMode mode = GATE_TAPE);
hipError_t launch_svd(const MpsView& st, int bond, GateWork& w, hipStream_t stream, GateMode mode = GATE_TAPE);
hipError_t launch_update(const MpsView& st, int bond, GateWork& w, hipStream_t stream, GateMode mode = GATE_TAPE);
size_t svd_shared_bytes(int dcap, int ldc, int ldv, GateMode mode);
// Block-pair schedules of one Jacobi sweep for P = 1, 2, 4, ..., 64 work-groups
// ([P index][round][work-group][2] block ids, concatenated); empty if the
// construction fails its own check.
std::vector<unsigned char> jacobi_schedule_table();
hipError_t svd_set_attributes(int dcap, size_t shm);

// ----------------------------------------------------------------------------
// Pauli sweeps
// ----------------------------------------------------------------------------
// One transfer job at a site: L_out = sum_i o_i (B^{i^x})^dagger L_in B^i.
struct SweepJob {
  int in_slot;    // -1: start from the identity environment of this site
  int out_slot;
  int xb;         // bit flip of the site operator
  int pad;
  zd o0, o1;      // O[i^x, i] = o_i
};

struct SweepBuffers {
  zd* Lid;        // [N+1][dcap][dcap] identity left environments
  zd* Rid;        // [N+1][dcap][dcap] identity right environments
  zd* Lslots;     // [chunk][dcap][dcap]
  zd* Y;          // [chunk][dcap][2 dcap] stage-1 products
  zd* Yid;        // [2 dcap][dcap] scratch for identity environments
  zd* termval;    // [K] unnormalised <P_k>
  double* energy; // [4]: E, Im E, Z, c0 sum
  int chunk;
};

// FP32 copies used by the matrix-core sweep (precision 1); same layouts.
typedef float2 cf;  // complex float, (x, y) = (re, im)
struct Sweep32 {
  cf* B;          // [N][dcap][2][dcap] FP32 copies of the sites
  cf* Lid;        // [N+1][dcap][dcap]
  cf* Rid;        // [N+1][dcap][dcap]
  cf* Lslots;     // [chunk][dcap][dcap]
  cf* Y;          // [chunk][dcap][2 dcap]
  cf* Yid;        // [2 dcap][dcap]
};

hipError_t launch_identity_envs(const MpsView& st, SweepBuffers& sb, hipStream_t stream);
hipError_t launch_transfer(const MpsView& st, SweepBuffers& sb, int n, const SweepJob* jobs, int njobs,
                           hipStream_t stream);
hipError_t launch_finalize(const MpsView& st, SweepBuffers& sb, int n, const int* slots, const int* terms,
                           int nfin, hipStream_t stream);
hipError_t launch_energy_sum(const MpsView& st, SweepBuffers& sb, const double* coeff, int64_t K, double c0,
                             hipStream_t stream);

// One environment-transfer job of the sweep adjoint with FP32 buffers
// (precision 1): the FP64 job's fields with its pointers moved to the FP32
// copies of the same buffers.
struct EnvJob32 {
  const cf* in;   // input environment
  cf* out;        // output environment
  cf* y;          // stage-1 buffer ([dc][2 dc])
  const cf* rr;   // right environment of the contribution
  cf* g;          // contribution buffer ([dc][2 dc])
  double c;       // term coefficient
  int xb;         // bit flip of the site operator
  int acc;        // stage 2 accumulates into out
  zd o0, o1;      // O[i^x, i] = o_i
};
struct InjectItem32 {
  const cf* src;
  double c;
  double pad;
};
hipError_t launch_env32_right(const EnvJob32* jobs, int nj, const cf* B, int a, int b, int dc, hipStream_t s);
hipError_t launch_env32_left(const EnvJob32* jobs, int nj, const cf* B, zd* Bbar, int a, int b, int dc,
                             hipStream_t s);
hipError_t launch_inject32(const InjectItem32* items, int ni, zd* dst, int d, int dc, hipStream_t s);

hipError_t launch_sites_f32(const MpsView& st, cf* B32, hipStream_t stream);
hipError_t launch_identity_envs_f32(const MpsView& st, Sweep32& s, hipStream_t stream);
hipError_t launch_transfer_f32(const MpsView& st, Sweep32& s, int n, const SweepJob* jobs, int njobs,
                               hipStream_t stream);
hipError_t launch_finalize_f32(const MpsView& st, Sweep32& s, zd* termval, int n, const int* slots,
                               const int* terms, int nfin, hipStream_t stream);
hipError_t launch_norm_from_f32(const MpsView& st, Sweep32& s, zd* dst, hipStream_t stream);

__global__ void k_init_product(MpsView st, const uint8_t* occ);
