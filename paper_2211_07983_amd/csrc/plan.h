// Host-side objects behind the opaque ABI handles.
#pragma once

#include <string>
#include <vector>

#include "../../include/mpsvqe.h"
#include "engine.h"

// Owning device allocation that grows on demand.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf();
  void release();
  void* ensure(size_t n);
};

struct DevCircuit {
  int G = 0;
  GateTable tab{};
  std::vector<int> bond_h, kind_h, param_h;
  std::vector<double> coeff_h;
  uint64_t hash = 0;   // of the uploaded gate table
  DevBuf d_bond, d_kind, d_pre, d_post, d_param, d_coeff;
  void upload_from(const mps_circuit* c, hipStream_t s);
};

struct SiteList {
  size_t job_off = 0, fin_off = 0;
  int njobs = 0, nfin = 0;
};

struct Chunk {
  int lo = 0, hi = -1;
  std::vector<SiteList> sites;
};

struct DevHamiltonian {
  int64_t K = 0;
  double c0 = 0.0;
  int N_ = 0;
  int chunk = 1;
  std::vector<int> a_t, b_t;
  std::vector<uint64_t> xs, zs;
  std::vector<double> coeff_h;
  std::vector<int64_t> order;
  std::vector<Chunk> chunks;
  DevBuf d_coeff, d_jobs, d_fin_slot, d_fin_term;
  const double* d_coeff_ptr = nullptr;
  const SweepJob* d_jobs_ptr = nullptr;
  const int* d_fin_slot_ptr = nullptr;
  const int* d_fin_term_ptr = nullptr;
  void upload_from(const mps_paulisum* h, int N, int dcap, hipStream_t s, size_t budget);
};

struct mps_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  size_t sweep_budget = (size_t)6 << 30;   // bytes for per-term environments
  int last_degen_grad = 0;
  int prof_every = 0;                      // sample every k-th SVD launch (0 = off)
  mps_progress_fn progress = nullptr;      // per-segment progress report (nullable)
  void* progress_user = nullptr;
  std::vector<hipEvent_t> prof_ev;         // [2 * samples]
  std::vector<int> prof_n;                 // samples taken in the current call
  DevBuf b_prof;                           // [max samples][4] ints: rows, cols, sweeps
  GateWork gw{};
  SweepBuffers sb{};
  DevBuf b_C, b_A, b_V, b_sv, b_perm, b_gmeta, b_gdmeta, b_rot, b_nrm, b_stats, b_stats2, b_theta;
  DevBuf b_sched;   // Jacobi block schedules
  DevBuf b_Lid, b_Rid, b_Lslots, b_Y, b_Yid, b_energy, b_termval;
  DevBuf b_B32, b_Lid32, b_Rid32, b_Lslots32, b_Y32, b_Yid32;   // precision 1 sweep
  Sweep32 s32{};
  ~mps_ctx();
  void set_device();
  void ensure_gate_work(int dcap, const mps_trunc& tr, int max_sweeps);
  void ensure_sweep(int N, int dcap, int chunk, int precision = 0);
  void reset_stats();
};

struct mps_state {
  mps_ctx* ctx = nullptr;
  int N = 0;
  int dcap = 0;
  mps_trunc trunc{};
  DevBuf B, dims, lam, occ;
};

// A plan: the working state, the circuit, the Hamiltonian, the checkpoints of
// the last forward pass and the buffers of the reverse pass.
struct mps_plan {
  mps_ctx* ctx = nullptr;
  int N = 0;
  int n_theta = 0;
  mps_trunc trunc{};
  mps_grad_opts opts{256, 0.0, 64, 0};
  std::vector<uint8_t> occ_h;
  mps_state* state = nullptr;      // working state
  std::vector<mps_state*> replays; // one state per lane of the batched segment recompute
  std::vector<GateLane> lanes_h;   // host copy of the lane table
  DevBuf lanes_dev;                // device lane table
  DevBuf lane_aux;                 // per-lane counters, partial sums, stats, barrier words
  DevBuf adjl_dev;                 // adjoint lane records of the current batch
  DevBuf meta_dev;                 // gathered gate sizes of the current batch
  DevCircuit C;
  DevCircuit Cinv;                 // the circuit's inverse (Algorithm 1's reverse walk)
  bool cinv_built = false;
  DevBuf alg1_work, alg1_op, alg1_dq;   // overlap workspace, eta and dE/dphi, derivative operators
  DevBuf alg1_terms, alg1_cws;          // string masks and weights, compression workspace
  DevHamiltonian H;
  DevBuf theta, grad, gphi;
  DevBuf ckpt;                     // [n_seg][B | dims | lam] snapshots
  size_t ckpt_stride = 0;
  int n_seg = 0;
  double E = 0.0, Z = 1.0, Eim = 0.0;
  // reverse pass
  DevBuf Bbar, lambar;             // cotangents of the site tensors and Schmidt vectors
  DevBuf tape;                     // per-gate records of the segments recomputed together
  DevBuf work;                     // per-gate adjoint workspace
  DevBuf sweep_work;               // sweep-adjoint buffers
  void* adj = nullptr;             // reverse-pass state (adjoint.hip)
  ~mps_plan();
};
