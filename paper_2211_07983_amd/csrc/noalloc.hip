// Allocation-free variant of mps_apply_circuit for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  Every buffer beyond the caller's state,
// the gate workspace, the circuit (in chunks), theta, the statistics and the
// Jacobi block schedules, lives in one file-scope device array, `scratch`,
// of kScratchBytes bytes.  Each device holds its own copy of the array until
// the process ends; its address on a device is taken once, with that device
// current, by noalloc_device_init (called from mps_ctx_create) and used for
// every kernel argument and copy.  All calls on one device share the array
// and it keeps the last call's contents: calls that overlap on one device
// (other threads, other streams) race.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mpsvqe.h"
#include "engine.h"
#include "errors.h"
#include "plan.h"
#include "plan_impl.h"

namespace {

// Limits of the allocation-free path.
constexpr int kMaxDcap = 128;          // bond capacity (d_max <= 128)
constexpr int kGateChunk = 1024;       // gates uploaded per chunk
constexpr int kMaxTheta = 8192;        // parameters
constexpr size_t kSchedBytes = 32768;  // Jacobi block schedules for P = 1 .. 64

constexpr size_t al256(size_t x) { return (x + 255) / 256 * 256; }

// Byte offsets inside the scratch array (all 256-byte aligned).
struct Layout {
  size_t C, A, sv, perm, gmeta, gdmeta, rot, nrm, stats, sched, theta, bond, kind, param, coeff, pre, post, total;
};

constexpr Layout make_layout() {
  const size_t ldc = 2 * kMaxDcap;
  const size_t ncap = 2 * kMaxDcap;   // 2 P W >= 2 dcap for every width at dcap <= 128
  Layout L{};
  size_t o = 0;
  L.C = o; o = al256(o + ncap * ldc * sizeof(zd));
  L.A = o; o = al256(o + ncap * ldc * sizeof(zd));
  L.sv = o; o = al256(o + ncap * sizeof(double));
  L.perm = o; o = al256(o + ncap * sizeof(int));
  L.gmeta = o; o = al256(o + 16 * sizeof(int));
  L.gdmeta = o; o = al256(o + 16 * sizeof(double));
  L.rot = o; o = al256(o + 128 * sizeof(int) + 64);   // sweep flags, then the SVD barrier counter
  L.nrm = o; o = al256(o + 256 * sizeof(double));
  L.stats = o; o = al256(o + sizeof(GateStats));
  L.sched = o; o = al256(o + kSchedBytes);
  L.theta = o; o = al256(o + kMaxTheta * sizeof(double));
  L.bond = o; o = al256(o + kGateChunk * sizeof(int));
  L.kind = o; o = al256(o + kGateChunk * sizeof(int));
  L.param = o; o = al256(o + kGateChunk * sizeof(int));
  L.coeff = o; o = al256(o + kGateChunk * sizeof(double));
  L.pre = o; o = al256(o + (size_t)kGateChunk * 16 * sizeof(zd));
  L.post = o; o = al256(o + (size_t)kGateChunk * 16 * sizeof(zd));
  L.total = o;
  return L;
}

constexpr Layout kLayout = make_layout();
constexpr size_t kScratchBytes = kLayout.total;   // about 2.7 MiB

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` per device (nullptr: not set up)
std::mutex g_scratch_mu;

__global__ void k_zero_words(unsigned long long* p, int words) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) p[i] = 0ull;
}

}  // namespace

// The array itself.  In host code this name is a host-side stand-in, not a
// device address: only the per-device pointers in g_scratch are used.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Takes the array's address on `device` (which must be current) and uploads
// the Jacobi block schedules into it, once per device.
void noalloc_device_init(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return;
  const std::vector<unsigned char> tab = jacobi_schedule_table();
  if (tab.empty() || tab.size() > kSchedBytes) return;
  if (hipMemcpy((char*)ptr + kLayout.sched, tab.data(), tab.size(), hipMemcpyHostToDevice) != hipSuccess) return;
  g_scratch[device] = ptr;
}

static void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch[device];
}

extern "C" mps_status mps_apply_circuit_noalloc(mps_state* st, const mps_circuit* circuit, const double* theta,
                                               int32_t n_theta, mps_stats* stats) {
  if (!st) return MPS_EINVAL;
  mps_ctx* ctx = st->ctx;
  return guarded(ctx, [&] {
    if (st->dcap > kMaxDcap)
      fail(MPS_EINVAL, "mps_apply_circuit_noalloc: bond capacity " + std::to_string(st->dcap) +
                           " exceeds the allocation-free workspace (d_max <= " + std::to_string(kMaxDcap) + ")");
    if (n_theta > kMaxTheta)
      fail(MPS_EINVAL, "mps_apply_circuit_noalloc: more than " + std::to_string(kMaxTheta) + " parameters");
    validate_theta(theta, n_theta);
    validate_circuit(circuit, st->N, n_theta);
    char* base = (char*)scratch_of(ctx->device);
    if (!base) fail(MPS_EDEVICE, "mps_apply_circuit_noalloc: the workspace of this device is not set up");
    hipStream_t s = ctx->stream;
    const int dcap = st->dcap;
    const int W = svd_width(dcap);
    const int P = (2 * dcap + 2 * W - 1) / (2 * W);
    GateWork w{};
    w.ldc = 2 * dcap;
    w.ncap = 2 * P * W;
    w.ldv = w.ncap;
    w.C = (zd*)(base + kLayout.C);
    w.A = (zd*)(base + kLayout.A);
    w.V = nullptr;   // GATE_FWD accumulates no right rotations
    w.sv = (double*)(base + kLayout.sv);
    w.perm = (int*)(base + kLayout.perm);
    w.gmeta = (int*)(base + kLayout.gmeta);
    w.gdmeta = (double*)(base + kLayout.gdmeta);
    w.rotflag = (int*)(base + kLayout.rot);
    w.nrm_part = (double*)(base + kLayout.nrm);
    w.sched = (const unsigned char*)(base + kLayout.sched);
    w.stats = (GateStats*)(base + kLayout.stats);
    w.eps = st->trunc.eps;
    w.dmax = st->trunc.d_max;
    w.max_sweeps = 64;
    w.tol = std::max(1e-15, 8.0 * std::sqrt((double)w.ldc) * 2.220446049250313e-16);
    HIPCHK(svd_set_attributes(dcap, svd_shared_bytes(dcap, w.ldc, w.ldv, GATE_TAPE)));
    // statistics start at zero (a fill kernel, not a memset node)
    const int words = (int)((sizeof(GateStats) + 7) / 8);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, (unsigned long long*)w.stats, words);
    HIPCHK(hipGetLastError());
    double* th = (double*)(base + kLayout.theta);
    if (n_theta > 0) HIPCHK(hipMemcpyAsync(th, theta, (size_t)n_theta * sizeof(double), hipMemcpyHostToDevice, s));
    MpsView v = view_of(st);
    const int G = circuit->n_gates;
    for (int g0 = 0; g0 < G; g0 += kGateChunk) {
      const int ng = std::min(kGateChunk, G - g0);
      // the copies are stream-ordered after the previous chunk's gates
      HIPCHK(hipMemcpyAsync(base + kLayout.bond, circuit->bond + g0, ng * sizeof(int), hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(base + kLayout.kind, circuit->kind + g0, ng * sizeof(int), hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(base + kLayout.pre, circuit->pre + (size_t)g0 * 32, (size_t)ng * 16 * sizeof(zd),
                            hipMemcpyHostToDevice, s));
      if (circuit->post)
        HIPCHK(hipMemcpyAsync(base + kLayout.post, circuit->post + (size_t)g0 * 32, (size_t)ng * 16 * sizeof(zd),
                              hipMemcpyHostToDevice, s));
      if (circuit->param)
        HIPCHK(hipMemcpyAsync(base + kLayout.param, circuit->param + g0, ng * sizeof(int), hipMemcpyHostToDevice, s));
      if (circuit->coeff)
        HIPCHK(hipMemcpyAsync(base + kLayout.coeff, circuit->coeff + g0, ng * sizeof(double), hipMemcpyHostToDevice,
                              s));
      GateTable tab{};
      tab.bond = (const int*)(base + kLayout.bond);
      tab.kind = (const int*)(base + kLayout.kind);
      tab.pre = (const zd*)(base + kLayout.pre);
      tab.post = (const zd*)(base + kLayout.post);
      tab.param = (const int*)(base + kLayout.param);
      tab.coeff = (const double*)(base + kLayout.coeff);
      tab.G = ng;
      for (int k = 0; k < ng; ++k) HIPCHK(launch_gate(v, tab, k, circuit->bond[g0 + k], th, w, s, GATE_FWD));
    }
    GateStats gs;
    HIPCHK(hipMemcpyAsync(&gs, w.stats, sizeof(GateStats), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (gs.barrier_timeout) fail(MPS_EDEVICE, "a work-group barrier of the Jacobi SVD timed out");
    if (gs.noconv) fail(MPS_ENOCONV, "Jacobi SVD did not converge in " + std::to_string(w.max_sweeps) + " sweeps");
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->discarded_weight_sum = gs.disc_sum;
      stats->discarded_weight_max = gs.disc_max;
      stats->gates_truncated = gs.truncated;
      stats->max_sweeps_used = gs.max_sweeps;
      stats->degenerate_cuts = gs.degenerate_cuts;
      stats->max_bond = gs.max_bond;
      stats->n_gates_applied = G;
    }
  });
}
