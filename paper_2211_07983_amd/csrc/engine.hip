// Host side of the MPS engine: contexts, states, plans and the C ABI of
// include/mpsvqe.h.  Every step of the path runs in the kernels of gate.hip,
// sweep.hip and adjoint.hip; this file allocates device memory, uploads the
// circuit and the Hamiltonian and enqueues kernels on the context's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mpsvqe.h"
#include "engine.h"
#include "errors.h"
#include "plan.h"
#include "plan_impl.h"

// ----------------------------------------------------------------------------
// device buffers
// ----------------------------------------------------------------------------
DevBuf::~DevBuf() { release(); }
void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}
void* DevBuf::ensure(size_t n) {
  if (n <= bytes && p) return p;
  release();
  if (n == 0) n = 16;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) {
    p = nullptr;
    throw Failure{MPS_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed"};
  }
  bytes = n;
  return p;
}

// ----------------------------------------------------------------------------
// context
// ----------------------------------------------------------------------------
mps_ctx::~mps_ctx() {
  for (hipEvent_t ev : prof_ev) (void)hipEventDestroy(ev);
}

void mps_ctx::set_device() { HIPCHK(hipSetDevice(device)); }

void mps_ctx::ensure_gate_work(int dcap, const mps_trunc& tr, int max_sweeps) {
  const int W = svd_width(dcap);
  const int P = (2 * dcap + 2 * W - 1) / (2 * W);
  const int ncap = 2 * P * W;
  const int ldc = 2 * dcap;
  gw.ldc = ldc;
  gw.ldv = ncap;
  gw.ncap = ncap;
  gw.C = (zd*)b_C.ensure((size_t)ncap * ldc * sizeof(zd));
  gw.A = (zd*)b_A.ensure((size_t)ncap * ldc * sizeof(zd));
  gw.V = (zd*)b_V.ensure((size_t)ncap * ncap * sizeof(zd));
  gw.sv = (double*)b_sv.ensure((size_t)ncap * sizeof(double));
  gw.perm = (int*)b_perm.ensure((size_t)ncap * sizeof(int));
  gw.gmeta = (int*)b_gmeta.ensure(16 * sizeof(int));
  gw.gdmeta = (double*)b_gdmeta.ensure(16 * sizeof(double));
  gw.rotflag = (int*)b_rot.ensure(128 * sizeof(int) + 64);   // flags, then the SVD barrier counter
  gw.nrm_part = (double*)b_nrm.ensure(256 * sizeof(double));
  if (!b_sched.p) {
    const std::vector<unsigned char> tab = jacobi_schedule_table();
    if (tab.empty()) fail(MPS_EDEVICE, "Jacobi block schedule failed its check");
    upload(b_sched, tab.data(), tab.size(), stream);
    HIPCHK(hipStreamSynchronize(stream));   // tab is released at the end of this block
  }
  gw.sched = (const unsigned char*)b_sched.p;
  gw.stats = (GateStats*)b_stats.ensure(sizeof(GateStats));
  gw.eps = tr.eps;
  gw.dmax = tr.d_max;
  gw.max_sweeps = std::min(std::max(max_sweeps, 1), 100);   // per-sweep counters: 128 slots
  gw.tol = std::max(1e-15, 8.0 * std::sqrt((double)ldc) * 2.220446049250313e-16);
  // the kernel width depends on dcap: set the LDS limit of this width's kernels
  HIPCHK(svd_set_attributes(dcap, svd_shared_bytes(dcap, ldc, ncap, GATE_TAPE)));
}

void mps_ctx::reset_stats() { HIPCHK(hipMemsetAsync(gw.stats, 0, sizeof(GateStats), stream)); }

// ----------------------------------------------------------------------------
// state helpers
// ----------------------------------------------------------------------------
MpsView view_of(mps_state* st) {
  MpsView v;
  v.B = (zd*)st->B.p;
  v.dims = (int*)st->dims.p;
  v.lam = (double*)st->lam.p;
  v.N = st->N;
  v.dcap = st->dcap;
  return v;
}

void alloc_state(mps_state* st) {
  const size_t site = (size_t)st->dcap * 2 * st->dcap;
  st->B.ensure((size_t)st->N * site * sizeof(zd));
  st->dims.ensure((size_t)(st->N + 1) * sizeof(int));
  st->lam.ensure((size_t)(st->N + 1) * st->dcap * sizeof(double));
}

void init_product(mps_state* st, const uint8_t* occ_dev) {
  hipStream_t s = st->ctx->stream;
  HIPCHK(hipMemsetAsync(st->B.p, 0, st->B.bytes, s));
  hipLaunchKernelGGL(k_init_product, dim3(st->N + 1), dim3(256), 0, s, view_of(st), occ_dev);
  HIPCHK(hipGetLastError());
}

void copy_state(mps_state* dst, mps_state* src, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(dst->B.p, src->B.p, src->B.bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(dst->dims.p, src->dims.p, src->dims.bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(dst->lam.p, src->lam.p, src->lam.bytes, hipMemcpyDeviceToDevice, s));
}

// ----------------------------------------------------------------------------
// validation and upload of circuits and Hamiltonians
// ----------------------------------------------------------------------------
void validate_circuit(const mps_circuit* c, int N, int n_theta) {
  if (!c) fail(MPS_EINVAL, "circuit is NULL");
  if (c->n_qubits != N) fail(MPS_EINVAL, "circuit n_qubits does not match the state");
  if (c->n_gates < 0) fail(MPS_EINVAL, "negative gate count");
  if (c->n_gates > 0 && (!c->bond || !c->kind || !c->pre)) fail(MPS_EINVAL, "circuit arrays are NULL");
  for (int g = 0; g < c->n_gates; ++g) {
    if (c->bond[g] < 0 || c->bond[g] > N - 2) fail(MPS_EINVAL, "gate " + std::to_string(g) + ": bond out of range");
    if (c->kind[g] != 0 && c->kind[g] != 1) fail(MPS_EINVAL, "gate " + std::to_string(g) + ": bad kind");
    if (c->kind[g] == 1) {
      if (!c->post || !c->param || !c->coeff) fail(MPS_EINVAL, "parametric gate without post/param/coeff");
      if (c->param[g] < 0 || c->param[g] >= n_theta)
        fail(MPS_EINVAL, "gate " + std::to_string(g) + ": parameter index out of range");
      if (!std::isfinite(c->coeff[g])) fail(MPS_EINVAL, "non-finite gate coefficient");
    }
    for (int k = 0; k < 32; ++k)
      if (!std::isfinite(c->pre[(size_t)g * 32 + k]) || (c->kind[g] == 1 && !std::isfinite(c->post[(size_t)g * 32 + k])))
        fail(MPS_EINVAL, "non-finite gate matrix");
  }
}

void validate_theta(const double* theta, int n_theta) {
  if (n_theta < 0 || (n_theta > 0 && !theta)) fail(MPS_EINVAL, "theta is NULL");
  for (int k = 0; k < n_theta; ++k)
    if (!std::isfinite(theta[k])) fail(MPS_EINVAL, "non-finite theta");
}

void DevCircuit::upload_from(const mps_circuit* c, hipStream_t s) {
  G = c->n_gates;
  std::vector<double> post((size_t)G * 32, 0.0);
  std::vector<int> param(G, 0);
  std::vector<double> coeff(G, 0.0);
  for (int g = 0; g < G; ++g) {
    if (c->kind[g] == 1) {
      std::memcpy(&post[(size_t)g * 32], c->post + (size_t)g * 32, 32 * sizeof(double));
      param[g] = c->param[g];
      coeff[g] = c->coeff[g];
    }
  }
  bond_h.assign(c->bond, c->bond + G);
  kind_h.assign(c->kind, c->kind + G);
  param_h = param;
  coeff_h = coeff;
  // FNV-1a over everything the gate table holds, so that plans built from the
  // same circuit can be recognised as such
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  mix(&G, sizeof(G));
  if (G > 0) {
    mix(c->bond, (size_t)G * sizeof(int32_t));
    mix(c->kind, (size_t)G * sizeof(int32_t));
    mix(c->pre, (size_t)G * 32 * sizeof(double));
    mix(post.data(), post.size() * sizeof(double));
    mix(param.data(), param.size() * sizeof(int));
    mix(coeff.data(), coeff.size() * sizeof(double));
  }
  hash = h;
  tab.bond = upload(d_bond, c->bond, G, s);
  tab.kind = upload(d_kind, c->kind, G, s);
  tab.pre = (const zd*)upload(d_pre, c->pre, (size_t)G * 32, s);
  tab.post = (const zd*)upload(d_post, post.data(), (size_t)G * 32, s);
  tab.param = upload(d_param, param.data(), G, s);
  tab.coeff = upload(d_coeff, coeff.data(), G, s);
  tab.G = G;
}

static int pauli_letter(uint64_t x, uint64_t z, int q) {
  const int xb = (x >> q) & 1, zb = (z >> q) & 1;
  return xb | (zb << 1);
}

void DevHamiltonian::upload_from(const mps_paulisum* h, int N, int dcap, hipStream_t s, size_t budget) {
  if (!h) fail(MPS_EINVAL, "Hamiltonian is NULL");
  if (h->n_qubits != N) fail(MPS_EINVAL, "Hamiltonian n_qubits does not match the state");
  if (h->n_terms < 0 || (h->n_terms > 0 && (!h->x_mask || !h->z_mask || !h->coeff)))
    fail(MPS_EINVAL, "Hamiltonian arrays are NULL");
  if (h->words != (N + 63) / 64) fail(MPS_EINVAL, "words must be ceil(n_qubits/64)");
  if (N > 64) fail(MPS_EINVAL, "more than 64 qubits are not supported");
  if (!std::isfinite(h->c0)) fail(MPS_EINVAL, "non-finite c0");
  K = h->n_terms;
  c0 = h->c0;
  order.clear();
  a_t.assign(K, 0);
  b_t.assign(K, 0);
  xs.assign(K, 0);
  zs.assign(K, 0);
  std::vector<double> coeff(K);
  const uint64_t valid = N == 64 ? ~0ull : ((1ull << N) - 1);
  for (int64_t k = 0; k < K; ++k) {
    const uint64_t x = h->x_mask[k], z = h->z_mask[k];
    if (!std::isfinite(h->coeff[k])) fail(MPS_EINVAL, "non-finite Hamiltonian coefficient");
    if (((x | z) & ~valid) != 0) fail(MPS_EINVAL, "Pauli mask beyond n_qubits");
    const uint64_t m = x | z;
    if (m == 0) fail(MPS_EINVAL, "identity string must be passed as c0");
    a_t[k] = __builtin_ctzll(m);
    b_t[k] = 63 - __builtin_clzll(m);
    xs[k] = x;
    zs[k] = z;
    coeff[k] = h->coeff[k];
  }
  d_coeff_ptr = upload(d_coeff, coeff.data(), K, s);
  coeff_h = coeff;
  // terms sorted by (first site, last site) and cut into chunks that fit the budget
  order.resize(K);
  for (int64_t k = 0; k < K; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int64_t p, int64_t q) {
    return a_t[p] != a_t[q] ? a_t[p] < a_t[q] : b_t[p] < b_t[q];
  });
  const size_t per_term = (size_t)3 * dcap * dcap * sizeof(zd);
  chunk = (int)std::max<size_t>(1, std::min<size_t>(K > 0 ? K : 1, budget / per_term));
  chunks.clear();
  std::vector<SweepJob> jobs;
  std::vector<int> fin_slot, fin_term;
  for (int64_t c0i = 0; c0i < K; c0i += chunk) {
    const int64_t c1i = std::min<int64_t>(K, c0i + chunk);
    Chunk ch;
    ch.lo = N;
    ch.hi = -1;
    for (int64_t j = c0i; j < c1i; ++j) {
      ch.lo = std::min(ch.lo, a_t[order[j]]);
      ch.hi = std::max(ch.hi, b_t[order[j]]);
    }
    for (int n = ch.lo; n <= ch.hi; ++n) {
      SiteList sl;
      sl.job_off = jobs.size();
      sl.fin_off = fin_slot.size();
      for (int64_t j = c0i; j < c1i; ++j) {
        const int64_t k = order[j];
        if (a_t[k] <= n && n <= b_t[k]) {
          SweepJob jb;
          jb.in_slot = (n == a_t[k]) ? -1 : (int)(j - c0i);
          jb.out_slot = (int)(j - c0i);
          const int let = pauli_letter(xs[k], zs[k], n);
          const int xb = let & 1, zb = let >> 1;
          jb.xb = xb;
          jb.pad = 0;
          // O[i^x, i] = i^{x z} (-1)^{z i}
          zd base = (xb && zb) ? zmk(0.0, 1.0) : zmk(1.0, 0.0);
          jb.o0 = base;
          jb.o1 = zb ? zmk(-base.x, -base.y) : base;
          jobs.push_back(jb);
        }
        if (b_t[k] == n) {
          fin_slot.push_back((int)(j - c0i));
          fin_term.push_back((int)k);
        }
      }
      sl.njobs = (int)(jobs.size() - sl.job_off);
      sl.nfin = (int)(fin_slot.size() - sl.fin_off);
      ch.sites.push_back(sl);
    }
    chunks.push_back(ch);
  }
  d_jobs_ptr = upload(d_jobs, jobs.data(), jobs.size(), s);
  d_fin_slot_ptr = upload(d_fin_slot, fin_slot.data(), fin_slot.size(), s);
  d_fin_term_ptr = upload(d_fin_term, fin_term.data(), fin_term.size(), s);
  N_ = N;
}

void mps_ctx::ensure_sweep(int N, int dcap, int chunk, int precision) {
  const size_t dd = (size_t)dcap * dcap;
  // the FP64 identity environments (and their scratch Yid) also serve the
  // gradient in either precision, and Lid holds Z
  sb.Lid = (zd*)b_Lid.ensure((N + 1) * dd * sizeof(zd));
  sb.Rid = (zd*)b_Rid.ensure((N + 1) * dd * sizeof(zd));
  sb.Yid = (zd*)b_Yid.ensure(2 * dd * sizeof(zd));
  if (precision == 0) {
    sb.Lslots = (zd*)b_Lslots.ensure((size_t)chunk * dd * sizeof(zd));
    sb.Y = (zd*)b_Y.ensure((size_t)chunk * 2 * dd * sizeof(zd));
  } else {
    s32.B = (cf*)b_B32.ensure((size_t)N * 2 * dd * sizeof(cf));
    s32.Lid = (cf*)b_Lid32.ensure((N + 1) * dd * sizeof(cf));
    s32.Rid = (cf*)b_Rid32.ensure((N + 1) * dd * sizeof(cf));
    s32.Lslots = (cf*)b_Lslots32.ensure((size_t)chunk * dd * sizeof(cf));
    s32.Y = (cf*)b_Y32.ensure((size_t)chunk * 2 * dd * sizeof(cf));
    s32.Yid = (cf*)b_Yid32.ensure(2 * dd * sizeof(cf));
  }
  sb.energy = (double*)b_energy.ensure(8 * sizeof(double));
  sb.chunk = chunk;
}

// S5 with FP32 matrix-core transfers (precision 1); Z is written where the
// FP64 energy sum reads it.
static void run_energy_f32(mps_state* st, DevHamiltonian& H) {
  mps_ctx* ctx = st->ctx;
  hipStream_t s = ctx->stream;
  MpsView v = view_of(st);
  Sweep32& s32 = ctx->s32;
  HIPCHK(hipMemsetAsync(s32.Lid, 0, ctx->b_Lid32.bytes, s));
  HIPCHK(hipMemsetAsync(s32.Rid, 0, ctx->b_Rid32.bytes, s));
  HIPCHK(launch_sites_f32(v, s32.B, s));
  HIPCHK(launch_identity_envs_f32(v, s32, s));
  for (auto& ch : H.chunks) {
    for (int n = ch.lo; n <= ch.hi; ++n) {
      const SiteList& sl = ch.sites[n - ch.lo];
      if (sl.njobs) HIPCHK(launch_transfer_f32(v, s32, n, H.d_jobs_ptr + sl.job_off, sl.njobs, s));
      if (sl.nfin)
        HIPCHK(launch_finalize_f32(v, s32, ctx->sb.termval, n, H.d_fin_slot_ptr + sl.fin_off,
                                   H.d_fin_term_ptr + sl.fin_off, sl.nfin, s));
    }
  }
  HIPCHK(launch_norm_from_f32(v, s32, ctx->sb.Lid + (size_t)st->N * st->dcap * st->dcap, s));
  HIPCHK(launch_energy_sum(v, ctx->sb, H.d_coeff_ptr, H.K, H.c0, s));
}

// FP64 identity environments of a state (the sweep adjoint's inputs).
void run_identity_envs(mps_state* st) {
  mps_ctx* ctx = st->ctx;
  hipStream_t s = ctx->stream;
  HIPCHK(hipMemsetAsync(ctx->sb.Lid, 0, ctx->b_Lid.bytes, s));
  HIPCHK(hipMemsetAsync(ctx->sb.Rid, 0, ctx->b_Rid.bytes, s));
  MpsView v = view_of(st);
  HIPCHK(launch_identity_envs(v, ctx->sb, s));
}

// Runs S5-S6 on a state: identity environments, every term, the energy sum.
void run_energy(mps_state* st, DevHamiltonian& H) {
  mps_ctx* ctx = st->ctx;
  hipStream_t s = ctx->stream;
  const int dc = st->dcap;
  ctx->ensure_sweep(st->N, dc, H.chunk, st->trunc.precision);
  ctx->sb.termval = (zd*)ctx->b_termval.ensure(std::max<int64_t>(1, H.K) * sizeof(zd));
  if (st->trunc.precision == 1) {
    run_energy_f32(st, H);
    return;
  }
  HIPCHK(hipMemsetAsync(ctx->sb.Lid, 0, ctx->b_Lid.bytes, s));
  HIPCHK(hipMemsetAsync(ctx->sb.Rid, 0, ctx->b_Rid.bytes, s));
  MpsView v = view_of(st);
  HIPCHK(launch_identity_envs(v, ctx->sb, s));
  for (auto& ch : H.chunks) {
    for (int n = ch.lo; n <= ch.hi; ++n) {
      const SiteList& sl = ch.sites[n - ch.lo];
      if (sl.njobs) HIPCHK(launch_transfer(v, ctx->sb, n, H.d_jobs_ptr + sl.job_off, sl.njobs, s));
      if (sl.nfin)
        HIPCHK(launch_finalize(v, ctx->sb, n, H.d_fin_slot_ptr + sl.fin_off, H.d_fin_term_ptr + sl.fin_off, sl.nfin, s));
    }
  }
  HIPCHK(launch_energy_sum(v, ctx->sb, H.d_coeff_ptr, H.K, H.c0, s));
}

static const int kMaxProfSamples = 8192;

void run_gates(mps_state* st, DevCircuit& C, const double* theta_dev, int g0, int g1, GateMode mode) {
  mps_ctx* ctx = st->ctx;
  MpsView v = view_of(st);
  hipStream_t s = ctx->stream;
  for (int g = g0; g < g1; ++g) {
    const int k = (int)ctx->prof_n.size();
    if (ctx->prof_every > 0 && g % ctx->prof_every == 0 && k < kMaxProfSamples) {
      if ((int)ctx->prof_ev.size() < 2 * (k + 1)) {
        hipEvent_t a, b;
        HIPCHK(hipEventCreate(&a));
        HIPCHK(hipEventCreate(&b));
        ctx->prof_ev.push_back(a);
        ctx->prof_ev.push_back(b);
      }
      int* slots = (int*)ctx->b_prof.ensure((size_t)kMaxProfSamples * 4 * sizeof(int));
      HIPCHK(launch_contract(v, C.tab, g, theta_dev, ctx->gw, s, mode));
      HIPCHK(hipEventRecord(ctx->prof_ev[2 * k], s));
      HIPCHK(launch_svd(v, C.bond_h[g], ctx->gw, s, mode));
      HIPCHK(hipEventRecord(ctx->prof_ev[2 * k + 1], s));
      HIPCHK(hipMemcpyAsync(slots + 4 * k, ctx->gw.gmeta + 8, 3 * sizeof(int), hipMemcpyDeviceToDevice, s));
      HIPCHK(launch_update(v, C.bond_h[g], ctx->gw, s, mode));
      ctx->prof_n.push_back(g);
    } else {
      HIPCHK(launch_gate(v, C.tab, g, C.bond_h[g], theta_dev, ctx->gw, s, mode));
    }
  }
}

// Sums the sampled SVD launches of this call into stats (synchronises).
static void collect_profile(mps_ctx* ctx, mps_stats* out) {
  const int k = (int)ctx->prof_n.size();
  double ms = 0.0, flop = 0.0;
  if (k > 0) {
    std::vector<int> meta((size_t)4 * k);
    HIPCHK(hipMemcpyAsync(meta.data(), ctx->b_prof.p, meta.size() * sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int q = 0; q < k; ++q) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, ctx->prof_ev[2 * q], ctx->prof_ev[2 * q + 1]));
      ms += t;
      const double p = std::min(meta[4 * q], meta[4 * q + 1]);
      flop += 84.0 * p * p * p;
    }
  }
  if (out) {
    out->prof_svd_ms = ms;
    out->prof_svd_flop = flop;
    out->prof_svd_launches = k;
  }
  ctx->prof_n.clear();
}

void read_stats(mps_ctx* ctx, mps_stats* out, int64_t gates) {
  collect_profile(ctx, out);
  GateStats gs;
  HIPCHK(hipMemcpyAsync(&gs, ctx->gw.stats, sizeof(GateStats), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (gs.barrier_timeout) fail(MPS_EDEVICE, "a work-group barrier of the Jacobi SVD timed out");
  if (gs.noconv) fail(MPS_ENOCONV, "Jacobi SVD did not converge in " + std::to_string(ctx->gw.max_sweeps) + " sweeps");
  if (out) {
    out->discarded_weight_sum = gs.disc_sum;
    out->discarded_weight_max = gs.disc_max;
    out->gates_truncated = gs.truncated;
    out->max_sweeps_used = gs.max_sweeps;
    out->degenerate_cuts = gs.degenerate_cuts;
    out->max_bond = gs.max_bond;
    out->n_gates_applied = gates;
  }
  ctx->last_degen_grad = gs.degen_grad;
}

// ----------------------------------------------------------------------------
// ABI
// ----------------------------------------------------------------------------

extern "C" {

mps_status mps_ctx_create(int32_t device, void* hip_stream, mps_ctx** out) {
  if (!out) return MPS_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MPS_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return MPS_EDEVICE;
  int coop = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess || !coop)
    return MPS_EDEVICE;
  noalloc_device_init(device);
  mps_ctx* c = new mps_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  *out = c;
  return MPS_OK;
}

void mps_ctx_destroy(mps_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
}

const char* mps_last_error(const mps_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

mps_status mps_ctx_set_progress(mps_ctx* ctx, mps_progress_fn fn, void* user) {
  if (!ctx) return MPS_EINVAL;
  ctx->progress = fn;
  ctx->progress_user = user;
  return MPS_OK;
}

mps_status mps_ctx_set_profiling(mps_ctx* ctx, int32_t every) {
  if (!ctx || every < 0) return MPS_EINVAL;
  ctx->prof_every = every;
  return MPS_OK;
}

mps_status mps_init_product(mps_ctx* ctx, int32_t n_qubits, const uint8_t* occ_bits, const mps_trunc* trunc,
                            mps_state** out) {
  if (!ctx || !out) return MPS_EINVAL;
  return guarded(ctx, [&] {
    if (n_qubits < 2 || n_qubits > 64) fail(MPS_EINVAL, "n_qubits must be in [2, 64]");
    if (!occ_bits || !trunc) fail(MPS_EINVAL, "NULL argument");
    if (trunc->d_max < 1 || trunc->d_max > 256) fail(MPS_EINVAL, "d_max must be in [1, 256]");
    if (!(trunc->eps >= 0.0) || !std::isfinite(trunc->eps)) fail(MPS_EINVAL, "eps must be finite and >= 0");
    if (trunc->precision != 0 && trunc->precision != 1) fail(MPS_EINVAL, "precision must be 0 or 1");
    for (int q = 0; q < n_qubits; ++q)
      if (occ_bits[q] > 1) fail(MPS_EINVAL, "occupation bits must be 0 or 1");
    mps_state* st = new mps_state();
    try {
      st->ctx = ctx;
      st->N = n_qubits;
      st->trunc = *trunc;
      st->dcap = std::max(2, ((trunc->d_max + 1) / 2) * 2);
      alloc_state(st);
      uint8_t* occ = upload(st->occ, occ_bits, n_qubits, ctx->stream);
      init_product(st, occ);
      HIPCHK(hipStreamSynchronize(ctx->stream));
    } catch (...) {
      delete st;
      throw;
    }
    *out = st;
  });
}

mps_status mps_apply_circuit(mps_state* st, const mps_circuit* circuit, const double* theta, int32_t n_theta,
                             mps_stats* stats) {
  if (!st) return MPS_EINVAL;
  mps_ctx* ctx = st->ctx;
  return guarded(ctx, [&] {
    validate_theta(theta, n_theta);
    validate_circuit(circuit, st->N, n_theta);
    hipStream_t s = ctx->stream;
    DevCircuit C;
    C.upload_from(circuit, s);
    const double* th = upload(ctx->b_theta, theta, (size_t)std::max(n_theta, 1), s);
    ctx->ensure_gate_work(st->dcap, st->trunc, 64);
    ctx->reset_stats();
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
    run_gates(st, C, th, 0, C.G, GATE_FWD);
    HIPCHK(hipEventRecord(e1, s));
    read_stats(ctx, stats, C.G);
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (stats) stats->t_gates_ms = ms;
  });
}

mps_status mps_expect_paulisum(mps_state* st, const mps_paulisum* h, double* energy, double* term_vals,
                               mps_stats* stats) {
  if (!st || !energy) return MPS_EINVAL;
  mps_ctx* ctx = st->ctx;
  return guarded(ctx, [&] {
    hipStream_t s = ctx->stream;
    DevHamiltonian H;
    H.upload_from(h, st->N, st->dcap, s, ctx->sweep_budget);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
    run_energy(st, H);
    HIPCHK(hipEventRecord(e1, s));
    double ev[4];
    HIPCHK(hipMemcpyAsync(ev, ctx->sb.energy, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    std::vector<zd> tv;
    if (term_vals && H.K > 0) {
      tv.resize(H.K);
      HIPCHK(hipMemcpyAsync(tv.data(), ctx->sb.termval, H.K * sizeof(zd), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *energy = ev[0];
    if (term_vals)
      for (int64_t k = 0; k < H.K; ++k) term_vals[k] = tv[k].x / ev[2];
    if (stats) {
      stats->imag_E = ev[1];
      stats->norm = ev[2];
      stats->t_sweep_ms = ms;
    }
  });
}

mps_status mps_state_export(const mps_state* st, int32_t* dims, double* B, double* lam) {
  if (!st) return MPS_EINVAL;
  mps_ctx* ctx = st->ctx;
  return guarded(ctx, [&] {
    hipStream_t s = ctx->stream;
    const int N = st->N, dc = st->dcap;
    std::vector<int> d(N + 1);
    HIPCHK(hipMemcpyAsync(d.data(), st->dims.p, (N + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
    std::vector<zd> all((size_t)N * dc * 2 * dc);
    HIPCHK(hipMemcpyAsync(all.data(), st->B.p, all.size() * sizeof(zd), hipMemcpyDeviceToHost, s));
    std::vector<double> l((size_t)(N + 1) * dc);
    HIPCHK(hipMemcpyAsync(l.data(), st->lam.p, l.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (dims) std::memcpy(dims, d.data(), (N + 1) * sizeof(int));
    if (lam) std::memcpy(lam, l.data(), l.size() * sizeof(double));
    if (B) {
      size_t o = 0;
      for (int n = 0; n < N; ++n)
        for (int al = 0; al < d[n]; ++al)
          for (int i = 0; i < 2; ++i)
            for (int be = 0; be < d[n + 1]; ++be) {
              const zd v = all[(size_t)n * dc * 2 * dc + (size_t)al * 2 * dc + i * dc + be];
              B[o++] = v.x;
              B[o++] = v.y;
            }
    }
  });
}

mps_status mps_state_import(mps_ctx* ctx, int32_t n_qubits, const mps_trunc* trunc, const int32_t* dims,
                            const double* B, const double* lam, mps_state** out) {
  if (!ctx || !out) return MPS_EINVAL;
  return guarded(ctx, [&] {
    if (n_qubits < 2 || n_qubits > 64) fail(MPS_EINVAL, "n_qubits must be in [2, 64]");
    if (!trunc || !dims || !B || !lam) fail(MPS_EINVAL, "NULL argument");
    if (trunc->d_max < 1 || trunc->d_max > 256) fail(MPS_EINVAL, "d_max must be in [1, 256]");
    if (!(trunc->eps >= 0.0) || !std::isfinite(trunc->eps)) fail(MPS_EINVAL, "eps must be finite and >= 0");
    if (trunc->precision != 0 && trunc->precision != 1) fail(MPS_EINVAL, "precision must be 0 or 1");
    const int N = n_qubits;
    if (dims[0] != 1 || dims[N] != 1) fail(MPS_EINVAL, "dims[0] and dims[n_qubits] must be 1");
    for (int k = 1; k < N; ++k)
      if (dims[k] < 1 || dims[k] > trunc->d_max) fail(MPS_EINVAL, "bond dimension outside [1, d_max]");
    size_t nb = 0, nl = 0;
    for (int n = 0; n < N; ++n) nb += (size_t)2 * dims[n] * dims[n + 1];
    for (int k = 0; k <= N; ++k) nl += (size_t)dims[k];
    for (size_t i = 0; i < 2 * nb; ++i)
      if (!std::isfinite(B[i])) fail(MPS_EINVAL, "non-finite site tensor entry");
    for (size_t i = 0; i < nl; ++i)
      if (!std::isfinite(lam[i]) || lam[i] < 0.0) fail(MPS_EINVAL, "Schmidt values must be finite and >= 0");
    mps_state* st = new mps_state();
    try {
      st->ctx = ctx;
      st->N = N;
      st->trunc = *trunc;
      st->dcap = std::max(2, ((trunc->d_max + 1) / 2) * 2);
      const int dc = st->dcap;
      alloc_state(st);
      // scatter into the capacity layout on the host, then one upload per array
      std::vector<zd> all((size_t)N * dc * 2 * dc, zmk(0.0, 0.0));
      size_t o = 0;
      for (int n = 0; n < N; ++n)
        for (int al = 0; al < dims[n]; ++al)
          for (int i = 0; i < 2; ++i)
            for (int be = 0; be < dims[n + 1]; ++be, o += 2)
              all[(size_t)n * dc * 2 * dc + (size_t)al * 2 * dc + i * dc + be] = zmk(B[o], B[o + 1]);
      std::vector<double> l((size_t)(N + 1) * dc, 0.0);
      o = 0;
      for (int k = 0; k <= N; ++k)
        for (int j = 0; j < dims[k]; ++j) l[(size_t)k * dc + j] = lam[o++];
      std::vector<int> d(dims, dims + N + 1);
      HIPCHK(hipMemcpyAsync(st->B.p, all.data(), all.size() * sizeof(zd), hipMemcpyHostToDevice, ctx->stream));
      HIPCHK(hipMemcpyAsync(st->lam.p, l.data(), l.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
      HIPCHK(hipMemcpyAsync(st->dims.p, d.data(), d.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream));
      HIPCHK(hipStreamSynchronize(ctx->stream));   // the host vectors are released at the end of this block
    } catch (...) {
      delete st;
      throw;
    }
    *out = st;
  });
}

int64_t mps_state_size(const mps_state* st) {
  if (!st) return -1;
  std::vector<int> d(st->N + 1);
  if (hipMemcpy(d.data(), st->dims.p, (st->N + 1) * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return -1;
  int64_t tot = 0;
  for (int n = 0; n < st->N; ++n) tot += 2 * 2 * (int64_t)d[n] * d[n + 1];
  return tot;
}

int32_t mps_state_qubits(const mps_state* st) { return st ? st->N : -1; }

void mps_state_free(mps_state* st) {
  if (!st) return;
  (void)hipSetDevice(st->ctx->device);
  (void)hipStreamSynchronize(st->ctx->stream);
  delete st;
}

}  // extern "C"
