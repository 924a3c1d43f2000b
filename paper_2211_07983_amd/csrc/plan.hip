// Plans: a device copy of (product state, circuit, Hamiltonian, options) that
// evaluates E(theta) and dE/dtheta (arXiv:2211.07983, Sec. 4: the loss as the
// composition of the circuit evolution f(theta) and the expectation E(psi)).
// The forward pass saves the whole MPS every ckpt_gates gates so that the
// reverse pass can recompute one segment at a time.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mpsvqe.h"
#include "engine.h"
#include "plan_impl.h"

void plan_adj_free(void* a);

mps_plan::~mps_plan() {
  delete state;
  for (mps_state* r : replays) delete r;
  plan_adj_free(adj);
}

mps_state* plan_new_state(mps_ctx* ctx, int N, const mps_trunc& tr, const uint8_t* occ) {
  mps_state* st = new mps_state();
  try {
    st->ctx = ctx;
    st->N = N;
    st->trunc = tr;
    st->dcap = std::max(2, ((tr.d_max + 1) / 2) * 2);
    alloc_state(st);
    if (occ) upload(st->occ, occ, N, ctx->stream);
  } catch (...) {
    delete st;
    throw;
  }
  return st;
}

static void snapshot(mps_plan* p, int seg, bool save) {
  mps_state* st = p->state;
  char* base = (char*)p->ckpt.p + (size_t)seg * p->ckpt_stride;
  const size_t bB = st->B.bytes, bd = st->dims.bytes, bl = st->lam.bytes;
  hipStream_t s = p->ctx->stream;
  if (save) {
    HIPCHK(hipMemcpyAsync(base, st->B.p, bB, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(base + bB, st->dims.p, bd, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(base + bB + bd, st->lam.p, bl, hipMemcpyDeviceToDevice, s));
  }
}

void plan_restore(mps_plan* p, int seg, mps_state* dst) {
  mps_state* st = p->state;
  char* base = (char*)p->ckpt.p + (size_t)seg * p->ckpt_stride;
  const size_t bB = st->B.bytes, bd = st->dims.bytes, bl = st->lam.bytes;
  hipStream_t s = p->ctx->stream;
  HIPCHK(hipMemcpyAsync(dst->B.p, base, bB, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(dst->dims.p, base + bB, bd, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(dst->lam.p, base + bB + bd, bl, hipMemcpyDeviceToDevice, s));
}

void plan_forward_energy(mps_plan* p, const double* theta, int n_theta, int on_device, double* energy,
                         mps_stats* stats, bool keep_checkpoints) {
  mps_ctx* ctx = p->ctx;
  hipStream_t s = ctx->stream;
  if (n_theta != p->n_theta) fail(MPS_EINVAL, "n_theta does not match the circuit");
  double* th = (double*)p->theta.ensure((size_t)std::max(1, n_theta) * sizeof(double));
  if (n_theta > 0) {
    std::vector<double> host(n_theta);
    if (on_device) {
      HIPCHK(hipMemcpyAsync(th, theta, n_theta * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(host.data(), th, n_theta * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    } else {
      std::memcpy(host.data(), theta, n_theta * sizeof(double));
    }
    validate_theta(host.data(), n_theta);
    if (!on_device) HIPCHK(hipMemcpyAsync(th, host.data(), n_theta * sizeof(double), hipMemcpyHostToDevice, s));
  }
  mps_state* st = p->state;
  init_product(st, (const uint8_t*)st->occ.p);
  ctx->ensure_gate_work(st->dcap, p->trunc, p->opts.max_sweeps);
  ctx->reset_stats();
  const int G = p->C.G;
  const int K = p->opts.ckpt_gates;
  hipEvent_t e0, e1, e2;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventCreate(&e2));
  HIPCHK(hipEventRecord(e0, s));
  if (keep_checkpoints) {
    p->n_seg = (G + K - 1) / K;
    p->ckpt_stride = ((st->B.bytes + st->dims.bytes + st->lam.bytes + 255) / 256) * 256;
    p->ckpt.ensure((size_t)std::max(1, p->n_seg) * p->ckpt_stride);
    for (int sg = 0; sg < p->n_seg; ++sg) {
      snapshot(p, sg, true);
      run_gates(st, p->C, th, sg * K, std::min(G, (sg + 1) * K), GATE_TAPE);
      if (ctx->progress) {
        HIPCHK(hipStreamSynchronize(s));
        ctx->progress(ctx->progress_user, "forward", sg + 1, p->n_seg);
      }
    }
  } else {
    run_gates(st, p->C, th, 0, G, GATE_TAPE);
  }
  HIPCHK(hipEventRecord(e1, s));
  run_energy(st, p->H);
  HIPCHK(hipEventRecord(e2, s));
  double ev[3];
  HIPCHK(hipMemcpyAsync(ev, ctx->sb.energy, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  read_stats(ctx, stats, G);   // synchronises
  float t1 = 0.f, t2 = 0.f;
  HIPCHK(hipEventElapsedTime(&t1, e0, e1));
  HIPCHK(hipEventElapsedTime(&t2, e1, e2));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  p->E = ev[0];
  p->Eim = ev[1];
  p->Z = ev[2];
  *energy = ev[0];
  if (stats) {
    stats->t_gates_ms = t1;
    stats->t_sweep_ms = t2;
    stats->imag_E = ev[1];
    stats->norm = ev[2];
  }
}

extern "C" {

mps_status mps_plan_create(mps_ctx* ctx, const uint8_t* occ_bits, const mps_circuit* circuit,
                           const mps_paulisum* h, const mps_trunc* trunc, const mps_grad_opts* opts,
                           mps_plan** out) {
  if (!ctx || !out) return MPS_EINVAL;
  *out = nullptr;
  return guarded(ctx, [&] {
    if (!occ_bits || !circuit || !h || !trunc) fail(MPS_EINVAL, "NULL argument");
    const int N = circuit->n_qubits;
    if (N < 2 || N > 64) fail(MPS_EINVAL, "n_qubits must be in [2, 64]");
    if (trunc->d_max < 1 || trunc->d_max > 256) fail(MPS_EINVAL, "d_max must be in [1, 256]");
    if (!(trunc->eps >= 0.0) || !std::isfinite(trunc->eps)) fail(MPS_EINVAL, "eps must be finite and >= 0");
    if (trunc->precision != 0 && trunc->precision != 1) fail(MPS_EINVAL, "precision must be 0 or 1");
    for (int q = 0; q < N; ++q)
      if (occ_bits[q] > 1) fail(MPS_EINVAL, "occupation bits must be 0 or 1");
    mps_plan* p = new mps_plan();
    try {
      p->ctx = ctx;
      p->N = N;
      p->trunc = *trunc;
      if (opts) p->opts = *opts;
      if (p->opts.ckpt_gates <= 0) p->opts.ckpt_gates = 256;
      if (p->opts.max_sweeps <= 0) p->opts.max_sweeps = 64;
      if (!(p->opts.broaden >= 0.0) || !std::isfinite(p->opts.broaden)) fail(MPS_EINVAL, "bad broaden");
      if (p->opts.tape_budget_mib < -1) fail(MPS_EINVAL, "tape_budget_mib must be >= -1");
      int nth = 0;
      for (int g = 0; g < circuit->n_gates; ++g)
        if (circuit->kind && circuit->kind[g] == 1 && circuit->param) nth = std::max(nth, circuit->param[g] + 1);
      validate_circuit(circuit, N, nth);
      p->n_theta = nth;
      p->occ_h.assign(occ_bits, occ_bits + N);
      p->state = plan_new_state(ctx, N, *trunc, occ_bits);
      p->C.upload_from(circuit, ctx->stream);
      p->H.upload_from(h, N, p->state->dcap, ctx->stream, ctx->sweep_budget);
      HIPCHK(hipStreamSynchronize(ctx->stream));
    } catch (...) {
      delete p;
      throw;
    }
    *out = p;
  });
}

mps_status mps_plan_energy(mps_plan* plan, const double* theta, int32_t n_theta, double* energy,
                           mps_stats* stats) {
  if (!plan || !energy) return MPS_EINVAL;
  return guarded(plan->ctx, [&] { plan_forward_energy(plan, theta, n_theta, 0, energy, stats, false); });
}

mps_status mps_energy_grad(mps_plan* plan, const double* theta, int32_t n_theta, int32_t theta_on_device,
                           double* energy, double* grad, mps_stats* stats) {
  if (!plan || !energy || !grad) return MPS_EINVAL;
  return guarded(plan->ctx, [&] {
    double e = 0.0;
    plan_forward_energy(plan, theta, n_theta, theta_on_device, &e, stats, true);
    plan_backward(plan, grad, theta_on_device, stats);
    *energy = e;
  });
}

mps_status mps_energy_grad_batched(mps_plan* plan, int32_t n_batch, const double* thetas, int32_t n_theta,
                                   int32_t theta_on_device, double* energies, double* grads, mps_stats* stats) {
  if (!plan || !energies || !grads || (n_theta > 0 && !thetas)) return MPS_EINVAL;
  return guarded(plan->ctx, [&] {
    plan_energy_grad_batched(plan, n_batch, thetas, n_theta, theta_on_device, energies, grads, stats);
  });
}

mps_status mps_energy_grad_multi(mps_plan* const* plans, int32_t n_plans, const double* thetas, int32_t n_theta,
                                 double* energies, double* grads, mps_stats* stats) {
  if (!plans || n_plans < 1 || !plans[0] || !energies || (n_theta > 0 && (!thetas || !grads))) return MPS_EINVAL;
  return guarded(plans[0]->ctx, [&] {
    plan_energy_grad_multi(plans, n_plans, thetas, n_theta, energies, grads, stats);
  });
}

mps_status mps_energy_grad_plans(mps_plan* const* plans, int32_t n_plans, const double* const* thetas,
                                 double* energies, double* const* grads, mps_stats* stats) {
  if (!plans || n_plans < 1 || !plans[0] || !thetas || !energies || !grads) return MPS_EINVAL;
  return guarded(plans[0]->ctx, [&] { plan_energy_grad_plans(plans, n_plans, thetas, energies, grads, stats); });
}

mps_status mps_energy_grad_alg1(mps_plan* plan, const double* theta, int32_t n_theta, int32_t strings_per_group,
                                double* energy, double* grad, double* gate_grad, mps_stats* stats) {
  if (!plan || !energy || (plan->n_theta > 0 && !grad)) return MPS_EINVAL;
  return guarded(plan->ctx, [&] {
    plan_energy_grad_alg1(plan, theta, n_theta, strings_per_group, energy, grad, gate_grad, stats);
  });
}

mps_status mps_energy_grad_psr(mps_plan* plan, const double* theta, int32_t n_theta, double* energy, double* grad,
                               double* gate_grad, mps_stats* stats) {
  if (!plan || !energy || (plan->n_theta > 0 && !grad)) return MPS_EINVAL;
  return guarded(plan->ctx, [&] { plan_energy_grad_psr(plan, theta, n_theta, energy, grad, gate_grad, stats); });
}

int32_t mps_plan_batch_width(mps_plan* plan) {
  if (!plan) return MPS_EINVAL;
  int32_t w = 0;
  const mps_status st = guarded(plan->ctx, [&] { w = lanes_max(plan->state->dcap); });
  return st == MPS_OK ? w : st;
}

void mps_plan_free(mps_plan* plan) {
  if (!plan) return;
  (void)hipSetDevice(plan->ctx->device);
  (void)hipStreamSynchronize(plan->ctx->stream);
  delete plan;
}

}  // extern "C"
