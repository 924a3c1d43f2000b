// Host-side helpers shared by engine.hip, plan.hip and adjoint.hip.
#pragma once

#include <string>

#include "errors.h"
#include "plan.h"

template <class F>
mps_status guarded(mps_ctx* ctx, F&& f) {
  try {
    if (ctx) ctx->set_device();
    f();
    if (ctx) ctx->err.clear();
    return MPS_OK;
  } catch (const Failure& e) {
    if (ctx) ctx->err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    if (ctx) ctx->err = e.what();
    return MPS_ENOMEM;
  }
}

template <class T>
T* upload(DevBuf& buf, const T* src, size_t count, hipStream_t s) {
  T* d = (T*)buf.ensure(count * sizeof(T));
  if (count) HIPCHK(hipMemcpyAsync(d, src, count * sizeof(T), hipMemcpyHostToDevice, s));
  return d;
}

MpsView view_of(mps_state* st);
void alloc_state(mps_state* st);
void init_product(mps_state* st, const uint8_t* occ_dev);
void copy_state(mps_state* dst, mps_state* src, hipStream_t s);
void run_energy(mps_state* st, DevHamiltonian& H);
void run_identity_envs(mps_state* st);
// Applies gates [g0, g1).  A plan's forward pass uses GATE_TAPE so that the
// states it checkpoints are bitwise the ones its reverse pass recomputes.
void run_gates(mps_state* st, DevCircuit& C, const double* theta_dev, int g0, int g1, GateMode mode);
void read_stats(mps_ctx* ctx, mps_stats* out, int64_t gates);
void validate_circuit(const mps_circuit* c, int N, int n_theta);
void validate_theta(const double* theta, int n_theta);
// Sets up the allocation-free workspace of `device` (current), once per device.
void noalloc_device_init(int device);

mps_state* plan_new_state(mps_ctx* ctx, int N, const mps_trunc& tr, const uint8_t* occ);
void plan_forward_energy(mps_plan* p, const double* theta, int n_theta, int on_device, double* energy,
                         mps_stats* stats, bool keep_checkpoints);
void plan_backward(mps_plan* p, double* grad, int on_device, mps_stats* stats);
void plan_energy_grad_psr(mps_plan* p, const double* theta, int n_theta, double* energy, double* grad,
                          double* gate_grad, mps_stats* stats);
void plan_energy_grad_alg1(mps_plan* p, const double* theta, int n_theta, int per_group, double* energy,
                           double* grad, double* gate_grad, mps_stats* stats);
void plan_energy_grad_plans(mps_plan* const* plans, int n, const double* const* thetas, double* energies,
                            double* const* grads, mps_stats* stats);
void plan_energy_grad_multi(mps_plan* const* plans, int n, const double* thetas, int n_theta, double* energies,
                            double* grads, mps_stats* stats);
void plan_energy_grad_batched(mps_plan* p, int nb, const double* thetas, int n_theta, int on_device,
                              double* energies, double* grads, mps_stats* stats);
