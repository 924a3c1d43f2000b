/*
 * mpsvqe.h -- C ABI of the MI355X (gfx950) differentiable-MPS VQE engine.
 *
 * The engine simulates a variational circuit on a matrix product state and
 * returns the energy of a qubit Hamiltonian and its gradient, following
 * arXiv:2211.07983:
 *   - the Hartree-Fock product state as a D=1 MPS (Sec. 3, Eq. hf);
 *   - nearest-neighbour two-qubit gates applied with the Hastings update that
 *     keeps the right-canonical form and the Schmidt values (Sec. 3, Eq.
 *     rightcanonicalcondition and the two-qubit gate passage), truncated to at
 *     most D Schmidt values above a threshold eps;
 *   - E = sum_k c_k <psi|P_k|psi> as one-dimensional network contractions
 *     (Sec. 2, Eq. expect-val; Sec. 3, Eq. paulistringexp);
 *   - dE/dtheta by reverse mode through every gate, SVD and sweep (the local
 *     gradient discussed in Sec. 4, with the complex rules of App. A, Eqs.
 *     bp1-bp4), checkpointed and recomputed in the backward pass.
 *
 * Conventions (all calls):
 *   - Qubit q is MPS site q; q = 0 is the leftmost ket bit; |1> = occupied.
 *   - Bond k sits between sites k and k+1 (0 <= k <= n_qubits-2).
 *   - A 4x4 gate acting on bond k has row index 2*i'_k + i'_{k+1} and column
 *     index 2*i_k + i_{k+1}; complex numbers are (re, im) double pairs.
 *   - A Pauli string is a pair of bit masks (x, z), bit q%64 of word q/64 for
 *     qubit q; per qubit I=(0,0), X=(1,0), Z=(0,1), Y=(1,1); the operator is
 *     i^{|x&z|} X^x Z^z.
 *   - RZZ(phi) = exp(-i phi/2 Z(x)Z) = diag(e^{-i phi/2}, e^{i phi/2},
 *     e^{i phi/2}, e^{-i phi/2}).
 *
 * Ownership: input arrays are read during the call only; states and plans
 * copy what they keep (to device memory).  Objects returned through an out
 * pointer belong to the caller and are released with the matching *_free.
 *
 * Errors: every call returns an mps_status; no exception crosses the ABI, and
 * mps_last_error() describes the failure.  Errors found before any work
 * (MPS_EINVAL) leave the outputs unwritten.  MPS_ENOCONV and MPS_EDEGEN are
 * found when the work has finished: the outputs then hold what was computed
 * (with a non-converged SVD, or with the degenerate pair's adjoint term
 * dropped) and must not be used as results.  A
 * context is bound to one device and one HIP stream; it is not thread safe
 * (use one context per host thread).  Host pointers are plain host memory
 * unless a flag says a pointer is a device address.
 */
#ifndef MPSVQE_H
#define MPSVQE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mps_status;
enum {
  MPS_OK = 0,
  MPS_EINVAL = -1,   /* invalid argument (sizes, indices, NaN/Inf)           */
  MPS_ENOMEM = -2,   /* device allocation failed or capacity exceeded        */
  MPS_EDEVICE = -3,  /* HIP runtime error                                   */
  MPS_ENOCONV = -4,  /* Jacobi SVD did not converge within max_sweeps       */
  MPS_EDEGEN = -5    /* degenerate singular pair carries a cotangent        */
};

typedef struct mps_ctx mps_ctx;
typedef struct mps_state mps_state;
typedef struct mps_plan mps_plan;

/* Truncation of every two-qubit update (Sec. 3): keep
 * r = min(d_max, #{s_i > eps}) >= 1 Schmidt values of the normalised state
 * and renormalise them.
 * precision: 0 = FP64 everywhere.  1 = the Pauli sweep's transfers (Sec. 3,
 *   Eq. paulistringexp: identity environments and every term's left
 *   transfers) run as complex FP32 products on the matrix cores with FP32
 *   accumulation; the term inner products, Z and the energy sum stay FP64, as
 *   do the gates (contraction, SVD, update) and the whole reverse pass.  The
 *   energy is then accurate to about 1e-7 relative per term value.  Any other
 *   value gives MPS_EINVAL.                                                   */
typedef struct {
  int32_t d_max;
  double eps;
  int32_t precision;
} mps_trunc;

/* A compiled nearest-neighbour circuit (Sec. 3, two-qubit gates; Sec. 2,
 * UCCSD as Pauli rotations).  Gate g acts on bond bond[g]:
 *   kind[g] == 0 (FIXED): Q = pre[g]
 *   kind[g] == 1 (PARAM): Q = post[g] . RZZ(coeff[g] * theta[param[g]]) . pre[g]
 * pre/post: [n_gates][4][4][2] doubles (row-major 4x4, then re/im).          */
typedef struct {
  int32_t n_qubits;
  int32_t n_gates;
  const int32_t* bond;
  const int32_t* kind;
  const double* pre;
  const double* post;
  const int32_t* param;
  const double* coeff;
} mps_circuit;

/* H = c0 + sum_k coeff[k] P_k (Sec. 2, Eq. expect-val); x_mask/z_mask are
 * [n_terms][words] with words = ceil(n_qubits/64); coeff is real.  The
 * identity string belongs in c0: a term with x_mask = z_mask = 0, a mask bit
 * at or beyond n_qubits, or a non-finite coefficient is MPS_EINVAL.        */
typedef struct {
  int32_t n_qubits;
  int64_t n_terms;
  int32_t words;
  const uint64_t* x_mask;
  const uint64_t* z_mask;
  const double* coeff;
  double c0;
} mps_paulisum;

/* Backward-pass options: ckpt_gates = gates per checkpoint segment (the MPS
 * is saved every ckpt_gates gates and each segment is recomputed in reverse);
 * broaden = eta of the Lorentzian 1/(s_j^2-s_i^2) -> d/(d^2+eta^2) (0 = off);
 * max_sweeps = Jacobi sweep limit; strict_degenerate = 1 makes a degenerate
 * singular pair that carries a cotangent an error (MPS_EDEGEN);
 * tape_budget_mib = device memory (MiB) that mps_energy_grad_batched may hold
 * for gate tapes recorded by the forward pass, so that the reverse pass
 * recomputes only the segments that did not fit: 0 = the last segment only
 * (in the full-size tape slot); otherwise the slot plus, in the rest of the
 * budget, compact copies of the earlier segments' records (only the entries
 * the gate adjoint reads, at each gate's own bond sizes); -1 = as much as the
 * free device memory allows after a 16 GiB reserve, other negative values
 * are MPS_EINVAL.  The tapes stay allocated with the plan until
 * mps_plan_free.  Results do not depend on it.                              */
typedef struct {
  int32_t ckpt_gates;
  double broaden;
  int32_t max_sweeps;
  int32_t strict_degenerate;
  int64_t tape_budget_mib;
} mps_grad_opts;

/* Per-call statistics (any pointer to it may be NULL).                     */
typedef struct {
  double discarded_weight_sum;  /* sum over gates of discarded s^2 / total s^2 */
  double discarded_weight_max;
  double norm;                  /* Z = <psi|psi> of the final stored MPS        */
  double imag_E;                /* imaginary part of the energy sum            */
  int32_t max_bond;
  int32_t gates_truncated;      /* gates with discarded weight > 0            */
  int32_t max_sweeps_used;
  int32_t degenerate_cuts;      /* cuts with s_r - s_{r+1} < 1e-10 s_1         */
  double t_gates_ms, t_sweep_ms, t_backward_ms;
  int64_t n_gates_applied;
  /* SVD launches of the forward pass timed with HIP events on the context's
   * stream (see mps_ctx_set_profiling): summed kernel time, summed algorithmic
   * work 84 p^3 per SVD (p = min(rows, cols)) and the number of launches.
   * Single evaluations time every k-th launch; the batched form times every
   * forward step (one launch holds the SVDs of all vectors of the step).      */
  double prof_svd_ms;
  double prof_svd_flop;
  int32_t prof_svd_launches;
  int32_t prof_pad;
  /* Batched form: the gate GEMM work of the same timed launches (the two-site
   * contraction, the gate matrix and the left site update, 8 flops per
   * complex multiply-add; Sec. 3's gate update); 0 for single evaluations.   */
  double prof_gemm_flop;
} mps_stats;

/* Context on HIP device `device` using `hip_stream` (a hipStream_t; NULL =
 * the null stream).  Returns MPS_EDEVICE if the device is not usable.       */
mps_status mps_ctx_create(int32_t device, void* hip_stream, mps_ctx** out);
void mps_ctx_destroy(mps_ctx* ctx);
/* Bracket every `every`-th SVD launch of a forward pass with HIP events and
 * report the sampled kernel time in mps_stats (0 = off, the default).       */
mps_status mps_ctx_set_profiling(mps_ctx* ctx, int32_t every);
/* Progress report of long calls: a plan's forward and reverse passes call
 * fn(user, phase, done, total) on the calling thread after each checkpoint
 * segment has finished on the device ("forward" / "backward", segments done
 * out of total).  NULL fn = off (the default); with a callback set, the
 * library waits for each segment to complete before reporting it.          */
typedef void (*mps_progress_fn)(void* user, const char* phase, int64_t done, int64_t total);
mps_status mps_ctx_set_progress(mps_ctx* ctx, mps_progress_fn fn, void* user);
/* Text of the last error on ctx; valid until the next call on ctx.          */
const char* mps_last_error(const mps_ctx* ctx);

/* Sec. 3, Eq. hf: the product state |b_0 ... b_{N-1}> as a D=1 MPS with
 * capacity trunc->d_max on every bond.  occ_bits: host [n_qubits], 0 or 1.  */
mps_status mps_init_product(mps_ctx* ctx, int32_t n_qubits, const uint8_t* occ_bits,
                            const mps_trunc* trunc, mps_state** out);

/* Sec. 3 / Sec. 4 Eq. circuitevolve: apply every gate of `circuit` in order
 * with the Hastings update and truncation.  theta: host [n_theta].  On
 * validation failure the state is unchanged.                               */
mps_status mps_apply_circuit(mps_state* st, const mps_circuit* circuit, const double* theta,
                             int32_t n_theta, mps_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation and results as mps_apply_circuit on the same state, bit for bit,
 * with no device allocation of its own.  Its workspace is one fixed device
 * array per GPU (about 2.7 MiB, held until the process ends): the gate
 * workspace, theta, the statistics and the circuit, uploaded in chunks of
 * 1024 gates.  Limits: the state's d_max <= 128 and n_theta <= 8192; larger
 * requests give MPS_EINVAL before any work.  Every call on one GPU shares the
 * array: calls that overlap on one GPU (other threads or streams) race.
 * Arguments, ownership and the other errors as mps_apply_circuit; no
 * timing (stats->t_gates_ms is 0).                                          */
mps_status mps_apply_circuit_noalloc(mps_state* st, const mps_circuit* circuit, const double* theta,
                                     int32_t n_theta, mps_stats* stats);

/* Sec. 2 Eq. expect-val / Sec. 3 Eq. paulistringexp: energy = c0 +
 * sum_k coeff[k] <P_k> / <psi|psi> with a compensated final sum.
 * term_vals (nullable): host [n_terms] normalised <P_k> (real part).         */
mps_status mps_expect_paulisum(mps_state* st, const mps_paulisum* h, double* energy,
                               double* term_vals, mps_stats* stats);

/* A reusable device copy of (initial state, circuit, Hamiltonian, options)
 * for mps_plan_energy, mps_energy_grad and the batched, multi-instance,
 * Algorithm 1 and parameter-shift forms below.  occ_bits: host [n_qubits],
 * 0 or 1, the starting product state (Sec. 3, Eq. hf); circuit, h and trunc
 * as described above; opts (nullable): the backward-pass options, with
 * ckpt_gates <= 0 taken as 256 and max_sweeps <= 0 as 64.  The plan's
 * parameter count is one more than the largest param[] of a PARAM gate.
 * Every array is copied to the device during the call.  The gate matrices
 * are taken to be unitary (the update keeps the right-canonical form only
 * for unitaries); they are checked for finite entries, not for unitarity.
 * NULL arguments, n_qubits outside [2, 64], d_max outside [1, 256], a bad
 * eps, precision or option, a bond, kind or parameter index out of range, a
 * non-finite entry or a rejected Pauli sum: MPS_EINVAL with nothing
 * allocated; a failed device allocation: MPS_ENOMEM.  Release the plan with
 * mps_plan_free.                                                           */
mps_status mps_plan_create(mps_ctx* ctx, const uint8_t* occ_bits, const mps_circuit* circuit,
                           const mps_paulisum* h, const mps_trunc* trunc,
                           const mps_grad_opts* opts, mps_plan** out);

/* Sec. 4 (Eqs. expec, expecgrad, circuitevolvegrad): energy and
 * grad[p] = dE/dtheta_p.  theta and grad are host arrays, or device
 * addresses (on the context's device) when theta_on_device != 0; a device
 * theta must stay valid until the call returns.  Errors: n_theta other than
 * the plan's, NULL or non-finite theta: MPS_EINVAL before any work; a Jacobi
 * SVD that does not converge within max_sweeps: MPS_ENOCONV; with
 * strict_degenerate set, an exactly degenerate singular pair (equal to
 * 1e-10 relative) that carries a cotangent: MPS_EDEGEN (otherwise that
 * pair's term of the SVD adjoint is dropped, the d = 0 limit of the
 * broadened form, and the gradient is returned; the forward truncations
 * through nearly degenerate pairs are counted in stats->degenerate_cuts);
 * device allocation or runtime failures: MPS_ENOMEM / MPS_EDEVICE.        */
mps_status mps_energy_grad(mps_plan* plan, const double* theta, int32_t n_theta,
                           int32_t theta_on_device, double* energy, double* grad,
                           mps_stats* stats);

/* Batched form of mps_energy_grad: energies[b] and grads[b][:] of n_batch
 * parameter vectors thetas[b][:] of the same plan (row-major [n_batch][n_theta];
 * host arrays, or device addresses for thetas and grads when
 * theta_on_device != 0; energies is always host).  The vectors go through the
 * circuit together: each checkpoint segment is one launch of the gate-chain
 * kernel for all of them (as many as fit the device at once; larger batches
 * run in groups), so the compute units that a single evaluation's SVD chain
 * leaves idle are used.
 * Every result equals the one of mps_energy_grad on that vector alone.
 * stats: sums over the batch (truncation, bonds, sweeps) and the wall time of
 * the whole call in t_backward_ms.                                          */
mps_status mps_energy_grad_batched(mps_plan* plan, int32_t n_batch, const double* thetas, int32_t n_theta,
                                   int32_t theta_on_device, double* energies, double* grads,
                                   mps_stats* stats);

/* Gradient by the paper's memory-efficient back-propagation (Sec. 4,
 * Algorithm 1) with the Hamiltonian split into groups of strings_per_group
 * consecutive Pauli strings.  With one string per group (m = N_h) each group
 * state phi_k = 2 c_k P_k Psi_M is an exact MPS of Psi_M's bonds; with more,
 * phi_j = 2 sum_k c_k P_k Psi_M is built as a direct sum and compressed to the
 * plan's truncation (QR sweep from the left, truncated SVD sweep from the
 * right, then a lossless pair of sweeps for exact Schmidt values), which needs
 * strings_per_group * bond capacity <= 128.  Per group the circuit is walked
 * backwards with two states (Psi <- U^dagger Psi;
 * dE/dphi_g += Re <phi|dU_g/dphi_g|Psi>; phi <- U^dagger phi), each step the
 * forward gate update with the plan's
 * truncation; Psi stays normalised and phi keeps its norm (each truncation
 * scales it by the kept norm).  Without truncation the result is the exact
 * gradient at every theta, including theta = 0 where mps_energy_grad's local
 * gradient of the truncated evolution vanishes; with truncation it is the
 * global approximation the paper uses.  Costs 2 m passes over the circuit.
 * theta, grad: host [n_theta]; energy: E(theta); gate_grad (nullable): host
 * [n_gates], dE/dphi_g for PARAM gates and 0 for FIXED ones; stats: the
 * forward pass's.  strings_per_group < 1 or above the limit: MPS_EINVAL;
 * other errors as mps_energy_grad.                                          */
mps_status mps_energy_grad_alg1(mps_plan* plan, const double* theta, int32_t n_theta, int32_t strings_per_group,
                                double* energy, double* grad, double* gate_grad, mps_stats* stats);

/* Energies and gradients of several problem instances that share one
 * circuit, each with its own Hamiltonian (the batched-instance workload:
 * independent instances of one size class, i.e. the same qubit count and
 * bond dimension; Sec. 5 runs many molecules through one ansatz family).
 * plans[n_plans]: created by mps_plan_create on one context from the same
 * circuit (checked by a hash of the gate table), the same qubit count, d_max,
 * eps, precision and gradient options; the Hamiltonians and occupation bits may
 * differ.  Every instance is one lane of the same gate-chain launches
 * (mps_plan_batch_width(plans[0]) lanes per launch, larger sets in groups),
 * then each lane's energy and sweep adjoint run with its own plan.
 * thetas: host [n_plans][n_theta]; energies: host [n_plans]; grads: host
 * [n_plans][n_theta].  Results equal each plan's mps_energy_grad at its theta.
 * stats (nullable): sums and maxima over the instances.  Incompatible plans,
 * NULL or non-finite arguments: MPS_EINVAL before any work; the other errors as
 * mps_energy_grad.  Every plan's working buffers may be overwritten.        */
mps_status mps_energy_grad_multi(mps_plan* const* plans, int32_t n_plans, const double* thetas, int32_t n_theta,
                                 double* energies, double* grads, mps_stats* stats);

/* Energies and gradients of independent problem instances of any size in
 * shared launches (the batched-instance workload: instances that differ in
 * qubit count, circuit, Hamiltonian, d_max, eps, precision and checkpoint
 * interval; Sec. 5 runs many molecules through one ansatz family).  Each
 * plan is one lane of the same cooperative gate-chain launches: every lane
 * carries its own circuit, capacity, Jacobi block width and work-group
 * count, and a launch advances every lane by one of its own checkpoint
 * segments (lanes whose circuits are shorter finish early).  Energies and
 * sweep adjoints then run per plan.  The reverse pass works through windows
 * of segment indices from the last down: in a window every plan's segments
 * are recomputed side by side, one lane per (plan, segment), in one shared
 * launch, then the gate adjoints of all plans run down the window step by
 * step in shared launch sets.  Larger sets run in groups that one launch
 * holds.  plans[n_plans]: distinct plans of one context;
 * thetas[i]: host array of plan i's n_theta parameters; energies: host
 * [n_plans]; grads[i]: host array of plan i's n_theta.  Results equal each
 * plan's mps_energy_grad up to rounding.  stats (nullable): sums and maxima
 * over the instances, the wall time in t_backward_ms.  NULL, repeated or
 * non-finite arguments, or plans of different contexts: MPS_EINVAL before
 * any work; the other errors as mps_energy_grad (MPS_EDEGEN when any plan
 * asks for strict_degenerate).                                             */
mps_status mps_energy_grad_plans(mps_plan* const* plans, int32_t n_plans, const double* const* thetas,
                                 double* energies, double* const* grads, mps_stats* stats);

/* Parameter vectors that one batched launch holds for this plan (the SVD of
 * each vector occupies ceil(2 d_max / (2 W)) compute units); larger batches
 * run in groups of this size.  Returns <= 0 on error.                      */
int32_t mps_plan_batch_width(mps_plan* plan);

/* Parameter-shift gradient (Sec. 4, Eq. psr) of the plan's energy, the
 * baseline that mps_energy_grad's back-propagation replaces.  For each PARAM
 * gate g (angle phi_g = coeff[g] theta[param[g]]; RZZ(phi) = exp(-i phi ZZ/2),
 * generator eigenvalues +-1/2) the energy is evaluated with phi_g shifted by
 * +pi/2 and by -pi/2: dE/dphi_g = (E+ - E-)/2, and
 * grad[p] = sum over gates g with param[g] = p of coeff[g] dE/dphi_g.
 * 2M + 1 forward evaluations for M PARAM gates, run as lanes of batched
 * launches of the gate-chain kernel (mps_plan_batch_width per launch).
 * theta, grad: host [n_theta]; energy: E(theta); gate_grad (nullable): host
 * [n_gates], dE/dphi_g for PARAM gates and 0 for FIXED ones.  Without
 * truncation the result equals the back-propagated gradient; with it, each
 * shifted evaluation truncates on its own.  stats: sums over all evaluations,
 * the wall time in t_gates_ms.  Errors as mps_energy_grad.                  */
mps_status mps_energy_grad_psr(mps_plan* plan, const double* theta, int32_t n_theta, double* energy,
                               double* grad, double* gate_grad, mps_stats* stats);

/* Forward pass of a plan only (energy at theta, no gradient).              */
mps_status mps_plan_energy(mps_plan* plan, const double* theta, int32_t n_theta,
                           double* energy, mps_stats* stats);

/* Test access: bond dimensions (host int32 [n_qubits+1], dims[k] = bond left
 * of site k), site tensors and Schmidt vectors.  B: host complex [n][dl][2][dr]
 * packed per site in site order; lam: host double [n_qubits+1][d_max].      */
mps_status mps_state_export(const mps_state* st, int32_t* dims, double* B, double* lam);
int64_t mps_state_size(const mps_state* st);   /* doubles needed by B above */
/* Test access, the inverse of mps_state_export: a new state on ctx from host
 * copies of an MPS in the form of Sec. 3 (site tensors B_n[alpha][i][beta]
 * and the Schmidt vectors lambda_k of Eq. rightcanonicalcondition), so that
 * the expectation (Eq. paulistringexp) and the gate update can be checked on
 * states built elsewhere.  dims: [n_qubits+1] with dims[0] = dims[n_qubits]
 * = 1 and 1 <= dims[k] <= trunc->d_max; B: complex [n][dims[n]][2][dims[n+1]]
 * packed per site in site order (mps_state_export's layout, mps_state_size
 * doubles); lam: packed, dims[k] values for each k = 0..n_qubits.  The
 * tensors need not be canonical or normalised: mps_expect_paulisum divides
 * by <psi|psi>; the gate update weights with lam as given.  trunc: the
 * truncation of later updates, as in mps_init_product.  The arrays are read
 * during the call only.  Bad sizes, NULL or non-finite input: MPS_EINVAL,
 * nothing allocated.                                                       */
mps_status mps_state_import(mps_ctx* ctx, int32_t n_qubits, const mps_trunc* trunc, const int32_t* dims,
                            const double* B, const double* lam, mps_state** out);
int32_t mps_state_qubits(const mps_state* st);

/* Release a state or a plan and its device memory, after the work queued on
 * its context's stream has finished.  NULL is a no-op.                      */
void mps_state_free(mps_state* st);
void mps_plan_free(mps_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* MPSVQE_H */
