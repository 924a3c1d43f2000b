"""The remaining workload configurations as GPU parity cases:

* 40 qubits (20 orbitals, 4 electrons), D = 256, 233000 Pauli terms: the
  state after the first 3000 gates (capacity 256: 4-column Jacobi blocks) and
  its energy over every term, in FP64 and in precision 1;
* four instances of the batched set (qubits and D drawn per instance): one
  exact (12 q, D = 64) and three that truncate at the paper's threshold
  eps = 1e-6 (12 q at D = 32, 64 and 128), energy and gradient against the
  oracle; the conditioning of each case sets its tolerance (C4_CASES).  Where
  a truncation at D cuts through equal Schmidt values, which of them are kept
  is arbitrary and E_D and g_D are not unique; at the parity threshold 1e-12
  the set's truncating instances have such cuts among rounding-level values,
  at 1e-6 these have none (the oracle's degenerate-cut count, asserted on both
  sides);
* the first 2000 gates of the 40-qubit workload with every 100th Pauli term:
  energy and gradient with the MPS checkpointed and recomputed.

Expected values come from the oracle (tests/golden/make_golden.py)."""
import numpy as np
import pytest

from vqe_inputs import configs
from gpu_util import Prefix, golden, gpu_energy, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_07983_amd import Context
    c = Context(0)
    yield c
    c.close()


def grad_ok(g, ref, tol=1e-8):
    return np.abs(g - ref).max() <= tol * max(1.0, np.abs(ref).max())


def test_40_qubit_prefix_energy_matches_oracle(ctx):
    from paper_2211_07983_amd import State
    p, g = configs.load("c5")
    gold = golden()["c5_prefix"]
    pre = Prefix(g, gold["gates"])
    e, _, s1, s2, st = gpu_energy(ctx, p, pre, p.theta)
    dims, _, _ = st.export()
    st.free()
    assert list(dims[1:-1]) == gold["bonds"]
    assert rel(e, gold["E"]) <= 1e-10
    assert abs(s2["norm"] - gold["Z"]) <= 1e-12
    # precision 1 on the same circuit: the matrix-core sweep over all terms
    s32 = State.product(ctx, p.occ, p.bond_dim, p.eps, precision=1)
    s32.apply_circuit(pre, p.theta)
    e32, _, _ = s32.expect(p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0)
    s32.free()
    print(f"40 q prefix: E {e:.12f}, precision-1 difference {abs(e32 - e):.2e} Ha")
    assert abs(e32 - e) <= 1e-6


# Batched-set instances compared with the oracle: (instance, broadened
# gradient, E tolerance (relative), gradient tolerance).
#  4: 12 q, D = 64, eps = 1e-12: exact, strict.
#  5: 12 q, D = 64, eps = 1e-6: truncates by eps on 1157 gates, strict.
#  8: 12 q, D = 128, eps = 1e-6: the same physics at capacity 128; E strict;
#     its plain g_D holds nearly degenerate kept pairs that carry cotangents
#     (the oracle's own g_D moves by 3e-6 when eta = 1e-12), so the gradient is
#     compared broadened (eta = 1e-8 on both sides).
#  3: 12 q, D = 32, eps = 1e-6: truncates at D on 2249 gates (discarded
#     weight 3.3e-3) with cuts as close as 1.5e-7 s_1.  There E_D and g_D are
#     fixed only up to rounding: the oracle itself, rerun with another LAPACK
#     driver or BLAS thread count, moves E by up to ~2e-7 Ha and the broadened
#     gradient by ~1e-3 of its largest entry.  The GPU's Jacobi SVD is one
#     more such rounding, so it is held to twice the diameter of the oracle's
#     own rounding variants (None).
C4_CASES = [(4, False, 1e-10, 1e-8), (5, False, 1e-10, 1e-8), (8, True, 1e-10, 1e-8), (3, True, None, None)]
SPREAD_FACTOR = 2.0


@pytest.mark.parametrize("case", C4_CASES, ids=[f"instance{c[0]}" for c in C4_CASES])
def test_batched_set_instance_matches_oracle(ctx, case):
    """Instances of the batched set (qubits and D drawn per instance) against
    the oracle at their own D; none has a cut inside a degenerate pair at its
    threshold (the oracle's count and the GPU's are zero at eps = 1e-6; at the
    parity threshold 1e-12 cuts among rounding-level values may count and
    truncate nothing physical).  The 16-qubit instances 14 and 17 have stored
    oracle values too; one evaluation of theirs takes minutes here, so they
    are left to the benchmark's instance phase."""
    from paper_2211_07983_amd import Plan
    from vqe_inputs.compile import compile_problem
    from vqe_inputs.problem import make_problem
    i, broadened, e_tol, g_tol = case
    n, ne, D, s1, s2 = configs.batched_instances()[i]
    gold = golden()[f"c4_{i}" if i == 4 else f"c4p_{i}"]
    gref = golden()[f"c4p_{i}_b"] if broadened else gold
    assert (gold["n_qubits"], gold["D"]) == (n, D)
    eps = gold.get("eps", configs.PARITY_EPS)
    assert gold.get("degenerate_cuts", 0) == 0
    p = make_problem(f"c4_{i}", n, ne, D, eps, s1, s2, 0.05)
    g = compile_problem(p)
    plan = Plan(ctx, p.occ, g, p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, p.bond_dim, p.eps,
                broaden=gref.get("broaden", 0.0))
    e, grad, st = plan.energy_grad(p.theta)
    _, fst = plan.energy(p.theta)
    disc = fst["discarded_weight_sum"]
    ref = np.array(gref["grad"])
    gerr = np.abs(grad - ref).max() / max(1.0, np.abs(ref).max())
    print(f"instance {i}: {n} q, D={D}, eps={eps:g}, truncated gates {st['gates_truncated']}, discarded {disc:.3e}, "
          f"degenerate cuts {fst['degenerate_cuts']}, E error {abs(e - gold['E']):.2e}, "
          f"{'broadened ' if broadened else ''}grad error {gerr:.2e}")
    if eps > configs.PARITY_EPS:
        assert fst["degenerate_cuts"] == 0
    assert st["max_bond"] == max(gold["bonds"])
    if e_tol is None:
        # conditioning-limited: the diameter of the oracle's rounding variants
        # (energy, gradient and total discarded weight alike)
        runs = [gold] + golden()[f"c4p_{i}_b_variants"]["variants"]
        gscale = max(1.0, np.abs(ref).max())
        e_spread = max(abs(a["E"] - b["E"]) for a in runs for b in runs)
        d_spread = max(abs(a["discarded_sum"] - b["discarded_sum"]) for a in runs for b in runs)
        g_runs = [gref] + runs[1:]
        g_spread = max(np.abs(np.array(a["grad"]) - np.array(b["grad"])).max() for a in g_runs for b in g_runs) / gscale
        print(f"  oracle rounding variants: E spread {e_spread:.2e}, grad spread {g_spread:.2e}, "
              f"discarded-weight spread {d_spread:.2e} (GPU {abs(disc - gold['discarded_sum']):.2e})")
        assert abs(disc - gold["discarded_sum"]) <= SPREAD_FACTOR * d_spread
        assert abs(e - gref["E"]) <= SPREAD_FACTOR * e_spread
        assert gerr <= SPREAD_FACTOR * g_spread
    else:
        # each gate's discarded weight is 1 - kept / total in FP64: about 1e-16
        # of cancellation per gate on either side
        assert abs(disc - gold["discarded_sum"]) <= 1e-8 * gold["discarded_sum"] + 1e-15 * len(g.bond)
        assert rel(e, gold["E"]) <= e_tol
        assert gerr <= g_tol
    if i == 4:
        eb, gb, _ = plan.energy_grad_batched(np.stack([p.theta, p.theta]))
        assert abs(eb[1] - e) <= 1e-13 * abs(e)
        assert np.abs(gb[1] - grad).max() <= 1e-12 * np.abs(grad).max()
    plan.free()


def test_40_qubit_prefix_gradient_with_checkpoints_matches_oracle(ctx):
    """Energy and gradient of the first 2000 gates of the 40-qubit D = 256
    workload (capacity 256, 4-column Jacobi blocks) for every 100th Pauli
    term, with the MPS checkpointed every 426 gates (8 compiled rotation
    blocks on average) and each segment recomputed in the reverse pass."""
    import dataclasses
    from paper_2211_07983_amd import Plan
    p, g = configs.load("c5")
    gold = golden()["c5_prefix_grad"]
    pre = Prefix(g, gold["gates"])
    sub = slice(0, None, gold["term_stride"])
    ps = dataclasses.replace(p, ham_x=p.ham_x[sub], ham_z=p.ham_z[sub], ham_c=p.ham_c[sub])
    assert len(ps.ham_c) == gold["n_terms"] and gold["degenerate_cuts"] == 0
    plan = Plan(ctx, p.occ, pre, p.n_qubits, ps.ham_x, ps.ham_z, ps.ham_c, p.c0, p.bond_dim, p.eps,
                ckpt_gates=gold["ckpt_gates"])
    th = np.array(p.theta[: plan.n_theta])
    e, grad, st = plan.energy_grad(th)
    ref = np.array(gold["grad"])
    print(f"40 q prefix gradient: {plan.n_theta} parameters, E error {abs(e - gold['E']):.2e}, "
          f"grad error {np.abs(grad - ref).max() / np.abs(ref).max():.2e}")
    assert st["max_bond"] == max(gold["bonds"])
    assert rel(e, gold["E"]) <= 1e-10
    assert grad_ok(grad, ref)
    plan.free()
