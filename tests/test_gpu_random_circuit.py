"""Energy and gradient beyond the molecular workload (Sec. 3 gate update and
Pauli sweep, Sec. 4 back-propagation, Algorithm 1 and the parameter shift):
circuits of random complex two-qubit gates and Pauli sums of random strings
of every kind, from tests/random_circuit.py, through the plan calls, against
the oracle.  The molecular Hamiltonians hold only even-Y strings and the UCCSD
states are real up to a phase; here neither holds, so a phase or transpose
slip in the sweep, the sweep adjoint, the gate adjoint or the Pauli images of
Algorithm 1 would show.

The main case (8 qubits, 120 gates, 10 parameters, 300 strings, checkpoints
every 32 gates) runs at exact D = 16 and at a truncating D = 4 (41 truncating
gates, every cut at least 2.7e-2 s_1 from the next value, so the truncation is
unique) in FP64, E to 1e-10 relative and g to 1e-8 of its largest entry, and
at exact D = 16 in precision 1 (FP32 matrix-core sweep transfers), held to the
FP32 bound used for the molecular cases (term error 4 n 2D 2^-24 times
sum |c_k| for E, 1e-5 of the largest entry for g).  The same circuit then goes
through Algorithm 1, the batched parameter shift and a batch over two lane
groups; further cases cover three sizes in one plans-array call, the shortest
chains (2, 3 and 5 qubits, down to D = 1) and 64 qubits."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_07983_amd import Context
    c = Context(0)
    yield c
    c.close()


def case():
    import random_circuit as rc
    gl, th = rc.circuit(8, 120, 10, 5)
    return rc.problem(8, 300, 16, 1e-12, 6), gl, th


@pytest.mark.parametrize("D,precision", [(16, 0), (4, 0), (16, 1)])
def test_random_complex_circuit_matches_oracle(ctx, D, precision):
    from oracle import mps
    from paper_2211_07983_amd import Plan
    p, gl, th = case()
    e_ref, g_ref, info = mps.energy_grad(p, gl, th, D=D, ckpt=32)
    plan = Plan(ctx, p.occ, gl, 8, p.ham_x, p.ham_z, p.ham_c, p.c0, D, 1e-12, precision=precision,
                ckpt_gates=32)
    try:
        e, g, _ = plan.energy_grad(th)
        eb, gb, _ = plan.energy_grad_batched(np.stack([th, th]))
        _, s = plan.energy(th)          # forward-only statistics
    finally:
        plan.free()
    gerr = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print(f"D={D} precision {precision}: E error {abs(e - e_ref):.2e}, gradient error {gerr:.2e} of the largest "
          f"entry, discarded {s['discarded_weight_sum']:.3e} (oracle {sum(info['discarded']):.3e})")
    if precision == 0:
        assert abs(e - e_ref) <= 1e-10 * abs(e_ref)
        assert gerr <= 1e-8
    else:
        assert abs(e - e_ref) <= 4.0 * 8 * 2 * D * 2.0 ** -24 * np.abs(p.ham_c).sum()
        assert gerr <= 1e-5
    assert abs(s["discarded_weight_sum"] - sum(info["discarded"])) <= 1e-10
    assert abs(eb[1] - e) <= 1e-12 * abs(e)
    assert np.abs(gb[1] - g).max() <= 1e-9 * np.abs(g).max()


@pytest.mark.parametrize("per_group", [1, 4])
def test_random_complex_circuit_algorithm_1(ctx, per_group):
    """The paper's Algorithm 1 (Sec. 4) on the same circuit at exact D: the
    Pauli images P_k Psi carry odd numbers of Y's here, which the molecular
    strings never have.  Per-gate dE/dphi against the oracle's Algorithm 1 and
    the gradient against the oracle's back-propagated one (both exact at this
    D), to 1e-9 of the largest entry."""
    from oracle import alg1, mps
    from paper_2211_07983_amd import Plan
    p, gl, th = case()
    _, g_ref, _ = mps.energy_grad(p, gl, th, D=16)
    _, info = alg1.energy_grad(p, gl, th, per_group=per_group)
    plan = Plan(ctx, p.occ, gl, 8, p.ham_x, p.ham_z, p.ham_c, p.c0, 16, 1e-12)
    try:
        _, g, gphi, _ = plan.energy_grad_alg1(th, strings_per_group=per_group)
    finally:
        plan.free()
    gerr = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    perr = np.abs(gphi - info["gphi"]).max() / np.abs(info["gphi"]).max()
    print(f"Algorithm 1, {per_group} per group: gradient error {gerr:.2e}, per-gate error {perr:.2e}")
    assert gerr <= 1e-9
    assert perr <= 1e-9


def test_random_complex_circuit_parameter_shift(ctx):
    """Batched parameter shift (Sec. 4, Eq. psr) on the same circuit: every
    parametric gate's angle c theta_p shifted by +-pi/2, with random
    coefficients c in {-1, 1/2, 1, 2} carrying the chain rule.  Per-gate
    dE/dphi and the gradient against the oracle's back-propagated ones at
    exact D, to 1e-9 of the largest entry."""
    from oracle import mps
    from paper_2211_07983_amd import Plan
    p, gl, th = case()
    _, g_ref, info = mps.energy_grad(p, gl, th, D=16)
    plan = Plan(ctx, p.occ, gl, 8, p.ham_x, p.ham_z, p.ham_c, p.c0, 16, 1e-12)
    try:
        _, g, gphi, _ = plan.energy_grad_psr(th)
    finally:
        plan.free()
    gerr = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    perr = np.abs(gphi - info["gphi"]).max() / np.abs(info["gphi"]).max()
    print(f"parameter shift: gradient error {gerr:.2e}, per-gate error {perr:.2e}")
    assert gerr <= 1e-9 and perr <= 1e-9


def test_random_complex_circuits_of_three_sizes_in_shared_launches(ctx):
    """mps_energy_grad_plans with three random complex circuits of different
    qubit counts, D and checkpoint intervals: 8 q at exact D = 16, 6 q at
    D = 4 (10 truncating gates) and 10 q at D = 8 (23 truncating gates), every
    cut at least 1.7e-2 s_1 from the next value.  Each against the oracle at
    its own D: E to 1e-10 relative, g to 1e-8 of its largest entry."""
    import random_circuit as rc
    from oracle import mps
    from paper_2211_07983_amd import Plan, energy_grad_plans
    specs = [(8, 120, 10, 5, 16, 32), (6, 80, 6, 21, 4, 20), (10, 100, 8, 31, 8, 48)]
    cases, plans = [], []
    try:
        for n, G, T, seed, D, ck in specs:
            gl, th = rc.circuit(n, G, T, seed)
            p = rc.problem(n, 300 if n == 8 else 150, D, 1e-12, seed + 1, n_theta=T)
            cases.append((p, gl, th, D))
            plans.append(Plan(ctx, p.occ, gl, n, p.ham_x, p.ham_z, p.ham_c, p.c0, D, 1e-12, ckpt_gates=ck))
        es, gs, _ = energy_grad_plans(plans, [c[2] for c in cases])
    finally:
        for pl in plans:
            pl.free()
    for (p, gl, th, D), e, g in zip(cases, es, gs):
        e_ref, g_ref, _ = mps.energy_grad(p, gl, th, D=D)
        gerr = np.abs(g - g_ref).max() / np.abs(g_ref).max()
        print(f"  {p.n_qubits} q, D={D}: E error {abs(e - e_ref):.2e}, gradient error {gerr:.2e}")
        assert abs(e - e_ref) <= 1e-10 * abs(e_ref)
        assert gerr <= 1e-8


@pytest.mark.parametrize("n,D", [(2, 2), (2, 1), (3, 2), (3, 1), (5, 4), (5, 2)])
def test_short_chains(ctx, n, D):
    """The shortest chains the interface takes (2 qubits: one bond, both
    sites at the boundary; odd lengths 3 and 5), exact and truncating down to
    D = 1 (a product state after every gate), random complex circuits with
    every cut at least 8.9e-2 s_1 from the next value: E to 1e-10 relative and
    g to 1e-8 of its largest entry against the oracle."""
    import random_circuit as rc
    from oracle import mps
    from paper_2211_07983_amd import Plan
    G, T, seed = {2: (30, 4, 41), 3: (40, 5, 43), 5: (60, 6, 45)}[n]
    gl, th = rc.circuit(n, G, T, seed)
    p = rc.problem(n, 40, D, 1e-12, seed + 1, n_theta=T)
    e_ref, g_ref, info = mps.energy_grad(p, gl, th, D=D, ckpt=16)
    plan = Plan(ctx, p.occ, gl, n, p.ham_x, p.ham_z, p.ham_c, p.c0, D, 1e-12, ckpt_gates=16)
    try:
        e, g, _ = plan.energy_grad(th)
        _, s = plan.energy(th)
    finally:
        plan.free()
    gerr = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print(f"{n} q, D={D}: E error {abs(e - e_ref):.2e}, gradient error {gerr:.2e}, max bond {s['max_bond']}")
    assert s["max_bond"] == max(info["bonds"])
    assert abs(e - e_ref) <= 1e-10 * abs(e_ref)
    assert gerr <= 1e-8


def test_sixty_four_qubits(ctx):
    """The longest chain one mask word holds: 64 qubits, with bit 63 of the
    masks in use.  A 300-gate random complex circuit at D = 4 (105 truncating
    gates, every cut at least 3.6e-2 s_1 from the next value), 120 sparse
    random strings (1 to 4 qubits each) and three strings on the last qubit,
    one of them spanning the whole chain (Y_0 X_63): E to 1e-10 relative and
    g to 1e-8 of its largest entry against the oracle."""
    import random_circuit as rc
    from oracle import mps
    from paper_2211_07983_amd import Plan
    n = 64
    gl, th = rc.circuit(n, 300, 12, 61)
    p = rc.problem(n, 120, 4, 1e-12, 62, n_theta=12, max_weight=4)
    top = np.uint64(1) << np.uint64(63)
    p.ham_x = np.concatenate([p.ham_x, np.array([0, top | (np.uint64(1) << np.uint64(62)), top | np.uint64(1)],
                                                dtype=np.uint64)])
    p.ham_z = np.concatenate([p.ham_z, np.array([top, top, np.uint64(1)], dtype=np.uint64)])
    p.ham_c = np.concatenate([p.ham_c, [0.7, -0.4, 0.9]])
    e_ref, g_ref, _ = mps.energy_grad(p, gl, th, D=4, ckpt=64)
    plan = Plan(ctx, p.occ, gl, n, p.ham_x, p.ham_z, p.ham_c, p.c0, 4, 1e-12, ckpt_gates=64)
    try:
        e, g, _ = plan.energy_grad(th)
    finally:
        plan.free()
    gerr = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print(f"64 q, D=4: E error {abs(e - e_ref):.2e}, gradient error {gerr:.2e}")
    assert abs(e - e_ref) <= 1e-10 * abs(e_ref)
    assert gerr <= 1e-8


@pytest.mark.parametrize("budget", [0, -1])
def test_batch_spanning_two_lane_groups(ctx, budget):
    """More parameter vectors than one chain launch holds, so the batch runs
    as a full lane group and a remainder of two: the 8-qubit circuit at
    d_max = 64 (four work-groups per lane; the actual bonds stay at or below
    16), seeded vectors theta + 0.3 N(0, 1), with the forward tapes recomputed
    (budget 0) or archived (budget -1, the archive reused by the second
    group).  Vectors on both sides of the group boundary against the oracle
    (E to 1e-10 relative, g to 1e-8 of its largest entry), and a vector
    repeated in the second group equal to its first-group result."""
    from oracle import mps
    from paper_2211_07983_amd import Plan
    p, gl, th = case()
    plan = Plan(ctx, p.occ, gl, 8, p.ham_x, p.ham_z, p.ham_c, p.c0, 64, 1e-12, ckpt_gates=32,
                tape_budget_mib=budget)
    try:
        per = plan.lanes_per_launch()
        nb = per + 2
        rng = np.random.default_rng(19)
        thetas = th + 0.3 * rng.normal(size=(nb, len(th)))
        thetas[per + 1] = thetas[1]
        eb, gb, st = plan.energy_grad_batched(thetas)
    finally:
        plan.free()
    print(f"{nb} vectors, {per} per launch")
    assert st["n_gates_applied"] == nb * gl.n_gates
    for b in (0, per - 1, per):
        e_ref, g_ref, _ = mps.energy_grad(p, gl, thetas[b], D=64)
        gerr = np.abs(gb[b] - g_ref).max() / np.abs(g_ref).max()
        print(f"  vector {b}: E error {abs(eb[b] - e_ref):.2e}, gradient error {gerr:.2e}")
        assert abs(eb[b] - e_ref) <= 1e-10 * abs(e_ref)
        assert gerr <= 1e-8
    assert abs(eb[per + 1] - eb[1]) <= 1e-13 * abs(eb[1])
    assert np.abs(gb[per + 1] - gb[1]).max() <= 1e-12 * np.abs(gb[1]).max()
