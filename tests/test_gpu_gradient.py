"""GPU reverse pass (S7-S9) against the CPU oracle, through the C ABI."""
import numpy as np
import pytest

from vqe_inputs import configs
from gpu_util import Prefix, golden, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_07983_amd import Context
    c = Context(0)
    yield c
    c.close()


def make_plan(ctx, p, g, **kw):
    from paper_2211_07983_amd import Plan
    return Plan(ctx, p.occ, g, p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, p.bond_dim, p.eps, **kw)


def grad_ok(g, ref, tol=1e-8):
    d = np.abs(g - ref)
    return (np.linalg.norm(g - ref) <= tol * np.linalg.norm(ref)
            and d.max() <= tol * max(1.0, np.abs(ref).max()))


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_energy_grad_matches_oracle(ctx, name):
    p, g = configs.load(name)
    gold = golden()[name]
    plan = make_plan(ctx, p, g, ckpt_gates=256)
    e, grad, st = plan.energy_grad(p.theta)
    assert rel(e, gold["E"]) <= 1e-10
    assert grad_ok(grad, np.array(gold["grad"]))
    assert grad_ok(grad, np.array(gold["grad_exact"]), 1e-8)
    plan.free()


def test_paper_threshold_energy_grad_matches_oracle(ctx):
    """C2 at eps = 1e-6 (the paper's setting): truncation by the threshold on
    every bond; E_D and g_D against the oracle at the same threshold."""
    p, g = configs.load("c2", eps=configs.PAPER_EPS)
    gold = golden()["c2_paper"]
    assert gold["eps"] == p.eps
    plan = make_plan(ctx, p, g, ckpt_gates=512)
    e, grad, st = plan.energy_grad(p.theta)
    assert st["gates_truncated"] > 1000
    assert rel(e, gold["E"]) <= 1e-10
    assert grad_ok(grad, np.array(gold["grad"]))
    plan.free()


def test_benchmark_configuration_batched(ctx):
    """The benchmark's own launch configuration: 14 qubits at eps = 1e-6,
    512-gate checkpoints, as many vectors as one launch holds (the configured
    theta and the benchmark's seeded perturbations).  Vector 0 against the
    oracle at the same threshold; two others (the second and the last) against
    the single-vector path."""
    p, g = configs.load("c2", eps=configs.PAPER_EPS)
    gold = golden()["c2_paper"]
    plan = make_plan(ctx, p, g, ckpt_gates=512)
    nb = plan.lanes_per_launch()
    assert nb >= 2
    rng = np.random.default_rng(2024)
    thetas = np.stack([p.theta] + [p.theta + 0.05 * rng.normal(size=p.theta.shape) for _ in range(nb - 1)])
    eb, gb, st = plan.energy_grad_batched(thetas)
    assert st["n_gates_applied"] == nb * g.n_gates
    assert rel(eb[0], gold["E"]) <= 1e-10
    assert grad_ok(gb[0], np.array(gold["grad"]))
    for b in (1, nb - 1):
        e1, g1, _ = plan.energy_grad(thetas[b])
        assert abs(eb[b] - e1) <= 1e-13 * abs(e1)
        assert np.abs(gb[b] - g1).max() <= 1e-12 * np.abs(g1).max()
    plan.free()


@pytest.mark.parametrize("name,nb", [("c1", 5), ("c2", 3)])
def test_batched_equals_single(ctx, name, nb):
    """mps_energy_grad_batched on nb parameter vectors (the configured one and
    seeded perturbations of it) against mps_energy_grad on each alone, and the
    configured vector against the oracle."""
    p, g = configs.load(name)
    rng = np.random.default_rng(77)
    thetas = np.stack([p.theta] + [p.theta + 0.05 * rng.normal(size=p.theta.shape) for _ in range(nb - 1)])
    plan = make_plan(ctx, p, g, ckpt_gates=128)
    eb, gb, st = plan.energy_grad_batched(thetas)
    assert st["n_gates_applied"] == nb * g.n_gates
    for b in range(nb):
        e1, g1, _ = plan.energy_grad(thetas[b])
        assert abs(eb[b] - e1) <= 1e-13 * abs(e1)
        assert np.abs(gb[b] - g1).max() <= 1e-12 * np.abs(g1).max()
    gold = golden()[name]
    assert rel(eb[0], gold["E"]) <= 1e-10
    assert grad_ok(gb[0], np.array(gold["grad"]))
    plan.free()


@pytest.mark.parametrize("budget", [-1, 180, 64])
def test_batched_with_kept_forward_tapes_equals_single(ctx, budget):
    """The batched form with the forward pass's tapes kept (12 segments of
    128 gates; the last one stays in the tape slot, the others go to the
    compact archive while it has room: all eleven at budget -1 and 180 MiB,
    two at 64 MiB, the rest recomputed) against the single evaluations: the
    same arithmetic, so the same results, on two calls in a row."""
    p, g = configs.load("c1")
    rng = np.random.default_rng(78)
    nb = 3
    thetas = np.stack([p.theta] + [p.theta + 0.05 * rng.normal(size=p.theta.shape) for _ in range(nb - 1)])
    plan = make_plan(ctx, p, g, ckpt_gates=128, tape_budget_mib=budget)
    eb, gb, st = plan.energy_grad_batched(thetas)
    eb2, gb2, _ = plan.energy_grad_batched(thetas)     # buffers reused
    assert st["n_gates_applied"] == nb * g.n_gates
    for b in range(nb):
        e1, g1, _ = plan.energy_grad(thetas[b])
        assert abs(eb[b] - e1) <= 1e-13 * abs(e1) and abs(eb2[b] - e1) <= 1e-13 * abs(e1)
        assert np.abs(gb[b] - g1).max() <= 1e-12 * np.abs(g1).max()
        assert np.abs(gb2[b] - g1).max() <= 1e-12 * np.abs(g1).max()
    plan.free()


def test_negative_tape_budget_is_refused(ctx):
    from paper_2211_07983_amd import MPSError
    p, g = configs.load("c1")
    with pytest.raises(MPSError, match="tape_budget_mib"):
        make_plan(ctx, p, g, tape_budget_mib=-2)


def test_c3_prefix_energy_grad_matches_oracle(ctx):
    """First 2500 gates of the 24-qubit D=128 workload: the middle SVDs are
    256 x 256 and truncate to 128 at every step; E_D and g_D against the oracle."""
    p, g = configs.load("c3")
    gold = golden()["c3_prefix_grad"]
    pre = Prefix(g, gold["gates"])
    plan = make_plan(ctx, p, pre, ckpt_gates=256)
    assert plan.n_theta == gold["n_theta"]
    e, grad, st = plan.energy_grad(p.theta[:plan.n_theta])
    assert st["max_bond"] == 128 and st["gates_truncated"] > 100
    assert rel(e, gold["E"]) <= 1e-10
    assert grad_ok(grad, np.array(gold["grad"]))
    plan.free()


def test_c3_long_prefix_energy_grad_is_valid(ctx):
    """First 10000 gates of the 24-qubit D=128 workload (97 of its 1818
    parameters), checkpoints every 256 gates: 40 segments recomputed in three
    lane batches.  At the parity threshold 3123 of these gates truncate at D
    and 1299 of those cuts fall inside (nearly) degenerate pairs, where which
    of the equal values are kept is arbitrary: E_D is then fixed only up to
    rounding (the oracle with LAPACK's gesdd instead of gesvd moves it by
    1.8e-7 Ha) and g_D not at all (the same two oracle runs differ by 42 % of
    its largest entry).  So the test holds E_D to twice the oracle's driver
    spread, checks the bonds, the degenerate-cut count and a finite gradient,
    and leaves g_D unpinned here; the 2500-gate prefix pins it."""
    p, g = configs.load("c3")
    gold = golden()["c3_prefix_grad_long"]
    alt = golden()["c3_prefix_long_gesdd"]
    pre = Prefix(g, gold["gates"])
    plan = make_plan(ctx, p, pre, ckpt_gates=256)
    assert plan.n_theta == gold["n_theta"]
    e, grad, st = plan.energy_grad(p.theta[:plan.n_theta])
    spread = abs(alt["E"] - gold["E"])
    print(f"c3 long prefix: E error {abs(e - gold['E']):.2e} (oracle driver spread {spread:.2e}), "
          f"degenerate cuts {st['degenerate_cuts']} (oracle {alt['degenerate_cuts']}), "
          f"truncated gates {st['gates_truncated']}")
    assert st["max_bond"] == 128 and st["degenerate_cuts"] > 0 and alt["degenerate_cuts"] > 0
    assert abs(e - gold["E"]) <= 2.0 * spread
    assert np.all(np.isfinite(grad)) and np.abs(grad).max() > 0.0
    plan.free()


def test_sweep_limit_is_reported_as_nonconvergence(ctx):
    """With one Jacobi sweep allowed the SVDs cannot converge: MPS_ENOCONV and
    no outputs."""
    from paper_2211_07983_amd import MPSError
    from paper_2211_07983_amd._abi import MPS_ENOCONV
    p, g = configs.load("c1")
    plan = make_plan(ctx, p, g, max_sweeps=1)
    with pytest.raises(MPSError) as ei:
        plan.energy_grad(p.theta)
    assert ei.value.code == MPS_ENOCONV
    with pytest.raises(MPSError) as ei:
        plan.energy_grad_batched(np.stack([p.theta, p.theta]))
    assert ei.value.code == MPS_ENOCONV
    plan.free()


def test_batched_validation_errors(ctx):
    from paper_2211_07983_amd import MPSError
    from paper_2211_07983_amd._abi import MPS_EINVAL
    p, g = configs.load("c1")
    plan = make_plan(ctx, p, g)
    bad = np.stack([p.theta, p.theta])
    bad[1, 3] = np.nan
    for th in (bad, np.zeros((2, p.n_theta + 1)), np.zeros((0, p.n_theta))):
        with pytest.raises(MPSError) as ei:
            plan.energy_grad_batched(th)
        assert ei.value.code == MPS_EINVAL
    plan.free()


def test_checkpoint_interval_invariance(ctx):
    p, g = configs.load("c1")
    a = make_plan(ctx, p, g, ckpt_gates=7).energy_grad(p.theta)[1]
    b = make_plan(ctx, p, g, ckpt_gates=5000).energy_grad(p.theta)[1]
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()


def test_repeat_is_bitwise_deterministic(ctx):
    p, g = configs.load("c1")
    plan = make_plan(ctx, p, g)
    e1, g1, _ = plan.energy_grad(p.theta)
    e2, g2, _ = plan.energy_grad(p.theta)
    assert e1 == e2 and np.array_equal(g1, g2)


@pytest.mark.parametrize("seed", [1, 3])
def test_truncating_gradient_matches_oracle(ctx, seed):
    from oracle import mps
    p, g = configs.small(8, 4, 6, seed=seed, theta_sigma=0.3)
    E, grad, info = mps.energy_grad(p, g, p.theta)
    assert max(info["discarded"]) > 1e-3
    plan = make_plan(ctx, p, g)
    e, gg, st = plan.energy_grad(p.theta)
    assert rel(e, E) <= 1e-10
    assert grad_ok(gg, grad)


def test_energy_only_matches_energy_grad(ctx):
    p, g = configs.load("c1")
    plan = make_plan(ctx, p, g)
    e1, _ = plan.energy(p.theta)
    e2, _, _ = plan.energy_grad(p.theta)
    assert e1 == e2


def test_torch_autograd_function(ctx):
    torch = pytest.importorskip("torch")
    from paper_2211_07983_amd import EnergyGrad
    p, g = configs.load("c1")
    gold = golden()["c1"]
    plan = make_plan(ctx, p, g)
    th = torch.tensor(p.theta, dtype=torch.float64, device="cuda", requires_grad=True)
    E = EnergyGrad.apply(th, plan)
    (3.0 * E).backward()
    assert rel(E.item(), gold["E"]) <= 1e-10
    assert grad_ok(th.grad.cpu().numpy() / 3.0, np.array(gold["grad"]))


def test_gradient_validation_errors(ctx):
    from paper_2211_07983_amd import MPSError
    p, g = configs.load("c1")
    plan = make_plan(ctx, p, g)
    bad = p.theta.copy()
    bad[0] = np.inf
    with pytest.raises(MPSError) as ei:
        plan.energy_grad(bad)
    assert ei.value.code == -1
    with pytest.raises(MPSError) as ei:
        plan.energy_grad(p.theta[:-1])
    assert ei.value.code == -1


def test_broadened_svd_adjoint_matches_oracle(ctx):
    """C2 at eps = 1e-6 with the SVD adjoint's Lorentzian broadening (eta of
    d / (d^2 + eta^2), d = s_j^2 - s_i^2): against the oracle with the same
    eta, and visibly different from the unbroadened gradient, so a path that
    ignored eta would fail."""
    p, g = configs.load("c2", eps=configs.PAPER_EPS)
    gold = golden()["c2_paper_broaden"]
    plain = np.array(golden()["c2_paper"]["grad"])
    ref = np.array(gold["grad"])
    assert np.abs(ref - plain).max() > 1e-6 * np.abs(plain).max()
    plan = make_plan(ctx, p, g, ckpt_gates=512, broaden=gold["broaden"])
    e, grad, st = plan.energy_grad(p.theta)
    print(f"broadened: grad error {np.abs(grad - ref).max() / np.abs(ref).max():.2e}, "
          f"change from the plain gradient {np.abs(ref - plain).max() / np.abs(plain).max():.2e}")
    assert rel(e, gold["E"]) <= 1e-10
    assert grad_ok(grad, ref)
    plan.free()


def test_degenerate_cut_with_cotangent_is_reported(ctx):
    """A truncation through an exactly degenerate pair that carries a
    cotangent (the oracle raises there): strict_degenerate = 1 turns it into
    MPS_EDEGEN; by default the pair is dropped and the gradient is finite;
    so it is with broadening, whose Lorentzian is zero at d = 0."""
    import degenerate_case as dc
    from oracle import mps
    from paper_2211_07983_amd import MPSError
    p, g = dc.problem()
    with pytest.raises(mps.SVDDegenerate):
        mps.energy_grad(p, g, p.theta)
    plan = make_plan(ctx, p, g, strict_degenerate=1)
    with pytest.raises(MPSError, match="MPS_EDEGEN"):
        plan.energy_grad(p.theta)
    plan.free()
    for kw in ({}, {"broaden": 1e-6}):
        plan = make_plan(ctx, p, g, **kw)
        e, grad, st = plan.energy_grad(p.theta)
        assert st["degenerate_cuts"] == 1 and np.all(np.isfinite(grad))
        plan.free()
    # away from the degeneracy the strict plan evaluates
    plan = make_plan(ctx, p, g, strict_degenerate=1)
    plan.energy_grad(p.theta + 0.3)
    plan.free()
