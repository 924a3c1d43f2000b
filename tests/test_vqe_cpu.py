"""The VQE optimisation loops (host logic) against closed forms, and a full
BFGS run on the 8-qubit problem driven by the exact sector energy and
gradient of the oracle, checked against the variational bound set by the
sector's ground energy (Lanczos)."""
import numpy as np
import pytest

from oracle import sector as sec
from paper_2211_07983_amd import vqe
from vqe_inputs import configs


def quadratic(n=6, seed=0):
    rng = np.random.default_rng(seed)
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    lam = np.linspace(1.0, 4.0, n)
    A = Q @ np.diag(lam) @ Q.T
    b = rng.standard_normal(n)
    xs = np.linalg.solve(A, b)

    def fg(x):
        return 0.5 * float(x @ A @ x) - float(b @ x), A @ x - b
    return A, b, xs, fg


def test_gradient_descent_iterates_closed_form():
    """x_k - x* = (I - lr A)^k (x_0 - x*) on a quadratic."""
    A, b, xs, fg = quadratic()
    x0 = np.zeros(6)
    lr = 0.2
    r = vqe.gradient_descent(fg, x0, lr=lr, max_iter=7, e_tol=0.0, g_tol=0.0)
    M = np.linalg.matrix_power(np.eye(6) - lr * A, 7)
    assert r.iterations == 7 and r.reason == "max_iter"
    assert np.abs(r.theta - (xs + M @ (x0 - xs))).max() <= 1e-12
    assert len(r.energies) == 8 and r.evaluations == 8


def test_adam_first_step_closed_form():
    """After one step the bias-corrected moments give m/sqrt(v) = g/|g|
    elementwise: theta_1 = theta_0 - lr g/(|g| + eps)."""
    A, b, xs, fg = quadratic()
    x0 = np.full(6, 0.3)
    _, g0 = fg(x0)
    r = vqe.adam(fg, x0, lr=0.01, eps=1e-8, max_iter=1, e_tol=0.0, g_tol=0.0)
    assert np.abs(r.theta - (x0 - 0.01 * g0 / (np.abs(g0) + 1e-8))).max() <= 1e-15


def test_adam_and_bfgs_reach_the_quadratic_minimum():
    A, b, xs, fg = quadratic()
    r = vqe.bfgs(fg, np.zeros(6), e_tol=0.0, g_tol=1e-7, max_step=10.0)
    assert r.reason == "gradient"
    # |x - x*| <= |g| / lambda_min with lambda_min = 1
    assert np.abs(r.theta - xs).max() <= 1e-7
    assert r.iterations <= 20
    assert all(e1 <= e0 for e0, e1 in zip(r.energies, r.energies[1:]))
    ra = vqe.adam(fg, np.zeros(6), lr=0.05, e_tol=0.0, g_tol=1e-6, max_iter=5000)
    assert ra.reason == "gradient" and np.abs(ra.theta - xs).max() <= 1e-5


def test_bfgs_batched_line_search_matches_unbatched():
    """The batched trial evaluation is only a different way to call fg."""
    A, b, xs, fg = quadratic(seed=3)
    calls = []

    def fgb(ths):
        calls.append(len(ths))
        out = [fg(t) for t in ths]
        return np.array([o[0] for o in out]), np.stack([o[1] for o in out])
    r1 = vqe.bfgs(fg, np.ones(6), e_tol=0.0, g_tol=1e-9)
    r2 = vqe.bfgs(fg, np.ones(6), fg_batched=fgb, e_tol=0.0, g_tol=1e-9)
    assert np.array_equal(r1.theta, r2.theta) and r1.energies == r2.energies
    assert set(calls) == {4} and r2.evaluations == 1 + 4 * len(calls)


def test_stopping_rules():
    # stationary start: the gradient rule stops before any step
    r = vqe.bfgs(lambda x: (1.0, np.zeros(3)), np.ones(3))
    assert r.reason == "gradient" and r.iterations == 0
    # a step that changes E by less than 1e-6 stops on the energy rule
    r = vqe.gradient_descent(lambda x: (1e-7 * float(x @ x), np.ones(3)), np.zeros(3), lr=1e-3)
    assert r.reason == "energy" and r.iterations == 1
    # the paper's limits
    assert (vqe.MAX_ITER, vqe.E_TOL, vqe.G_TOL) == (100, 1e-6, 1e-5)


def test_bfgs_vqe_on_8_qubits_respects_the_variational_bound():
    """BFGS from the Hartree-Fock point (theta = 0) on the exact UCCSD energy
    of the 8-qubit problem: the energies decrease, the run ends on one of the
    paper's rules, and the final energy lies above the sector ground energy
    (variational principle) and below the Hartree-Fock energy."""
    p, _ = configs.load("c1")
    u = sec.UCCSD(p)
    e0 = u.ground_energy()          # the sector Hamiltonian holds the constant c0
    fg = lambda th: (u.energy(th), u.gradient(th))
    r = vqe.bfgs(fg, np.zeros(len(p.theta)))
    e_hf = r.energies[0]
    print(f"8 q BFGS: {r.iterations} iterations ({r.reason}), E {r.energy:.10f}, "
          f"ground {e0:.10f}, gap {r.energy - e0:.2e}, HF {e_hf:.6f}")
    assert r.reason in ("energy", "gradient")
    assert all(e1 <= e0_ + 1e-14 for e0_, e1 in zip(r.energies, r.energies[1:]))
    assert r.energy >= e0 - 1e-9
    assert r.energy < e_hf


def test_invalid_settings_are_refused():
    A, b, xs, fg = quadratic()
    with pytest.raises(ValueError):
        vqe.bfgs(fg, np.zeros(6), n_trial=0)
    with pytest.raises(ValueError):
        vqe.gradient_descent(fg, np.zeros(6), lr=0.0)
    with pytest.raises(ValueError):
        vqe.adam(fg, np.zeros(6), beta1=1.0)


class _PlanStub:
    """Stands in for a Plan: the fixed-rank gradient of a product state (zero
    at theta = 0, the quadratic's gradient elsewhere) and an Algorithm 1
    gradient (the quadratic's gradient everywhere); counts the calls."""

    def __init__(self, fg):
        self.fg = fg
        self.calls = {"local": 0, "batched": 0, "alg1": 0}

    def energy_grad(self, th):
        self.calls["local"] += 1
        e, g = self.fg(th)
        return e, (np.zeros_like(g) if not np.any(th) else g), {}

    def energy_grad_batched(self, ths):
        self.calls["batched"] += 1
        out = [self.energy_grad(t) for t in ths]
        return np.array([o[0] for o in out]), np.stack([o[1] for o in out]), {}

    def energy_grad_alg1(self, th, strings_per_group=1):
        self.calls["alg1"] += 1
        assert strings_per_group == 4
        e, g = self.fg(th)
        return e, g, None, {}


def test_minimize_from_a_product_state_uses_algorithm_1_or_raises():
    A, b, xs, fg = quadratic()
    x0 = np.zeros(6)
    with pytest.raises(ValueError, match="exactly zero"):
        vqe.minimize(_PlanStub(fg), x0, "bfgs", gradient="local")
    with pytest.raises(ValueError, match="unknown gradient"):
        vqe.minimize(_PlanStub(fg), x0, "bfgs", gradient="exact")
    for grad in ("auto", "alg1"):
        stub = _PlanStub(fg)
        r = vqe.minimize(stub, x0, "bfgs", gradient=grad, e_tol=0.0, g_tol=1e-7, max_step=10.0)
        assert r.reason == "gradient" and np.abs(r.theta - xs).max() <= 1e-7
        assert stub.calls["alg1"] == r.evaluations and stub.calls["batched"] == 0
        assert stub.calls["local"] == (1 if grad == "auto" else 0)
    # a generic start keeps the local gradient and the batched line search
    stub = _PlanStub(fg)
    r = vqe.minimize(stub, np.full(6, 0.1), "bfgs", e_tol=0.0, g_tol=1e-7, max_step=10.0)
    assert r.reason == "gradient" and stub.calls["alg1"] == 0 and stub.calls["batched"] > 0
