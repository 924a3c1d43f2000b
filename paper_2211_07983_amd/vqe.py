"""VQE optimisation loops over the engine's energy and gradient (Sec. 5).

The paper minimises E(theta) from the Hartree-Fock start with gradient
descent and BFGS on its back-propagated gradient.  Its stopping rules for
these gradient-based runs (Sec. 5, the caption of the optimiser-convergence
figure): at most 100 iterations; stop as soon as the energy changes by less
than 1e-6 between two successive iterations or the gradient norm drops below
1e-5.  Adam (Kingma and Ba, 2015) is included as the usual first-order
alternative.

The loops are host logic: every energy and gradient comes from the caller's
function, normally ``Plan.energy_grad`` (one vector) and
``Plan.energy_grad_batched`` (a batch of vectors in one launch).  BFGS uses
the batch for its line search: all trial step lengths of an iteration are
evaluated together, since a batched launch of a few vectors costs about as
much wall time as a single evaluation, and the largest step that meets the
Armijo condition is taken.  The inverse-Hessian update is the standard one
(Nocedal and Wright, Numerical Optimization, eq. 6.17); it is skipped when
the curvature s.y is not positive, which keeps the matrix positive definite.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MAX_ITER = 100
E_TOL = 1e-6
G_TOL = 1e-5


@dataclass
class Result:
    theta: np.ndarray
    energy: float
    grad: np.ndarray
    iterations: int
    reason: str                     # "energy", "gradient", "max_iter" or "line_search"
    energies: list = field(default_factory=list)     # E at the start and after every iteration
    grad_norms: list = field(default_factory=list)
    evaluations: int = 0            # energy+gradient evaluations (batched ones counted per vector)


def _stop(e_prev, e, g, e_tol, g_tol):
    if np.linalg.norm(g) < g_tol:
        return "gradient"
    if e_prev is not None and abs(e - e_prev) < e_tol:
        return "energy"
    return None


def gradient_descent(fg, theta0, lr=0.05, max_iter=MAX_ITER, e_tol=E_TOL, g_tol=G_TOL):
    """theta <- theta - lr * grad with a fixed step.  fg(theta) -> (E, grad)."""
    if lr <= 0.0:
        raise ValueError("lr must be > 0")
    th = np.array(theta0, dtype=np.float64)
    e, g = fg(th)
    res = Result(th, e, g, 0, "max_iter", [e], [float(np.linalg.norm(g))], 1)
    reason = _stop(None, e, g, e_tol, g_tol)
    it = 0
    while reason is None and it < max_iter:
        th = th - lr * g
        e_prev = e
        e, g = fg(th)
        it += 1
        res.energies.append(e)
        res.grad_norms.append(float(np.linalg.norm(g)))
        res.evaluations += 1
        reason = _stop(e_prev, e, g, e_tol, g_tol)
    res.theta, res.energy, res.grad, res.iterations = th, e, g, it
    res.reason = reason or "max_iter"
    return res


def adam(fg, theta0, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8, max_iter=MAX_ITER, e_tol=E_TOL, g_tol=G_TOL):
    """Adam with bias-corrected first and second moments."""
    if lr <= 0.0 or not 0.0 <= beta1 < 1.0 or not 0.0 <= beta2 < 1.0:
        raise ValueError("need lr > 0 and 0 <= beta1, beta2 < 1")
    th = np.array(theta0, dtype=np.float64)
    e, g = fg(th)
    res = Result(th, e, g, 0, "max_iter", [e], [float(np.linalg.norm(g))], 1)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    reason = _stop(None, e, g, e_tol, g_tol)
    it = 0
    while reason is None and it < max_iter:
        it += 1
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        mh = m / (1.0 - beta1 ** it)
        vh = v / (1.0 - beta2 ** it)
        th = th - lr * mh / (np.sqrt(vh) + eps)
        e_prev = e
        e, g = fg(th)
        res.energies.append(e)
        res.grad_norms.append(float(np.linalg.norm(g)))
        res.evaluations += 1
        reason = _stop(e_prev, e, g, e_tol, g_tol)
    res.theta, res.energy, res.grad, res.iterations = th, e, g, it
    res.reason = reason or "max_iter"
    return res


def bfgs(fg, theta0, fg_batched=None, n_trial=4, shrink=0.5, c1=1e-4, max_step=1.0,
         max_iter=MAX_ITER, e_tol=E_TOL, g_tol=G_TOL):
    """BFGS on the inverse Hessian with a batched backtracking line search.

    fg(theta) -> (E, grad) gives the starting point; fg_batched(thetas[k, n])
    -> (E[k], grads[k, n]) evaluates the trial points theta + a_i p,
    a_i = a0 * shrink**i for i < n_trial, in one call (without it, fg is
    called per trial).  a0 = 1, capped so that |a0 p| <= max_step.  The largest
    a_i with E(a_i) <= E + c1 a_i (g.p) is taken; if none qualifies the search
    restarts from the smallest trial step with the Hessian reset to the
    identity, and a second failure ends the run ("line_search")."""
    if n_trial < 1 or not 0.0 < shrink < 1.0 or not 0.0 < c1 < 1.0 or max_step <= 0.0:
        raise ValueError("need n_trial >= 1, 0 < shrink < 1, 0 < c1 < 1 and max_step > 0")
    th = np.array(theta0, dtype=np.float64)
    n = th.size
    e, g = fg(th)
    res = Result(th, e, g, 0, "max_iter", [e], [float(np.linalg.norm(g))], 1)
    if fg_batched is None:
        def fg_batched(ths):
            out = [fg(t) for t in ths]
            return np.array([o[0] for o in out]), np.stack([o[1] for o in out])
    H = np.eye(n)
    reason = _stop(None, e, g, e_tol, g_tol)
    it = 0
    a_start = 1.0
    failed = False
    while reason is None and it < max_iter:
        p = -H @ g
        slope = float(g @ p)
        if slope >= 0.0:            # not a descent direction: restart from steepest descent
            H = np.eye(n)
            p = -g
            slope = float(g @ p)
        a0 = min(a_start, max_step / max(np.linalg.norm(p), 1e-300))
        alphas = a0 * shrink ** np.arange(n_trial)
        es, gs = fg_batched(th[None, :] + alphas[:, None] * p[None, :])
        res.evaluations += n_trial
        ok = np.nonzero(es <= e + c1 * alphas * slope)[0]
        if ok.size == 0:
            if failed:
                reason = "line_search"
                break
            failed = True
            H = np.eye(n)
            a_start = alphas[-1] * shrink
            continue
        failed = False
        a_start = 1.0
        i = int(ok[0])
        s = alphas[i] * p
        th_new, e_new, g_new = th + s, float(es[i]), gs[i]
        y = g_new - g
        sy = float(s @ y)
        if sy > 0.0:
            rho = 1.0 / sy
            Hy = H @ y
            # (I - rho s y^T) H (I - rho y s^T) + rho s s^T, expanded
            H = H - rho * (np.outer(s, Hy) + np.outer(Hy, s)) + (rho * rho * float(y @ Hy) + rho) * np.outer(s, s)
        e_prev = e
        th, e, g = th_new, e_new, g_new
        it += 1
        res.energies.append(e)
        res.grad_norms.append(float(np.linalg.norm(g)))
        reason = _stop(e_prev, e, g, e_tol, g_tol)
    res.theta, res.energy, res.grad, res.iterations = th, e, g, it
    res.reason = reason or "max_iter"
    return res


GRADIENTS = ("auto", "local", "alg1")


def minimize(plan, theta0, method="bfgs", gradient="auto", strings_per_group=4, **kw):
    """Runs one of the loops on a Plan with energies and gradients from the GPU.

    gradient selects the derivative:
    - "local": the back-propagated fixed-rank gradient (Plan.energy_grad; the
      BFGS line search through Plan.energy_grad_batched).  At a product state
      such as the Hartree-Fock start theta = 0 it is exactly zero in every
      direction that would raise a bond's rank (the directions below the
      truncation are absent), so a run from there would stop at once; this
      choice raises ValueError when the starting gradient is exactly zero.
    - "alg1": the paper's Algorithm 1 with the Hamiltonian split into groups of
      strings_per_group strings (Plan.energy_grad_alg1; Sec. 5 runs its
      optimiser with four strings per group), exact in those directions.
    - "auto": "local", unless the starting local gradient is exactly zero;
      then the whole run uses "alg1"."""
    if gradient not in GRADIENTS:
        raise ValueError(f"unknown gradient {gradient!r} (one of {GRADIENTS})")
    if gradient != "alg1":
        e0, g0, _ = plan.energy_grad(np.asarray(theta0, dtype=np.float64))
        if not np.any(g0):
            if gradient == "local":
                raise ValueError("the fixed-rank gradient is exactly zero at theta0 (a product state such as the "
                                 "Hartree-Fock start); use gradient='alg1' or a generic theta0")
            gradient = "alg1"
    if gradient == "alg1":
        def fg(th):
            e, g, _, _ = plan.energy_grad_alg1(th, strings_per_group)
            return e, g
        if method == "bfgs":
            return bfgs(fg, theta0, **kw)
        if method == "gd":
            return gradient_descent(fg, theta0, **kw)
        if method == "adam":
            return adam(fg, theta0, **kw)
        raise ValueError(f"unknown method {method!r}")

    def fg(th):
        e, g, _ = plan.energy_grad(th)
        return e, g

    if method == "bfgs":
        def fgb(ths):
            es, gs, _ = plan.energy_grad_batched(np.ascontiguousarray(ths))
            return np.asarray(es), np.asarray(gs)
        return bfgs(fg, theta0, fg_batched=fgb, **kw)
    if method == "gd":
        return gradient_descent(fg, theta0, **kw)
    if method == "adam":
        return adam(fg, theta0, **kw)
    raise ValueError(f"unknown method {method!r}")
