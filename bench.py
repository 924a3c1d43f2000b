#!/usr/bin/env python3
"""Benchmark: energy + gradient evaluations per second of the UCCSD-MPS hot path
on one MI355X.

Workloads (seeded synthetic problems, see vqe_inputs/configs.py):
  c2 (default): 14 qubits (7 orbitals, 10 electrons), D = 64, 3381 Pauli
      terms, 140 parameters, 16899 compiled nearest-neighbour gates;
  c3: 24 qubits (12 orbitals, 12 electrons), D = 128, 29736 terms, 1818
      parameters, 428183 gates.  One evaluation is a chain of ~4.3e5
      dependent 256x256 SVDs (about 10 ms each on one GPU), i.e. hours: run it
      explicitly with --workload c3.
Truncation threshold eps = 1e-6 by default (the paper's setting, Sec. 5).

The whole run keeps to a wall-time budget (--budget-s, from process start):
warm-ups and timed steps start only while the slowest step so far still fits,
after the share held back for the CPU baseline; `steps` and `warmup` in the
line count the ones that ran (the requested counts are in `config`).

One step = --batch complete evaluations of the hot path, for --batch seeded
parameter vectors (the configured theta and perturbations of it): product
state, every compiled gate (contraction, one-sided Jacobi SVD, site update)
with a checkpoint every --ckpt-gates gates, the Pauli-term sweeps and the
compensated energy sum, then the reverse pass (sweep adjoint, segment
recompute with tape, gate adjoints, chain rule).  With --batch > 1 the vectors
go through the circuit together (mps_energy_grad_batched); `value` is the
whole-step throughput.  The single-vector path (mps_energy_grad) is timed as
well and reported as `single`.  Inputs are resident on the device before the
timed region.

Prints one JSON line on stdout; progress lines go to stderr.  The roofline
object refers to the dominant kernel, the persistent gate chain (one
cooperative launch per checkpoint segment, whose time is almost all Jacobi
SVD), timed with HIP events around its launches on the stream it runs on; the
CPU baseline times the FP64 oracle on the same workload on the host cores,
with BLAS on one thread and on the host's usable cores (nproc setting).

--phase sweep measures the Pauli-sweep phase alone (S5 + S6: identity
environments, every term's transfers, the compensated energy sum) on the
state after the first --prefix-gates gates of the workload, in plain FP64 and
in precision mode 1 (transfers as complex FP32 products on the matrix cores),
and prints its own JSON line with the matrix-core roofline of that phase.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

T_START = time.monotonic()   # wall-time budget of the whole run counts from here
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 (vector and matrix): 256 CU x 2.4 GHz x 128 flop/clk
PEAK_FP32_MFMA_TFLOPS = 157.3   # MI355X dense FP32 matrix: 256 CU x 2.4 GHz x 256 flop/clk
METRIC = "energy+grad evals/s (UCCSD-MPS 24q D=128) vs plain FP64; MFMA util %"
WORKLOADS = {
    "c1": "UCCSD-MPS 8 qubits (4 orbitals, 4 electrons), D=16",
    "c3": "UCCSD-MPS 24 qubits (12 orbitals, 12 electrons), D=128",
    "c2": "UCCSD-MPS 14 qubits (7 orbitals, 10 electrons), D=64",
}
# What a line of each workload stands for next to the metric's own
# configuration (24 qubits, D = 128).
WORKLOAD_NOTE = {
    "c2": "not the metric's 24-qubit D=128 configuration: one evaluation there is a chain of 428183 dependent "
          "SVDs (up to 256x256) that does not finish within a benchmark run; this is the 14-qubit D=64 "
          "configuration, the largest whose evaluation takes seconds",
    "c3": "the metric's configuration",
    "c1": "not the metric's configuration: the 8-qubit D=16 case",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    except Exception:
        return int(os.environ.get("OMP_NUM_THREADS", "1"))


def host_info():
    """Core counts and CPU model of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        libs = [f"{d.get('internal_api')}:{d.get('num_threads')}" for d in threadpool_info()]
    except Exception:
        libs = []
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS"), "thread_pools": libs}


def nproc_threads():
    """Threads of the nproc setting: the CPUs this process may run on, capped
    by OMP_NUM_THREADS when it is set (the host's share for this GPU)."""
    n = host_info()["usable_cpus"]
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def cpu_baseline_full(prob, gates, eps):
    """The FP64 oracle (T3) on the whole workload: one energy + gradient."""
    from oracle import mps as T3
    t0 = time.perf_counter()
    T3.energy_grad(prob, gates, prob.theta, D=prob.bond_dim, eps=eps, ckpt=256)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "evals/s", "cores": blas_threads(), "kind": "oracle",
            "sample": f"T3 FP64 oracle (NumPy/SciPy gesvd), one complete energy+gradient of the same workload "
                      f"({gates.n_gates} gates, {prob.n_terms} terms, eps={eps:g}): {dt:.1f} s",
            "seconds_per_eval": dt}


def cpu_baseline_settings(workload, eps, deadline):
    """The oracle in the two settings of the timing protocol: BLAS on one thread
    and on nproc threads (the whole evaluation for c1/c2, else the bounded
    sample), each in a child process whose thread count is fixed by the
    environment before NumPy loads (changing a loaded BLAS's pool in flight has
    crashed long oracle runs).  Each child is limited to what is left until
    `deadline` (time.monotonic), at least 15 s: on these small matrices many
    BLAS threads are far slower than one, and a setting that does not finish
    in time is listed with that error.  `value`/`cores` are the faster
    setting's; both are listed under `settings` with the host's core count and
    CPU model."""
    import subprocess
    runs = []
    mode = "full" if workload in ("c1", "c2") else "sample"
    for n in (1, nproc_threads()):
        if runs and n == runs[0]["requested_threads"]:
            break
        env = dict(os.environ, OPENBLAS_NUM_THREADS=str(n), OMP_NUM_THREADS=str(n), MKL_NUM_THREADS=str(n))
        cmd = [sys.executable, os.path.abspath(__file__), "--cpu-child", mode, "--workload", workload,
               "--eps", repr(eps)]
        timeout_s = max(15.0, min(150.0, deadline - time.monotonic()))
        try:
            p = subprocess.run(cmd, env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                               timeout=timeout_s)
            if p.returncode != 0:
                raise RuntimeError(f"exit {p.returncode}: {p.stderr.strip()[-300:]}")
            r = json.loads(p.stdout.strip().splitlines()[-1])
        except Exception as exc:   # a failed setting is reported, not fatal to the line
            log(f"cpu baseline with {n} thread(s) failed: {exc}")
            runs.append({"requested_threads": n, "mode": mode, "error": str(exc)[:300]})
            continue
        r["requested_threads"] = n
        r["mode"] = mode
        log(f"cpu baseline, {n} requested / {r['cores']} reported BLAS thread(s), {mode}: {r['value']:.3e} evals/s "
            f"({r['seconds_per_eval']:.1f} s/eval); pools {r['thread_pools']}")
        runs.append(r)
    ok = [r for r in runs if "value" in r]
    if not ok:
        return None
    out = dict(max(ok, key=lambda r: r["value"]))
    out["settings"] = [{k: r[k] for k in ("cores", "requested_threads", "mode", "value", "seconds_per_eval",
                                          "thread_pools", "error") if k in r} for r in runs]
    out["host"] = host_info()
    return out


def cpu_child(args):
    """--cpu-child full|sample: one CPU-baseline setting of the workload (the
    whole evaluation, or the bounded sample); prints one JSON line.  Touches
    no GPU."""
    from vqe_inputs import configs
    prob, gates = configs.load(args.workload, eps=args.eps)
    if args.cpu_child == "full":
        r = cpu_baseline_full(prob, gates, prob.eps)
    else:
        r = cpu_baseline_sample(prob, gates, prob.eps)
    r["thread_pools"] = host_info()["thread_pools"]
    print(json.dumps(r), flush=True)


def cpu_baseline_sample(prob, gates, eps, budget_s=25.0):
    """The FP64 oracle (T3) on a bounded sample, scaled to one evaluation.

    Sample: a random right-canonical MPS with the saturated bond dimensions of the
    workload; gates on the middle bonds (forward with tape and gate adjoint, all
    full-size SVDs) and a few hundred Pauli terms (energy and sweep adjoint).
    Per evaluation: G * (2 t_gate + t_adjoint) + K * (t_term + t_term_adjoint).
    """
    import numpy as np
    from oracle import mps as T3
    rng = np.random.default_rng(12345)
    N, D = prob.n_qubits, prob.bond_dim
    dims = [1] + [min(2 ** (n + 1), 2 ** (N - n - 1), D) for n in range(N - 1)] + [1]
    m = T3.MPS(prob.occ)
    for n in range(N):
        a, b = dims[n], dims[n + 1]
        X = rng.normal(size=(a, 2 * b)) + 1j * rng.normal(size=(a, 2 * b))
        q, _ = np.linalg.qr(X.conj().T)          # 2b x a, orthonormal columns
        m.B[n] = q.conj().T.reshape(a, 2, b)
        lam = np.sort(rng.random(b))[::-1] ** 4
        m.lam[n + 1] = lam / np.linalg.norm(lam)
    mid = N // 2
    t_gate, t_adj, n_g = 0.0, 0.0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.45 * budget_s and n_g < 64:
        n = mid - 2 + (n_g % 4)
        g = int(np.nonzero(gates.bond == n)[0][n_g % 10])
        Q, dQ = T3.gate_mats(gates, g, prob.theta)
        tape = []
        saved = (m.B[n].copy(), m.B[n + 1].copy(), m.lam[n + 1].copy())
        t1 = time.perf_counter()
        m.apply_gate(n, Q, D, eps, tape)
        t2 = time.perf_counter()
        T3.gate_backward(tape[0], Q, dQ, rng.normal(size=m.B[n].shape) + 0j,
                         rng.normal(size=m.B[n + 1].shape) + 0j, rng.normal(size=len(m.lam[n + 1])), check=0.0)
        t3 = time.perf_counter()
        m.B[n], m.B[n + 1], m.lam[n + 1] = saved
        t_gate += t2 - t1
        t_adj += t3 - t2
        n_g += 1
    t_gate /= n_g
    t_adj /= n_g
    K = prob.n_terms
    idx = rng.choice(K, size=min(K, 400), replace=False)
    L, R = m.identity_envs()
    t0 = time.perf_counter()
    n_t = 0
    for k in idx:
        m.term_values(prob.ham_x[k:k + 1], prob.ham_z[k:k + 1], (L, R))
        n_t += 1
        if time.perf_counter() - t0 > 0.25 * budget_s:
            break
    t_term = (time.perf_counter() - t0) / n_t
    t0 = time.perf_counter()
    n_c = 0
    for k in idx:
        m.energy_cotangents(prob.ham_x[k:k + 1], prob.ham_z[k:k + 1], prob.ham_c[k:k + 1], 0.0)
        n_c += 1
        if time.perf_counter() - t0 > 0.25 * budget_s:
            break
    t_cot = (time.perf_counter() - t0) / n_c
    G = gates.n_gates
    per_eval = G * (2 * t_gate + t_adj) + K * (t_term + t_cot)
    sample = (f"T3 FP64 oracle (NumPy/SciPy gesvd) on a random right-canonical MPS with the saturated bond dims of "
              f"the workload: {n_g} middle-bond gate updates with tape + gate adjoints ({2 * dims[mid]}x"
              f"{2 * dims[mid + 1]} SVDs), {n_t} + {n_c} of {K} Pauli terms (energy, naive sweep adjoint); scaled to "
              f"{G} gates x (forward + recompute + adjoint) + {K} terms per evaluation; t_gate={t_gate*1e3:.1f} ms, "
              f"t_adj={t_adj*1e3:.1f} ms, t_term={t_term*1e3:.2f} ms, t_term_adj={t_cot*1e3:.2f} ms")
    return {"value": 1.0 / per_eval, "unit": "evals/s", "cores": blas_threads(), "kind": "oracle", "sample": sample,
            "seconds_per_eval": per_eval}


# HBM traffic per launch of the dominant kernels, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE) of the default commands, each scaled by what the
# counter reads for a 1 GiB device copy in the same run (FETCH_SIZE reads 0.5 GiB
# for it: factor 2.0; WRITE_SIZE reads 1 GiB: factor 1.0).  Keyed by the SHA-256
# prefix of the kernel source the counters were taken on: a changed source
# reports null.
TRAFFIC = {
    ("evalgrad", "c2"): {"source": "paper_2211_07983_amd/csrc/gate.hip", "sha": "6be98bfd8f61f429",
                         "fetch_bytes": 4.489e9, "write_bytes": 116.811e9,
                         "per": "forward launch of k_chain_lanes<16>, 64 lanes x 512 gates (mean of the 34 launches "
                                "of a step, 7 of which keep their tapes)"},
    ("sweep", "c3"): {"source": "paper_2211_07983_amd/csrc/sweep32.hip", "sha": "9313886d959f9260",
                      "fetch_bytes": 276.64e9, "write_bytes": 106.78e9,
                      "per": "one sweep (all k_left1_f32 + k_left2_f32 dispatches)"},
}


def traffic_for(phase, workload):
    import hashlib
    t = TRAFFIC.get((phase, workload))
    if t is None:
        return None, None
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest()[:16] != t["sha"]:
            return None, None
    return t["fetch_bytes"] + t["write_bytes"], t


def calibration_copy(mib):
    """One elementwise device copy of `mib` MiB (reads and writes mib MiB)."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"calibration copy: {mib} MiB read, {mib} MiB written")
    del src, dst


def sweep_cmacs(dims, hx, hz):
    """Complex multiply-adds of one sweep: every (term, site) transfer is two
    GEMMs, a*a*2b + 2a*b*b = 2ab(a+b) with a, b the bonds left and right of the
    site; the left and right identity environments add one transfer per site
    each."""
    N = len(dims) - 1
    per_site = [2 * dims[n] * dims[n + 1] * (dims[n] + dims[n + 1]) for n in range(N)]
    active = [0] * (N + 1)
    for x, z in zip(hx, hz):
        m = int(x) | int(z)
        active[(m & -m).bit_length() - 1] += 1
        active[m.bit_length()] -= 1
    total, run = 0, 0
    for n in range(N):
        run += active[n]
        total += run * per_site[n]
    return total + 2 * sum(per_site)


class _GatePrefix:
    def __init__(self, gl, count):
        self.n_qubits = gl.n_qubits
        for f in ("bond", "kind", "pre", "post", "param", "coeff"):
            setattr(self, f, getattr(gl, f)[:count])


def sweep_phase(args):
    import numpy as np
    from vqe_inputs import configs
    from paper_2211_07983_amd import Context, State
    prob, gates = configs.load(args.workload, eps=args.eps)
    G = min(args.prefix_gates, gates.n_gates)
    pre = _GatePrefix(gates, G)
    ctx = Context(0)
    res = {}
    for prec in (0, 1):
        st = State.product(ctx, prob.occ, prob.bond_dim, prob.eps, precision=prec)
        t = time.perf_counter()
        st.apply_circuit(pre, prob.theta)
        log(f"precision {prec}: {G} gates applied in {time.perf_counter() - t:.1f}s")
        e, _, _ = st.expect(prob.n_qubits, prob.ham_x, prob.ham_z, prob.ham_c, prob.c0)   # warm-up
        times = []
        for _ in range(max(1, args.steps)):
            e, _, s = st.expect(prob.n_qubits, prob.ham_x, prob.ham_z, prob.ham_c, prob.c0)
            times.append(s["t_sweep_ms"])
        dims = [int(d) for d in st.export()[0]]
        res[prec] = dict(E=e, ms=float(np.median(times)), dims=dims)
        log(f"precision {prec}: sweep {res[prec]['ms']:.1f} ms (median of {len(times)}), E={e:.12f}")
        st.free()
    dims = res[0]["dims"]
    cmac = sweep_cmacs(dims, prob.ham_x, prob.ham_z)
    ms32 = res[1]["ms"]
    eff = 8.0 * cmac / (ms32 * 1e-3) / 1e12
    line = {
        "metric": "Pauli-sweep energy evaluations/s (all terms, S5+S6), precision 1 vs plain FP64",
        "value": 1e3 / ms32, "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": ms32, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-mfma (FP64 term sums)", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] + f", eps={prob.eps:g}, K={prob.n_terms} Pauli terms, "
                               f"state after the first {G} gates", "bonds": dims,
                   "fp64_ms": res[0]["ms"], "speedup_vs_fp64": res[0]["ms"] / ms32,
                   "energy_error_ha": abs(res[1]["E"] - res[0]["E"]), "E_fp64": res[0]["E"]},
        "roofline": {"kernel": "k_left1_f32 + k_left2_f32 (whole sweep phase)", "bound": "mfma",
                     "achieved": eff, "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": eff / PEAK_FP32_MFMA_TFLOPS, "traffic": traffic_for("sweep", args.workload)[0],
                     "issued_tflops": 0.75 * eff, "cmac_per_sweep": cmac,
                     "fp64_achieved": 8.0 * cmac / (res[0]["ms"] * 1e-3) / 1e12},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def psr_phase(args):
    """Gradient by the parameter-shift rule (2M + 1 batched forward evaluations)
    against back-propagation (one forward + reverse pass) on the same plan."""
    import numpy as np
    from vqe_inputs import configs
    from paper_2211_07983_amd import Context, Plan
    prob, gates = configs.load(args.workload, eps=args.eps)
    ctx = Context(0)
    plan = Plan(ctx, prob.occ, gates, prob.n_qubits, prob.ham_x, prob.ham_z, prob.ham_c, prob.c0,
                prob.bond_dim, prob.eps, ckpt_gates=args.ckpt_gates)
    M = int((np.asarray(gates.kind) == 1).sum())
    plan.energy_grad(prob.theta)                       # warm-up
    t0 = time.perf_counter()
    e_bp, g_bp, _ = plan.energy_grad(prob.theta)
    t_bp = time.perf_counter() - t0
    t0 = time.perf_counter()
    e_ps, g_ps, _, st = plan.energy_grad_psr(prob.theta)
    t_ps = time.perf_counter() - t0
    log(f"back-propagation {t_bp:.3f}s, parameter shift {t_ps:.3f}s ({2 * M + 1} evaluations)")
    diff = float(np.abs(g_ps - g_bp).max() / max(1e-300, np.abs(g_bp).max()))
    line = {
        "metric": "gradient time, parameter shift / back-propagation (same plan, one GPU)",
        "value": t_ps / t_bp, "unit": "ratio", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * t_ps, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] + f", eps={prob.eps:g}, {gates.n_gates} NN gates, "
                               f"M={M} parametric gates, n_theta={prob.n_theta}",
                   "t_backprop_s": t_bp, "t_psr_s": t_ps, "psr_evaluations": 2 * M + 1,
                   "psr_lanes_per_launch": plan.lanes_per_launch(),
                   "max_rel_grad_diff": diff, "E": e_bp},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def vqe_phase(args):
    """A VQE run: BFGS with the paper's stopping rules, every energy and
    gradient from the GPU; the line search evaluates its trial steps as one
    batched launch.  It starts from the workload's seeded theta, not from the
    Hartree-Fock point theta = 0, where the state is a product state and the
    gradient through the truncated SVDs is the fixed-rank one (zero)."""
    import numpy as np
    from vqe_inputs import configs
    from paper_2211_07983_amd import Context, Plan, vqe
    prob, gates = configs.load(args.workload, eps=args.eps)
    ctx = Context(0)
    plan = Plan(ctx, prob.occ, gates, prob.n_qubits, prob.ham_x, prob.ham_z, prob.ham_c, prob.c0,
                prob.bond_dim, prob.eps, ckpt_gates=args.ckpt_gates)
    th0 = np.array(prob.theta)
    plan.energy_grad(th0)                              # warm-up
    t0 = time.perf_counter()
    r = vqe.minimize(plan, th0, "bfgs", max_iter=args.vqe_iters)
    dt = time.perf_counter() - t0
    log(f"BFGS: {r.iterations} iterations ({r.reason}) in {dt:.2f}s, E {r.energies[0]:.8f} -> {r.energy:.8f}")
    line = {
        "metric": "VQE BFGS iterations/s (energy+gradient on the GPU, batched line search)",
        "value": r.iterations / dt, "unit": "iterations/s", "n_gpus": 1, "steps": r.iterations, "warmup": 1,
        "ms_per_step": 1e3 * dt / max(1, r.iterations), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] + f", eps={prob.eps:g}, {gates.n_gates} NN gates, "
                               f"n_theta={prob.n_theta}, start: the seeded theta",
                   "stop": r.reason, "evaluations": r.evaluations, "E_start": r.energies[0], "E_final": r.energy,
                   "grad_norm_final": float(np.linalg.norm(r.grad)), "seconds": dt},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def instances_phase(args):
    """The batched-instance set, one size class: the instances with
    args.class_qubits qubits and D = args.class_d (one compiled circuit, a
    seeded Hamiltonian and theta each) evaluated as lanes of shared gate-chain
    launches (mps_energy_grad_multi), against the same instances evaluated one
    after another on the plain FP64 path."""
    import numpy as np
    from vqe_inputs import configs
    from vqe_inputs.compile import compile_problem
    from vqe_inputs.problem import make_problem
    from paper_2211_07983_amd import Context, Plan, energy_grad_multi
    members = [i for i, (n, ne, D, s1, s2) in enumerate(configs.batched_instances())
               if n == args.class_qubits and D == args.class_d]
    if not members:
        raise SystemExit(f"no instance with {args.class_qubits} qubits and D={args.class_d}")
    ctx = Context(0)
    probs, plans = [], []
    for i in members:
        n, ne, D, s1, s2 = configs.batched_instances()[i]
        p = make_problem(f"c4_{i}", n, ne, D, args.eps, s1, s2, 0.05)
        g = compile_problem(p)
        probs.append(p)
        plans.append(Plan(ctx, p.occ, g, p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, p.bond_dim, p.eps,
                          ckpt_gates=args.ckpt_gates))
    thetas = np.stack([p.theta for p in probs])
    log(f"class {args.class_qubits} q, D={args.class_d}: instances {members}, {g.n_gates} gates each")
    t0 = time.perf_counter()
    e_m, g_m, st = energy_grad_multi(plans, thetas)
    t_multi = time.perf_counter() - t0
    log(f"one call: {len(plans)} instances in {t_multi:.2f}s")
    t0 = time.perf_counter()
    worst = 0.0
    for k, (pl, p) in enumerate(zip(plans, probs)):
        e1, g1, _ = pl.energy_grad(p.theta)
        worst = max(worst, abs(e1 - e_m[k]) / abs(e1), float(np.abs(g1 - g_m[k]).max() / np.abs(g1).max()))
    t_seq = time.perf_counter() - t0
    log(f"one after another: {t_seq:.2f}s; max relative difference {worst:.1e}")
    line = {
        "metric": "instance energy+grad evals/s, one size class of the batched-instance set in shared launches",
        "value": len(plans) / t_multi, "unit": "instance-evals/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * t_multi, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded per-instance integrals and theta)",
        "config": {"workload": f"batched-instance set, class {args.class_qubits} qubits D={args.class_d}: "
                               f"{len(plans)} instances, {g.n_gates} NN gates, n_theta={probs[0].n_theta}, "
                               f"eps={args.eps:g}",
                   "instances": members, "sequential_evals_per_s": len(plans) / t_seq,
                   "speedup_vs_sequential": t_seq / t_multi, "max_rel_diff_vs_single": worst,
                   "max_bond": st["max_bond"]},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def mixed_phase(args):
    """The batched-instance set across size classes: every instance with at
    most args.max_qubits qubits (its own circuit, D and Hamiltonian) in one
    mps_energy_grad_plans call, whose lanes share the gate-chain launches.
    The sequential reference evaluates one instance per (qubits, D) class on
    its own and weights it by the class's count (a sample, stated in the
    line); the full sequential run is the sum of those per-class times."""
    import numpy as np
    from vqe_inputs import configs
    from vqe_inputs.compile import compile_problem
    from vqe_inputs.problem import make_problem
    from paper_2211_07983_amd import Context, Plan, energy_grad_plans
    members = [i for i, (n, ne, D, s1, s2) in enumerate(configs.batched_instances())
               if n <= args.max_qubits and D <= args.max_d]
    ctx = Context(0)
    last = [time.perf_counter()]

    def progress(phase, done, total):
        now = time.perf_counter()
        if done == total or now - last[0] >= 15.0:
            log(f"  {phase} {done}/{total}")
            last[0] = now

    ctx.set_progress(progress)
    probs, plans, circuits = [], [], {}
    for i in members:
        n, ne, D, s1, s2 = configs.batched_instances()[i]
        p = make_problem(f"c4_{i}", n, ne, D, args.eps, s1, s2, 0.05)
        g = circuits.get((n, ne)) or compile_problem(p)
        circuits[(n, ne)] = g
        probs.append(p)
        plans.append(Plan(ctx, p.occ, g, p.n_qubits, p.ham_x, p.ham_z, p.ham_c, p.c0, p.bond_dim, p.eps,
                          ckpt_gates=args.ckpt_gates))
    classes = {}
    for k, p in enumerate(probs):
        classes.setdefault((p.n_qubits, p.bond_dim), []).append(k)
    log(f"{len(plans)} instances up to {args.max_qubits} q: classes "
        + ", ".join(f"{q}q D{d} x{len(v)}" for (q, d), v in sorted(classes.items())))
    t0 = time.perf_counter()
    e_m, g_m, st = energy_grad_plans(plans, [p.theta for p in probs])
    t_mixed = time.perf_counter() - t0
    log(f"one call: {len(plans)} instances in {t_mixed:.2f}s, max bond {st['max_bond']}")
    seq_est, worst, per_class = 0.0, 0.0, {}
    for (q, d), ks in sorted(classes.items()):
        k = ks[0]
        t0 = time.perf_counter()
        e1, g1, _ = plans[k].energy_grad(probs[k].theta)
        dt = time.perf_counter() - t0
        worst = max(worst, abs(e1 - e_m[k]) / abs(e1), float(np.abs(g1 - g_m[k]).max() / np.abs(g1).max()))
        per_class[f"{q}q_D{d}"] = {"count": len(ks), "instance": members[k], "single_s": dt}
        seq_est += dt * len(ks)
        log(f"  {q} q, D={d}: instance {members[k]} alone {dt:.2f}s (x{len(ks)})")
    line = {
        "metric": "instance energy+grad evals/s, batched-instance set across size classes in shared launches",
        "value": len(plans) / t_mixed, "unit": "instance-evals/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * t_mixed, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded per-instance integrals and theta)",
        "config": {"workload": f"batched-instance set, the {len(plans)} instances with at most {args.max_qubits} "
                               f"qubits and D <= {args.max_d} ({len(classes)} (qubits, D) classes), eps={args.eps:g}",
                   "instances": members, "classes": per_class,
                   "sequential_estimate_s": seq_est,
                   "sequential_note": "one instance per class timed alone, times the class count",
                   "speedup_vs_sequential_estimate": seq_est / t_mixed,
                   "max_rel_diff_vs_single": worst, "max_bond": st["max_bond"]},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def alg1_accuracy_phase(args):
    """Gradient accuracy under truncation on the GPU path (Sec. 4's comparison
    of the local gradient with Algorithm 1): the 8-qubit problem at
    D = 2, 4, 8 against its untruncated gradient (D = 16 holds every Schmidt
    value of 8 qubits), for the back-propagated fixed-rank gradient g_D, the
    parameter-shift gradient of the truncated circuit, and Algorithm 1 with
    four strings per group.  R = |g - g_exact| / |g_exact|."""
    import numpy as np
    from vqe_inputs import configs
    from paper_2211_07983_amd import Context, Plan
    prob, gates = configs.load("c1")
    ctx = Context(0)

    def plan_at(D):
        return Plan(ctx, prob.occ, gates, prob.n_qubits, prob.ham_x, prob.ham_z, prob.ham_c, prob.c0, D, 1e-12)

    exact_plan = plan_at(16)
    e_ex, g_ex, st = exact_plan.energy_grad(prob.theta)
    exact_plan.free()
    if st["gates_truncated"] != 0:
        raise SystemExit("D = 16 truncated the 8-qubit circuit")
    nrm = float(np.linalg.norm(g_ex))
    rows = []
    for D in (2, 4, 8):
        pl = plan_at(D)
        t0 = time.perf_counter()
        e_d, g_d, sd = pl.energy_grad(prob.theta)
        _, g_ps, _, _ = pl.energy_grad_psr(prob.theta)
        row = {"D": D, "E_error": e_d - e_ex, "discarded": sd["discarded_weight_sum"],
               "R_local": float(np.linalg.norm(g_d - g_ex)) / nrm, "R_psr": float(np.linalg.norm(g_ps - g_ex)) / nrm}
        for spg in (4,):   # the paper's optimiser runs use four strings per group
            if spg * D > 128:
                continue
            t1 = time.perf_counter()
            _, g_a, _, _ = pl.energy_grad_alg1(prob.theta, strings_per_group=spg)
            row[f"R_alg1_{spg}"] = float(np.linalg.norm(g_a - g_ex)) / nrm
            row[f"t_alg1_{spg}_s"] = time.perf_counter() - t1
        row["t_s"] = time.perf_counter() - t0
        log(f"D={D}: " + ", ".join(f"{k} {v:.3g}" for k, v in row.items() if k != "D"))
        rows.append(row)
        pl.free()
    line = {
        "metric": "relative gradient error R under truncation (GPU path): local g_D, parameter shift, Algorithm 1",
        "value": rows[0]["R_alg1_4"] if "R_alg1_4" in rows[0] else None, "unit": "R at D=2, Algorithm 1 (4/group)",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": None, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS["c1"] + f", eps=1e-12, {gates.n_gates} NN gates, {prob.n_terms} strings",
                   "exact": "the same circuit at D = 16 (no truncation)", "E_exact": e_ex, "rows": rows},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def alg1_phase(args):
    """Algorithm 1 (one Pauli string per group, 2 N_h reverse walks) against
    back-propagation on the same plan: 6 qubits (3 orbitals, 2 electrons),
    D = 8, no truncation, where both give the exact gradient."""
    import numpy as np
    from vqe_inputs import configs
    from paper_2211_07983_amd import Context, Plan
    prob, gates = configs.small(6, 2, 8, seed=1)
    ctx = Context(0)
    plan = Plan(ctx, prob.occ, gates, prob.n_qubits, prob.ham_x, prob.ham_z, prob.ham_c, prob.c0,
                prob.bond_dim, prob.eps)
    plan.energy_grad(prob.theta)                       # warm-up
    t0 = time.perf_counter()
    e_bp, g_bp, _ = plan.energy_grad(prob.theta)
    t_bp = time.perf_counter() - t0
    t0 = time.perf_counter()
    e_a1, g_a1, _, _ = plan.energy_grad_alg1(prob.theta)
    t_a1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, g_a4, _, _ = plan.energy_grad_alg1(prob.theta, strings_per_group=4)
    t_a4 = time.perf_counter() - t0
    diff = float(np.abs(g_a1 - g_bp).max() / np.abs(g_bp).max())
    diff4 = float(np.abs(g_a4 - g_bp).max() / np.abs(g_bp).max())
    log(f"back-propagation {t_bp:.3f}s, Algorithm 1 {t_a1:.3f}s ({len(prob.ham_c)} strings, one per group), "
        f"{t_a4:.3f}s (4 per group); rel diff {diff:.1e}, {diff4:.1e}")
    line = {
        "metric": "gradient time, Algorithm 1 (one string per group) / back-propagation (same plan, one GPU)",
        "value": t_a1 / t_bp, "unit": "ratio", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * t_a1, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"UCCSD-MPS 6 qubits (3 orbitals, 2 electrons), D=8, eps={prob.eps:g}, "
                               f"{gates.n_gates} NN gates, {len(prob.ham_c)} Pauli strings, n_theta={prob.n_theta}",
                   "t_backprop_s": t_bp, "t_alg1_s": t_a1, "max_rel_grad_diff": diff, "E": e_bp,
                   "t_alg1_4_per_group_s": t_a4, "max_rel_grad_diff_4_per_group": diff4},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c2")
    ap.add_argument("--batch", type=int, default=0,
                    help="parameter vectors per step (0: as many as one launch holds)")
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--ckpt-gates", type=int, default=512)
    ap.add_argument("--tape-budget-mib", type=int, default=-1,
                    help="device memory for gate tapes the batched forward pass keeps (-1: what is free after a "
                         "16 GiB reserve; 0: the last segment only)")
    ap.add_argument("--profile-every", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="wall-time budget of the whole run from process start (steps that would not fit are "
                         "not started; the line reports the steps that ran)")
    ap.add_argument("--cpu-reserve-s", type=float, default=90.0,
                    help="share of --budget-s held back for the CPU baseline")
    ap.add_argument("--phase", choices=["evalgrad", "sweep", "psr", "vqe", "instances", "mixed", "alg1",
                                        "alg1_accuracy"],
                    default="evalgrad")
    ap.add_argument("--max-qubits", type=int, default=16, help="--phase mixed: largest instance size taken")
    ap.add_argument("--max-d", type=int, default=128, help="--phase mixed: largest bond dimension taken")
    ap.add_argument("--class-qubits", type=int, default=12, help="--phase instances: qubit count of the class")
    ap.add_argument("--class-d", type=int, default=64, help="--phase instances: bond dimension of the class")
    ap.add_argument("--vqe-iters", type=int, default=100, help="--phase vqe: iteration limit")
    ap.add_argument("--precision", type=int, choices=[0, 1], default=0,
                    help="evalgrad phase: 0 plain FP64, 1 Pauli sweeps and sweep adjoint on FP32 matrix cores")
    ap.add_argument("--prefix-gates", type=int, default=3000,
                    help="--phase sweep: gates applied before the sweeps are timed")
    ap.add_argument("--cpu-child", choices=["full", "sample"], default=None, help=argparse.SUPPRESS)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (a reference "
                         "dispatch of known traffic for hardware byte counters)")
    args = ap.parse_args()
    if args.cpu_child:
        cpu_child(args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one MI355X: the hot path runs on a single GPU "
              "(the multi-GPU split is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy_mib > 0:
        calibration_copy(args.calibrate_copy_mib)
    if args.phase == "sweep":
        sweep_phase(args)
        return
    if args.phase == "psr":
        psr_phase(args)
        return
    if args.phase == "vqe":
        vqe_phase(args)
        return
    if args.phase == "instances":
        instances_phase(args)
        return
    if args.phase == "mixed":
        mixed_phase(args)
        return
    if args.phase == "alg1":
        alg1_phase(args)
        return
    if args.phase == "alg1_accuracy":
        alg1_accuracy_phase(args)
        return
    import numpy as np
    from vqe_inputs import configs
    from paper_2211_07983_amd import Context, Plan
    t = time.time()
    prob, gates = configs.load(args.workload, eps=args.eps)
    log(f"workload {args.workload} built in {time.time() - t:.1f}s: N={prob.n_qubits} K={prob.n_terms} "
        f"n_theta={prob.n_theta} gates={gates.n_gates} D={prob.bond_dim} eps={prob.eps:g}")
    ctx = Context(0)
    ctx.set_profiling(args.profile_every)
    last = [time.perf_counter(), None]

    def progress(phase, done, total):
        now = time.perf_counter()
        if done == total or now - last[0] >= 15.0:
            log(f"  {phase} segment {done}/{total} ({now - last[1]:.0f}s into the step)")
            last[0] = now

    ctx.set_progress(progress)
    plan = Plan(ctx, prob.occ, gates, prob.n_qubits, prob.ham_x, prob.ham_z, prob.ham_c, prob.c0,
                prob.bond_dim, prob.eps, precision=args.precision, ckpt_gates=args.ckpt_gates,
                tape_budget_mib=args.tape_budget_mib)
    nb = args.batch if args.batch > 0 else plan.lanes_per_launch()
    rng = np.random.default_rng(2024)
    thetas = np.stack([prob.theta] + [prob.theta + 0.05 * rng.normal(size=prob.theta.shape) for _ in range(nb - 1)])
    # The whole run keeps to --budget-s of wall time from process start: the
    # CPU baseline's share is held back, and a warm-up or timed step only
    # starts when the slowest step so far still fits.  steps/warmup in the line
    # are the ones that ran.
    cpu_reserve = 0.0 if args.no_cpu_baseline else args.cpu_reserve_s
    gpu_deadline = args.budget_s - cpu_reserve

    def fits(step_s):
        return time.monotonic() - T_START + step_s <= gpu_deadline

    # single-vector path: the plain FP64 evaluation of one vector (the metric's
    # denominator), also the first warm-up of the plan's buffers
    last[1] = time.perf_counter()
    t0 = time.perf_counter()
    e, g, st = plan.energy_grad(prob.theta)
    t_single = time.perf_counter() - t0
    log(f"single: {t_single:.1f}s E={e:.12f} |g|={float((g ** 2).sum()) ** 0.5:.6e} "
        f"gates={st['t_gates_ms']/1e3:.1f}s sweep={st['t_sweep_ms']/1e3:.1f}s backward={st['t_backward_ms']/1e3:.1f}s")
    step_est = t_single * max(1.0, nb / 8.0)    # a first guess until a batched step has run
    warm_done = 0
    for w in range(args.warmup):
        # warm-ups after the first only when every requested timed step still
        # fits behind the remaining ones: timed steps come first
        if w > 0 and not fits((args.warmup - w + args.steps) * step_est):
            break
        if not fits(step_est):
            break
        last[1] = time.perf_counter()
        plan.energy_grad_batched(thetas)
        dt = time.perf_counter() - last[1]
        step_est = dt if w == 0 else max(step_est, dt)
        warm_done += 1
        log(f"warmup {w}: {dt:.1f}s")
    done = 0
    T = 0.0
    eb = gb = sb = None
    while done < args.steps and (done == 0 or fits(step_est)):
        last[1] = time.perf_counter()
        eb, gb, sb = plan.energy_grad_batched(thetas)
        dt = time.perf_counter() - last[1]
        T += dt
        step_est = max(step_est, dt) if done or warm_done else dt
        done += 1
        log(f"step {done - 1}: {dt:.1f}s for {nb} evaluations, E[0]={eb[0]:.12f}")
    ctx.set_progress(None)
    if done < args.steps:
        log(f"wall budget of {args.budget_s:.0f}s: {done} of {args.steps} timed steps and {warm_done} of "
            f"{args.warmup} warm-ups ran")
    if abs(eb[0] - e) > 1e-12 * abs(e) or np.abs(gb[0] - g).max() > 1e-10 * np.abs(g).max():
        raise SystemExit("batched and single evaluation of the same vector disagree")
    value = done * nb / T
    # dominant kernel of the step: the batched gate chain (one cooperative launch
    # per checkpoint segment: contraction, Jacobi SVD and site update of every
    # gate of every vector), each forward launch timed with HIP events on the
    # context stream; work counted = the SVDs' 84 p^3 plus the gate GEMMs the
    # same launches run (contraction, gate matrix, left update; 8 flops per
    # complex multiply-add), both reported
    dcap = max(2, ((prob.bond_dim + 1) // 2) * 2)
    W = 32 if dcap <= 32 else 16 if dcap <= 64 else 8 if dcap <= 128 else 4
    src = sb if nb > 1 else st
    n_svd = src["prof_svd_launches"]
    avg_ms = src["prof_svd_ms"] / max(1, n_svd)
    svd_flop = src["prof_svd_flop"] / max(1, n_svd)
    gemm_flop = src.get("prof_gemm_flop", 0.0) / max(1, n_svd)
    flop_per_launch = svd_flop + gemm_flop
    achieved = flop_per_launch / (avg_ms * 1e-3) / 1e12 if n_svd else None
    roofline = {"kernel": f"k_chain_lanes<{W}>" if nb > 1 else f"k_svd_jacobi<{W}, true>", "bound": "alu",
                "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": (achieved / PEAK_FP64_TFLOPS) if achieved else None,
                "traffic": traffic_for("evalgrad", args.workload)[0] if nb == 64 and args.precision == 0 else None,
                "avg_launch_ms": avg_ms, "flop_per_launch": flop_per_launch, "svd_flop_per_launch": svd_flop,
                "gemm_flop_per_launch": gemm_flop, "timed_launches": n_svd}
    stats_single = dict(st)
    plan.free()
    ctx.close()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_settings(args.workload, prob.eps, T_START + args.budget_s)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": done,
        "warmup": warm_done,
        "ms_per_step": 1e3 * T / done,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f64 gates, f32-mfma sweeps",
        "data": "synthetic (seeded random integrals, JW Hamiltonian, spin-orbital UCCSD, theta~N(0,0.05); "
                "batch: that theta and seeded perturbations of 0.05 N(0,1))",
        "config": {"workload": WORKLOADS[args.workload] + f", eps={prob.eps:g}, K={prob.n_terms} Pauli terms, "
                               f"{gates.n_gates} NN gates, n_theta={prob.n_theta}, "
                               + ("plain FP64" if args.precision == 0 else "precision 1 (FP32-MFMA sweeps)"),
                   "headline_note": WORKLOAD_NOTE.get(args.workload, ""),
                   "global_batch": nb,
                   "requested_steps": args.steps, "requested_warmup": args.warmup,
                   "budget_s": args.budget_s, "wall_s": time.monotonic() - T_START,
                   "single": {"evals_per_s": 1.0 / t_single, "seconds": t_single},
                   "speedup_vs_single_fp64": value * t_single,
                   "energy": e, "grad_norm": float((g ** 2).sum()) ** 0.5,
                   "t_gates_s": stats_single["t_gates_ms"] / 1e3, "t_sweep_s": stats_single["t_sweep_ms"] / 1e3,
                   "t_backward_s": stats_single["t_backward_ms"] / 1e3, "max_bond": stats_single["max_bond"],
                   "discarded_weight_sum": stats_single["discarded_weight_sum"],
                   "max_jacobi_sweeps": stats_single["max_sweeps_used"], "ckpt_gates": args.ckpt_gates,
                   "tape_budget_mib": args.tape_budget_mib},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
