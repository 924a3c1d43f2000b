"""bench.py contract checks that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "single GPU" in r.stderr and r.stdout == ""


def test_every_phase_is_offered():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0
    for phase in ("evalgrad", "sweep", "psr", "vqe", "instances", "mixed", "alg1"):
        assert phase in r.stdout


def test_instance_classes_share_their_circuit():
    """The batched-instance phase and mps_energy_grad_multi rely on every
    instance of one qubit count compiling to the same gate list."""
    import numpy as np
    from vqe_inputs import configs
    from vqe_inputs.compile import compile_problem
    from vqe_inputs.problem import make_problem
    members = [i for i, (n, ne, D, s1, s2) in enumerate(configs.batched_instances()) if n == 12][:3]
    lists = []
    for i in members:
        n, ne, D, s1, s2 = configs.batched_instances()[i]
        lists.append(compile_problem(make_problem(f"c4_{i}", n, ne, D, 1e-6, s1, s2, 0.05)))
    for g in lists[1:]:
        for k in ("bond", "kind", "pre", "post", "param", "coeff"):
            assert np.array_equal(np.asarray(getattr(g, k)), np.asarray(getattr(lists[0], k)))


def test_cpu_baseline_reports_both_thread_settings_and_the_host():
    """The CPU baseline times the oracle with BLAS on one thread and on the
    nproc setting, each in a child process whose BLAS pool the environment
    fixes, and records the host's core counts and CPU model."""
    sys.path.insert(0, ROOT)
    import bench
    import time
    r = bench.cpu_baseline_settings("c1", 1e-12, time.monotonic() + 300.0)
    assert r["kind"] == "oracle" and r["unit"] == "evals/s" and r["value"] > 0
    assert all("error" not in s for s in r["settings"])
    assert r["settings"][0]["requested_threads"] == 1 and r["settings"][0]["cores"] == 1
    assert all(s["mode"] == "full" for s in r["settings"])
    assert r["cores"] in [s["cores"] for s in r["settings"]]
    assert r["value"] == max(s["value"] for s in r["settings"])
    host = r["host"]
    assert host["nproc"] >= 1 and host["usable_cpus"] >= 1 and "cpu_model" in host
