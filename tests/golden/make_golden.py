"""Writes oracle_values.json: expected values computed by the CPU oracle only.

Run from the repository root:
    python tests/golden/make_golden.py                 # every entry
    python tests/golden/make_golden.py c2_paper        # selected entries, merged
Every number here comes from oracle/ (T1 sector simulator, T3 FP64 MPS) on the
seeded synthetic problems of vqe_inputs; nothing is taken from the HIP path.
"""
import json
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from vqe_inputs import configs  # noqa: E402
from oracle import mps, sector  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")
C3_PREFIX = 3000
C3_GRAD_PREFIX = 2500


def exact_config(name):
    """C1/C2 at the parity threshold: T3 energy, gradient, bonds and Schmidt
    values, plus the exact T1 energy and gradient."""
    p, g = configs.load(name)
    E, grad, info = mps.energy_grad(p, g, p.theta)
    _, finfo = mps.energy(p, g, p.theta)
    u = sector.UCCSD(p)
    return dict(E=E, grad=grad.tolist(), bonds=finfo["bonds"],
                lam=[l.tolist() for l in finfo["mps"].lam],
                E_exact=u.energy(p.theta), grad_exact=u.gradient(p.theta).tolist(),
                n_gates=int(g.n_gates), n_terms=int(p.n_terms))


def c2_paper():
    """C2 at the paper's truncation threshold eps = 1e-6 (Sec. 5): T3 energy,
    gradient g_D and final bonds."""
    p, g = configs.load("c2", eps=configs.PAPER_EPS)
    E, grad, info = mps.energy_grad(p, g, p.theta)
    _, finfo = mps.energy(p, g, p.theta)
    return dict(eps=p.eps, E=E, grad=grad.tolist(), bonds=finfo["bonds"])


def c3_prefix_grad():
    """Energy and gradient of the first C3_GRAD_PREFIX gates of C3 at the parity
    threshold: every middle SVD is full size (256 x 256) and truncates to 128."""
    import dataclasses
    p, g = configs.load("c3")
    pre = dataclasses.replace(g, bond=g.bond[:C3_GRAD_PREFIX], kind=g.kind[:C3_GRAD_PREFIX],
                              pre=g.pre[:C3_GRAD_PREFIX], post=g.post[:C3_GRAD_PREFIX],
                              param=g.param[:C3_GRAD_PREFIX], coeff=g.coeff[:C3_GRAD_PREFIX])
    n_theta = int(pre.param.max()) + 1
    E, grad, info = mps.energy_grad(p, pre, p.theta, ckpt=256)
    return dict(gates=C3_GRAD_PREFIX, n_theta=n_theta, E=E, grad=grad[:n_theta].tolist(),
                degenerate_cuts=int(info.get("degenerate_cuts", 0)) if isinstance(info, dict) else 0)


def c3_prefix():
    """The first C3_PREFIX gates of C3 (the middle bonds reach D=128)."""
    p, g = configs.load("c3")
    m = mps.forward(p, g, p.theta, count=C3_PREFIX)
    e, eim, Z, _ = m.energy(p.ham_x, p.ham_z, p.ham_c, p.c0)
    return dict(gates=C3_PREFIX, E=e, Eim=eim, Z=Z.real, bonds=m.bond_dims(), lam_mid=m.lam[12].tolist())


C5_PREFIX = 3000


def c5_prefix():
    """The first C5_PREFIX gates of the 40-qubit, D=256 workload (233000 terms):
    energy and bonds at the parity threshold."""
    p, g = configs.load("c5")
    m = mps.forward(p, g, p.theta, count=C5_PREFIX)
    e, eim, Z, _ = m.energy(p.ham_x, p.ham_z, p.ham_c, p.c0)
    return dict(gates=C5_PREFIX, E=e, Eim=eim, Z=Z.real, bonds=m.bond_dims())


def batched_instance(i):
    """Instance i of the batched set (qubits and D drawn per instance): the
    energy, gradient and bonds at its own D and the parity threshold."""
    from vqe_inputs.compile import compile_problem
    from vqe_inputs.problem import make_problem
    n, ne, D, s1, s2 = configs.batched_instances()[i]
    p = make_problem(f"c4_{i}", n, ne, D, configs.PARITY_EPS, s1, s2, 0.05)
    g = compile_problem(p)
    E, grad, info = mps.energy_grad(p, g, p.theta)
    _, finfo = mps.energy(p, g, p.theta)
    return dict(n_qubits=n, D=D, E=E, grad=grad.tolist(), bonds=finfo["bonds"],
                discarded_sum=float(sum(finfo["discarded"])))


ENTRIES = {"c1": lambda: exact_config("c1"), "c2": lambda: exact_config("c2"), "c2_paper": c2_paper,
           "c3_prefix": c3_prefix, "c3_prefix_grad": c3_prefix_grad, "c5_prefix": c5_prefix,
           "c4_3": lambda: batched_instance(3), "c4_4": lambda: batched_instance(4)}


def main(names):
    res = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            res = json.load(f)
    res["source"] = "oracle/ (T1 sector simulator, T3 FP64 MPS); seeds as in vqe_inputs.configs"
    for name in names or list(ENTRIES):
        t = time.time()
        res[name] = ENTRIES[name]()
        print(name, "done", round(time.time() - t, 1), flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:])
