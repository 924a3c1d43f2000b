"""Writes oracle_values.json: expected values computed by the CPU oracle only.

Run from the repository root:  python tests/golden/make_golden.py
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

import numpy as np  # noqa: E402

from vqe_inputs import configs  # noqa: E402
from oracle import mps, sector  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")
C3_PREFIX = 3000


def main():
    res = {"source": "oracle/ (T1 sector simulator, T3 FP64 MPS); seeds as in vqe_inputs.configs"}
    for name in ("c1", "c2"):
        t = time.time()
        p, g = configs.load(name)
        E, grad, info = mps.energy_grad(p, g, p.theta)
        _, finfo = mps.energy(p, g, p.theta)
        u = sector.UCCSD(p)
        res[name] = dict(E=E, grad=grad.tolist(), bonds=finfo["bonds"],
                         lam=[l.tolist() for l in finfo["mps"].lam],
                         E_exact=u.energy(p.theta), grad_exact=u.gradient(p.theta).tolist(),
                         n_gates=int(g.n_gates), n_terms=int(p.n_terms))
        print(name, "done", time.time() - t, flush=True)
    t = time.time()
    p, g = configs.load("c3")
    E, info = mps.energy(p, g, p.theta, count=None) if False else (None, None)
    m = mps.forward(p, g, p.theta, count=C3_PREFIX)
    e, eim, Z, _ = m.energy(p.ham_x, p.ham_z, p.ham_c, p.c0)
    res["c3_prefix"] = dict(gates=C3_PREFIX, E=e, Eim=eim, Z=Z.real, bonds=m.bond_dims(),
                            lam_mid=m.lam[12].tolist())
    print("c3 prefix done", time.time() - t, flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
