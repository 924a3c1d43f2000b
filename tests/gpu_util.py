"""Shared helpers of the GPU tests (the HIP path through the C ABI)."""
import json
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_values.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


class Prefix:
    """The first `count` gates of a gate list (same arrays, sliced)."""

    def __init__(self, gl, count):
        self.n_qubits = gl.n_qubits
        self.bond = gl.bond[:count]
        self.kind = gl.kind[:count]
        self.pre = gl.pre[:count]
        self.post = gl.post[:count]
        self.param = gl.param[:count]
        self.coeff = gl.coeff[:count]


def gpu_energy(ctx, prob, gates, theta, d_max=None, eps=None, terms=False):
    from paper_2211_07983_amd import State
    st = State.product(ctx, prob.occ, prob.bond_dim if d_max is None else d_max,
                       prob.eps if eps is None else eps)
    s1 = st.apply_circuit(gates, theta)
    e, tv, s2 = st.expect(prob.n_qubits, prob.ham_x, prob.ham_z, prob.ham_c, prob.c0, terms=terms)
    return e, tv, s1, s2, st


def rel(a, b):
    return abs(a - b) / max(1e-300, abs(b))
