"""mps_apply_circuit_noalloc (the entry point for callers that cannot
allocate device memory) against mps_apply_circuit through the C ABI: the same
kernels on the same inputs, so the states must agree bit for bit.  Two calls
in a row share the per-device workspace: the 8-qubit workload (1415 gates, two
circuit chunks) and then a smaller input (its first 300 gates at D = 8), each
against the allocating entry point; then the size limit."""
import numpy as np
import pytest

from vqe_inputs import configs
from gpu_util import Prefix

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2211_07983_amd import Context
    c = Context(0)
    yield c
    c.close()


def _pair(ctx, p, gates, theta, d_max, eps):
    from paper_2211_07983_amd import State
    a = State.product(ctx, p.occ, d_max, eps)
    b = State.product(ctx, p.occ, d_max, eps)
    sa = a.apply_circuit(gates, theta)
    sb = b.apply_circuit_noalloc(gates, theta)
    ea, eb = a.export(), b.export()
    a.free()
    b.free()
    return sa, sb, ea, eb


def _same(ea, eb):
    assert np.array_equal(ea[0], eb[0])
    for x, y in zip(ea[1], eb[1]):
        assert np.array_equal(x, y)
    for x, y in zip(ea[2], eb[2]):
        assert np.array_equal(x, y)


def test_noalloc_equals_allocating_entry_point_twice(ctx):
    p, g = configs.load("c1")
    for gates, d_max, eps in ((g, p.bond_dim, p.eps), (Prefix(g, 300), 8, 1e-6)):
        sa, sb, ea, eb = _pair(ctx, p, gates, p.theta, d_max, eps)
        _same(ea, eb)
        for k in ("discarded_weight_sum", "max_bond", "gates_truncated", "degenerate_cuts", "n_gates_applied"):
            assert sa[k] == sb[k], k
    # the smaller second input really truncated (D = 8 < 16)
    assert sb["gates_truncated"] > 0 and sb["max_bond"] == 8


def test_noalloc_refuses_sizes_beyond_its_workspace(ctx):
    from paper_2211_07983_amd import MPSError, State
    p, g = configs.load("c1")
    st = State.product(ctx, p.occ, 256, p.eps)
    with pytest.raises(MPSError, match="MPS_EINVAL"):
        st.apply_circuit_noalloc(Prefix(g, 10), p.theta)
    st.free()
