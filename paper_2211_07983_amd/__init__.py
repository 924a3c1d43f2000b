"""MI355X-native differentiable-MPS VQE engine (arXiv:2211.07983 hot path).

Thin Python binding over libmpsvqe.so (include/mpsvqe.h): argument marshalling
only.  Every step of the path -- product state, gate contractions, Jacobi
SVDs, Pauli sweeps and the reverse pass -- runs in the HIP kernels of the
library.  There is no CPU fallback: if the library is missing, loading fails.
"""
from __future__ import annotations

import atexit
import ctypes as C
import sys
import weakref

import numpy as np

from . import _abi
from ._abi import GradOpts, PauliSum, Stats, Trunc

__all__ = ["MPSError", "Context", "State", "Plan", "EnergyGrad", "energy_grad_multi", "energy_grad_plans", "lib"]


def lib():
    return _abi.load()


class MPSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_abi.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_live_children = weakref.WeakSet()    # states and plans
_live_contexts = weakref.WeakSet()


@atexit.register
def _release_all():
    """Free every live handle before the interpreter (and the HIP runtime) shuts
    down: states and plans first, then their contexts."""
    for obj in list(_live_children):
        try:
            obj.free()
        except Exception:
            pass
    for obj in list(_live_contexts):
        try:
            obj.close()
        except Exception:
            pass


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class _CircuitArgs:
    """Keeps the numpy buffers of an mps_circuit alive for the duration of a call."""

    def __init__(self, gates):
        G = int(len(gates.bond))
        self.bond = np.ascontiguousarray(gates.bond, dtype=np.int32)
        self.kind = np.ascontiguousarray(gates.kind, dtype=np.int32)
        self.pre = np.ascontiguousarray(np.asarray(gates.pre, dtype=np.complex128).reshape(G, 4, 4)).view(np.float64)
        self.post = np.ascontiguousarray(np.asarray(gates.post, dtype=np.complex128).reshape(G, 4, 4)).view(np.float64)
        self.param = np.ascontiguousarray(gates.param, dtype=np.int32)
        self.coeff = np.ascontiguousarray(gates.coeff, dtype=np.float64)
        self.c = _abi.Circuit(int(gates.n_qubits), G, _ptr(self.bond, C.c_int32), _ptr(self.kind, C.c_int32),
                              _ptr(self.pre, C.c_double), _ptr(self.post, C.c_double),
                              _ptr(self.param, C.c_int32), _ptr(self.coeff, C.c_double))


class _PauliArgs:
    def __init__(self, n_qubits, x, z, coeff, c0):
        self.x = np.ascontiguousarray(x, dtype=np.uint64)
        self.z = np.ascontiguousarray(z, dtype=np.uint64)
        self.coeff = np.ascontiguousarray(coeff, dtype=np.float64)
        words = (int(n_qubits) + 63) // 64
        self.p = PauliSum(int(n_qubits), len(self.coeff), words, _ptr(self.x, C.c_uint64),
                          _ptr(self.z, C.c_uint64), _ptr(self.coeff, C.c_double), float(c0))


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)   # torch.cuda.Stream


class Context:
    """One device and one HIP stream (torch's current stream if stream == 'torch')."""

    def __init__(self, device=0, stream=None):
        self._lib = lib()
        if stream == "torch":
            import torch
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        st = self._lib.mps_ctx_create(int(device), _stream_handle(stream), C.byref(h))
        if st != 0:
            raise MPSError(st, "mps_ctx_create failed (no usable HIP device with cooperative launch)")
        self.h = h
        self.device = device
        _live_contexts.add(self)

    def set_profiling(self, every):
        self.check(self._lib.mps_ctx_set_profiling(self.h, int(every)))

    def set_progress(self, fn):
        """fn(phase: str, done: int, total: int) after each checkpoint segment of a
        plan's forward and reverse passes (None = off)."""
        if fn is None:
            self._progress = None
            self.check(self._lib.mps_ctx_set_progress(self.h, _abi.ProgressFn(), None))
            return
        self._progress = _abi.ProgressFn(lambda user, phase, done, total: fn(phase.decode(), done, total))
        self.check(self._lib.mps_ctx_set_progress(self.h, self._progress, None))

    def check(self, status):
        if status != 0:
            raise MPSError(status, self._lib.mps_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            for obj in list(_live_children):
                if getattr(obj, "ctx", None) is self:
                    obj.free()
            self._lib.mps_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class State:
    """An MPS on the device (mps_state)."""

    def __init__(self, ctx, handle, n_qubits, d_max):
        self.ctx, self.h, self.n, self.d_max = ctx, handle, n_qubits, d_max
        _live_children.add(self)

    @classmethod
    def product(cls, ctx, occ, d_max, eps, precision=0):
        occ = np.ascontiguousarray(occ, dtype=np.uint8)
        tr = Trunc(int(d_max), float(eps), int(precision))
        h = C.c_void_p()
        ctx.check(ctx._lib.mps_init_product(ctx.h, len(occ), _ptr(occ, C.c_uint8), C.byref(tr), C.byref(h)))
        return cls(ctx, h, len(occ), d_max)

    @classmethod
    def from_tensors(cls, ctx, tensors, lams, d_max, eps, precision=0):
        """mps_state_import: tensors[n] complex [dl, 2, dr], lams[k] the Schmidt
        vector left of site k (k = 0..n)."""
        n = len(tensors)
        dims = np.array([1] + [int(t.shape[2]) for t in tensors], dtype=np.int32)
        B = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.complex128).ravel() for t in tensors]))
        lam = np.ascontiguousarray(np.concatenate([np.asarray(l, dtype=np.float64).ravel() for l in lams]))
        tr = Trunc(int(d_max), float(eps), int(precision))
        h = C.c_void_p()
        ctx.check(ctx._lib.mps_state_import(ctx.h, n, C.byref(tr), _ptr(dims, C.c_int32),
                                            _ptr(B.view(np.float64), C.c_double), _ptr(lam, C.c_double),
                                            C.byref(h)))
        return cls(ctx, h, n, d_max)

    def apply_circuit(self, gates, theta):
        args = _CircuitArgs(gates)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        s = Stats()
        self.ctx.check(self.ctx._lib.mps_apply_circuit(self.h, C.byref(args.c), _ptr(th, C.c_double),
                                                       len(th), C.byref(s)))
        return s.as_dict()

    def apply_circuit_noalloc(self, gates, theta):
        """mps_apply_circuit_noalloc: the same update with the library's fixed
        per-device workspace instead of device allocations."""
        args = _CircuitArgs(gates)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        s = Stats()
        self.ctx.check(self.ctx._lib.mps_apply_circuit_noalloc(self.h, C.byref(args.c), _ptr(th, C.c_double),
                                                               len(th), C.byref(s)))
        return s.as_dict()

    def expect(self, n_qubits, x, z, coeff, c0, terms=False):
        args = _PauliArgs(n_qubits, x, z, coeff, c0)
        e = C.c_double()
        s = Stats()
        tv = np.zeros(len(args.coeff)) if terms else None
        self.ctx.check(self.ctx._lib.mps_expect_paulisum(
            self.h, C.byref(args.p), C.byref(e), _ptr(tv, C.c_double) if terms else None, C.byref(s)))
        return e.value, tv, s.as_dict()

    def export(self):
        lib = self.ctx._lib
        dims = np.zeros(self.n + 1, dtype=np.int32)
        size = lib.mps_state_size(self.h)
        B = np.zeros(max(size, 2))
        dcap = max(2, ((self.d_max + 1) // 2) * 2)
        lam = np.zeros((self.n + 1) * dcap)
        self.ctx.check(lib.mps_state_export(self.h, _ptr(dims, C.c_int32), _ptr(B, C.c_double),
                                            _ptr(lam, C.c_double)))
        tensors, o = [], 0
        Bc = B[: 2 * (size // 2)].view(np.complex128)
        for n in range(self.n):
            k = dims[n] * 2 * dims[n + 1]
            tensors.append(Bc[o:o + k].reshape(dims[n], 2, dims[n + 1]).copy())
            o += k
        lam = lam.reshape(self.n + 1, dcap)
        lams = [lam[n, : dims[n]].copy() for n in range(self.n + 1)]
        return dims, tensors, lams

    def free(self):
        if self.h and getattr(self.ctx, "h", None):
            self.ctx._lib.mps_state_free(self.h)
        self.h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


class Plan:
    """Device copy of (initial state, circuit, Hamiltonian, options): mps_plan."""

    def __init__(self, ctx, occ, gates, n_qubits, x, z, coeff, c0, d_max, eps, precision=0,
                 ckpt_gates=256, broaden=0.0, max_sweeps=64, strict_degenerate=0, tape_budget_mib=0):
        self.ctx = ctx
        occ = np.ascontiguousarray(occ, dtype=np.uint8)
        ca = _CircuitArgs(gates)
        pa = _PauliArgs(n_qubits, x, z, coeff, c0)
        tr = Trunc(int(d_max), float(eps), int(precision))
        go = GradOpts(int(ckpt_gates), float(broaden), int(max_sweeps), int(strict_degenerate), int(tape_budget_mib))
        h = C.c_void_p()
        ctx.check(ctx._lib.mps_plan_create(ctx.h, _ptr(occ, C.c_uint8), C.byref(ca.c), C.byref(pa.p),
                                           C.byref(tr), C.byref(go), C.byref(h)))
        self.h = h
        self.n_theta = int(np.max(gates.param)) + 1 if np.any(np.asarray(gates.kind) == 1) else 0
        self.n_gates = len(gates.bond)
        _live_children.add(self)

    def energy(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        e = C.c_double()
        s = Stats()
        self.ctx.check(self.ctx._lib.mps_plan_energy(self.h, _ptr(th, C.c_double), len(th), C.byref(e),
                                                     C.byref(s)))
        return e.value, s.as_dict()

    def energy_grad(self, theta):
        """theta: numpy array (host) or a device torch tensor; returns (E, grad, stats)."""
        s = Stats()
        e = C.c_double()
        if hasattr(theta, "is_cuda") and theta.is_cuda:
            import torch
            th = theta.detach().to(torch.float64).contiguous()
            g = torch.empty_like(th)
            self.ctx.check(self.ctx._lib.mps_energy_grad(self.h, C.c_void_p(th.data_ptr()), th.numel(), 1,
                                                         C.byref(e), C.c_void_p(g.data_ptr()), C.byref(s)))
            return e.value, g, s.as_dict()
        th = np.ascontiguousarray(theta, dtype=np.float64)
        g = np.zeros_like(th)
        self.ctx.check(self.ctx._lib.mps_energy_grad(self.h, th.ctypes.data_as(C.c_void_p), len(th), 0,
                                                     C.byref(e), g.ctypes.data_as(C.c_void_p), C.byref(s)))
        return e.value, g, s.as_dict()

    def lanes_per_launch(self):
        """Parameter vectors one batched launch holds (mps_plan_batch_width)."""
        w = self.ctx._lib.mps_plan_batch_width(self.h)
        if w <= 0:
            self.ctx.check(w)
        return w

    def energy_grad_batched(self, thetas):
        """thetas: [n_batch, n_theta] numpy array or device torch tensor; returns
        (energies [n_batch], grads [n_batch, n_theta], stats)."""
        s = Stats()
        if hasattr(thetas, "is_cuda") and thetas.is_cuda:
            import torch
            th = thetas.detach().to(torch.float64).contiguous()
            nb = th.shape[0]
            e = np.zeros(nb)
            g = torch.empty_like(th)
            self.ctx.check(self.ctx._lib.mps_energy_grad_batched(
                self.h, nb, C.c_void_p(th.data_ptr()), th.shape[1], 1, _ptr(e, C.c_double), C.c_void_p(g.data_ptr()),
                C.byref(s)))
            return e, g, s.as_dict()
        th = np.ascontiguousarray(thetas, dtype=np.float64)
        if th.ndim != 2:
            raise ValueError("thetas must be [n_batch, n_theta]")
        nb = th.shape[0]
        e = np.zeros(nb)
        g = np.zeros_like(th)
        self.ctx.check(self.ctx._lib.mps_energy_grad_batched(
            self.h, nb, th.ctypes.data_as(C.c_void_p), th.shape[1], 0, _ptr(e, C.c_double),
            g.ctypes.data_as(C.c_void_p), C.byref(s)))
        return e, g, s.as_dict()

    def energy_grad_psr(self, theta):
        """Parameter-shift gradient: (E, grad [n_theta], dE/dphi per gate [n_gates], stats)."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        e = C.c_double()
        g = np.zeros(max(1, len(th)))
        gg = np.zeros(max(1, self.n_gates))
        s = Stats()
        self.ctx.check(self.ctx._lib.mps_energy_grad_psr(self.h, _ptr(th, C.c_double) if len(th) else None, len(th),
                                                         C.byref(e), _ptr(g, C.c_double), _ptr(gg, C.c_double),
                                                         C.byref(s)))
        return e.value, g[:len(th)], gg[:self.n_gates], s.as_dict()

    def energy_grad_alg1(self, theta, strings_per_group=1):
        """Gradient by the paper's Algorithm 1 with the Hamiltonian split into
        groups of strings_per_group strings (mps_energy_grad_alg1):
        (E, grad [n_theta], dE/dphi per gate [n_gates], stats)."""
        th = np.ascontiguousarray(theta, dtype=np.float64)
        e = C.c_double()
        g = np.zeros(max(1, len(th)))
        gg = np.zeros(max(1, self.n_gates))
        s = Stats()
        self.ctx.check(self.ctx._lib.mps_energy_grad_alg1(self.h, _ptr(th, C.c_double) if len(th) else None,
                                                          len(th), strings_per_group, C.byref(e),
                                                          _ptr(g, C.c_double), _ptr(gg, C.c_double), C.byref(s)))
        return e.value, g[:len(th)], gg[:self.n_gates], s.as_dict()

    def free(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            self.ctx._lib.mps_plan_free(self.h)
        self.h = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


def energy_grad_multi(plans, thetas):
    """Energies and gradients of several instances that share one circuit, each
    plan with its own Hamiltonian, as lanes of the same gate-chain launches
    (mps_energy_grad_multi).  plans: Plans of one context built from the same
    circuit, truncation and options; thetas: [n_plans, n_theta].  Returns
    (energies [n_plans], grads [n_plans, n_theta], stats)."""
    plans = list(plans)
    if not plans:
        raise ValueError("no plans")
    ctx = plans[0].ctx
    th = np.ascontiguousarray(thetas, dtype=np.float64)
    if th.ndim != 2 or th.shape[0] != len(plans):
        raise ValueError("thetas must be [n_plans, n_theta]")
    hs = (C.c_void_p * len(plans))(*[p.h for p in plans])
    e = np.zeros(len(plans))
    g = np.zeros_like(th)
    s = Stats()
    ctx.check(ctx._lib.mps_energy_grad_multi(hs, len(plans), th.ctypes.data_as(C.c_void_p), th.shape[1],
                                             _ptr(e, C.c_double), g.ctypes.data_as(C.c_void_p), C.byref(s)))
    return e, g, s.as_dict()


def energy_grad_plans(plans, thetas):
    """Energies and gradients of independent instances of any size (each plan
    its own circuit, qubit count, d_max and Hamiltonian) as lanes of shared
    gate-chain launches (mps_energy_grad_plans).  plans: distinct Plans of one
    context; thetas: one parameter array per plan.  Returns (energies
    [n_plans], [grad per plan], stats)."""
    plans = list(plans)
    if not plans or len(thetas) != len(plans):
        raise ValueError("one theta array per plan")
    ctx = plans[0].ctx
    ths = [np.ascontiguousarray(t, dtype=np.float64) for t in thetas]
    gs = [np.zeros(max(1, len(t))) for t in ths]
    hs = (C.c_void_p * len(plans))(*[p.h for p in plans])
    tp = (C.c_void_p * len(plans))(*[t.ctypes.data if len(t) else None for t in ths])
    gp = (C.c_void_p * len(plans))(*[g.ctypes.data for g in gs])
    e = np.zeros(len(plans))
    s = Stats()
    ctx.check(ctx._lib.mps_energy_grad_plans(hs, len(plans), tp, _ptr(e, C.c_double), gp, C.byref(s)))
    return e, [g[:len(t)] for g, t in zip(gs, ths)], s.as_dict()


def _energy_grad_function():
    import torch

    class _EnergyGrad(torch.autograd.Function):
        """E(theta) with dE/dtheta from mps_energy_grad; backward returns E_bar * g
        (the outer-scalar rule of Sec. 4, Eq. expecgrad)."""

        @staticmethod
        def forward(ctx, theta, plan):
            e, g, _ = plan.energy_grad(theta)
            if not isinstance(g, torch.Tensor):
                g = torch.from_numpy(g)
            ctx.save_for_backward(g.to(theta.device))
            return torch.tensor(e, dtype=torch.float64, device=theta.device)

        @staticmethod
        def backward(ctx, ebar):
            (g,) = ctx.saved_tensors
            return ebar * g, None

    return _EnergyGrad


class _Lazy:
    _fn = None

    def apply(self, theta, plan):
        if _Lazy._fn is None:
            _Lazy._fn = _energy_grad_function()
        return _Lazy._fn.apply(theta, plan)


EnergyGrad = _Lazy()
