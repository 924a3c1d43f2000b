"""ctypes mirror of include/mpsvqe.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpsvqe.so")

MPS_OK, MPS_EINVAL, MPS_ENOMEM, MPS_EDEVICE, MPS_ENOCONV, MPS_EDEGEN = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "MPS_OK", -1: "MPS_EINVAL", -2: "MPS_ENOMEM", -3: "MPS_EDEVICE",
                -4: "MPS_ENOCONV", -5: "MPS_EDEGEN"}

EXPORTS = [
    "mps_ctx_create", "mps_ctx_destroy", "mps_ctx_set_profiling", "mps_ctx_set_progress", "mps_last_error", "mps_init_product",
    "mps_apply_circuit", "mps_apply_circuit_noalloc", "mps_expect_paulisum", "mps_plan_create", "mps_energy_grad",
    "mps_energy_grad_batched", "mps_energy_grad_multi", "mps_energy_grad_plans", "mps_plan_batch_width", "mps_energy_grad_psr",
    "mps_energy_grad_alg1",
    "mps_plan_energy", "mps_state_export", "mps_state_import", "mps_state_size", "mps_state_qubits",
    "mps_state_free", "mps_plan_free",
]


# void (*)(void* user, const char* phase, int64_t done, int64_t total)
ProgressFn = C.CFUNCTYPE(None, C.c_void_p, C.c_char_p, C.c_int64, C.c_int64)


class Trunc(C.Structure):
    _fields_ = [("d_max", C.c_int32), ("eps", C.c_double), ("precision", C.c_int32)]


class Circuit(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_gates", C.c_int32),
                ("bond", C.POINTER(C.c_int32)), ("kind", C.POINTER(C.c_int32)),
                ("pre", C.POINTER(C.c_double)), ("post", C.POINTER(C.c_double)),
                ("param", C.POINTER(C.c_int32)), ("coeff", C.POINTER(C.c_double))]


class PauliSum(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_terms", C.c_int64), ("words", C.c_int32),
                ("x_mask", C.POINTER(C.c_uint64)), ("z_mask", C.POINTER(C.c_uint64)),
                ("coeff", C.POINTER(C.c_double)), ("c0", C.c_double)]


class GradOpts(C.Structure):
    _fields_ = [("ckpt_gates", C.c_int32), ("broaden", C.c_double),
                ("max_sweeps", C.c_int32), ("strict_degenerate", C.c_int32),
                ("tape_budget_mib", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("discarded_weight_sum", C.c_double), ("discarded_weight_max", C.c_double),
                ("norm", C.c_double), ("imag_E", C.c_double),
                ("max_bond", C.c_int32), ("gates_truncated", C.c_int32),
                ("max_sweeps_used", C.c_int32), ("degenerate_cuts", C.c_int32),
                ("t_gates_ms", C.c_double), ("t_sweep_ms", C.c_double),
                ("t_backward_ms", C.c_double), ("n_gates_applied", C.c_int64),
                ("prof_svd_ms", C.c_double), ("prof_svd_flop", C.c_double),
                ("prof_svd_launches", C.c_int32), ("prof_pad", C.c_int32),
                ("prof_gemm_flop", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path=LIB_PATH):
    """Loads the HIP library; raises if it is not built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2211_07983_amd.build.build()")
    # One HIP runtime per process: when PyTorch is installed its bundled
    # libamdhip64.so.7 is loaded first and the library binds to the same one, so
    # torch device pointers and streams are valid in both.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.mps_ctx_create.argtypes = [C.c_int32, vp, C.POINTER(vp)]
    lib.mps_ctx_create.restype = C.c_int32
    lib.mps_ctx_destroy.argtypes = [vp]
    lib.mps_ctx_destroy.restype = None
    lib.mps_ctx_set_profiling.argtypes = [vp, C.c_int32]
    lib.mps_ctx_set_profiling.restype = C.c_int32
    lib.mps_ctx_set_progress.argtypes = [vp, ProgressFn, vp]
    lib.mps_ctx_set_progress.restype = C.c_int32
    lib.mps_last_error.argtypes = [vp]
    lib.mps_last_error.restype = C.c_char_p
    lib.mps_init_product.argtypes = [vp, C.c_int32, C.POINTER(C.c_uint8), C.POINTER(Trunc), C.POINTER(vp)]
    lib.mps_init_product.restype = C.c_int32
    lib.mps_apply_circuit.argtypes = [vp, C.POINTER(Circuit), C.POINTER(C.c_double), C.c_int32, C.POINTER(Stats)]
    lib.mps_apply_circuit.restype = C.c_int32
    lib.mps_apply_circuit_noalloc.argtypes = [vp, C.POINTER(Circuit), C.POINTER(C.c_double), C.c_int32,
                                              C.POINTER(Stats)]
    lib.mps_apply_circuit_noalloc.restype = C.c_int32
    lib.mps_expect_paulisum.argtypes = [vp, C.POINTER(PauliSum), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.POINTER(Stats)]
    lib.mps_expect_paulisum.restype = C.c_int32
    lib.mps_plan_create.argtypes = [vp, C.POINTER(C.c_uint8), C.POINTER(Circuit), C.POINTER(PauliSum),
                                    C.POINTER(Trunc), C.POINTER(GradOpts), C.POINTER(vp)]
    lib.mps_plan_create.restype = C.c_int32
    lib.mps_energy_grad.argtypes = [vp, vp, C.c_int32, C.c_int32, C.POINTER(C.c_double), vp,
                                    C.POINTER(Stats)]
    lib.mps_energy_grad.restype = C.c_int32
    lib.mps_energy_grad_batched.argtypes = [vp, C.c_int32, vp, C.c_int32, C.c_int32, C.POINTER(C.c_double), vp,
                                            C.POINTER(Stats)]
    lib.mps_energy_grad_batched.restype = C.c_int32
    lib.mps_energy_grad_multi.argtypes = [C.POINTER(vp), C.c_int32, vp, C.c_int32, C.POINTER(C.c_double), vp,
                                          C.POINTER(Stats)]
    lib.mps_energy_grad_multi.restype = C.c_int32
    lib.mps_energy_grad_plans.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(vp), C.POINTER(C.c_double),
                                          C.POINTER(vp), C.POINTER(Stats)]
    lib.mps_energy_grad_plans.restype = C.c_int32
    lib.mps_energy_grad_alg1.argtypes = [vp, vp, C.c_int32, C.c_int32, C.POINTER(C.c_double), vp, vp,
                                         C.POINTER(Stats)]
    lib.mps_energy_grad_alg1.restype = C.c_int32
    lib.mps_energy_grad_psr.argtypes = [vp, vp, C.c_int32, C.POINTER(C.c_double), vp, vp, C.POINTER(Stats)]
    lib.mps_energy_grad_psr.restype = C.c_int32
    lib.mps_plan_batch_width.argtypes = [vp]
    lib.mps_plan_batch_width.restype = C.c_int32
    lib.mps_plan_energy.argtypes = [vp, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double),
                                    C.POINTER(Stats)]
    lib.mps_plan_energy.restype = C.c_int32
    lib.mps_state_export.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.mps_state_export.restype = C.c_int32
    lib.mps_state_import.argtypes = [vp, C.c_int32, C.POINTER(Trunc), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(vp)]
    lib.mps_state_import.restype = C.c_int32
    lib.mps_state_size.argtypes = [vp]
    lib.mps_state_size.restype = C.c_int64
    lib.mps_state_qubits.argtypes = [vp]
    lib.mps_state_qubits.restype = C.c_int32
    lib.mps_state_free.argtypes = [vp]
    lib.mps_state_free.restype = None
    lib.mps_plan_free.argtypes = [vp]
    lib.mps_plan_free.restype = None
    _lib = lib
    return lib
