"""ctypes declarations of libnqs (mirrors include/nqs.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnqs.so")

NQS_OK, NQS_EINVAL, NQS_ENOMEM, NQS_EDEVICE, NQS_EUNSUPPORTED, NQS_ENUMERIC = range(6)
F64, F32, F16, BF16, FP8_E4M3 = range(5)
RBM, FFNN, RESCNN, CRBM = 0, 1, 2, 3
MOVE_FLIP, MOVE_EXCHANGE = 0, 1
TFIM, HEISENBERG = 0, 1
MAX_LAYERS = 8

DTYPE_CODES = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16, "e4m3": FP8_E4M3, "fp8": FP8_E4M3}

# every function the headers under include/ declare
EXPORTS = [
    "nqs_model_create", "nqs_model_set_params", "nqs_model_set_params_device", "nqs_model_destroy",
    "nqs_model_num_params", "nqs_model_prepare", "nqs_downcast", "nqs_sample", "nqs_sample_checked", "nqs_sample_batched", "nqs_sample_plan",
    "nqs_local_energy", "nqs_energy_stats", "nqs_energy_stats_noalloc",
    "nqs_logpsi_grad", "nqs_logpsi_grad_cols", "nqs_forces", "nqs_gram", "nqs_sample_gram", "nqs_sample_gram_factored",
    "nqs_sr_solve", "nqs_sr_solve_mixed", "nqs_sr_solve_complex", "nqs_sr_update", "nqs_sample_noisy", "nqs_local_energy_complex",
    "nqs_last_error",
    "nqs_version",
    "nqs_probe_rate",
]

PROBE_KINDS = {"fma_f32": 0, "log_f32": 1, "exp_f32": 2, "mfma_bf16_k16": 3, "mfma_bf16_k32": 4, "mfma_f32": 5,
               "mfma_f64": 6, "hbm_read": 7, "hbm_copy": 8, "mul_f32": 9, "xor_u32": 10, "dpp_add_f32": 11,
               "mulhi_u32": 12, "fma_f32_w1": 13, "fma_f32_w2": 14, "fma_f32_dep": 15,
               "lds_read": 16, "mfma_bf16_32": 17, "mfma_bf16_32_lds": 18,
               "mfma_bf16_32_lds_jit": 19}


class ModelDesc(ctypes.Structure):
    _fields_ = [("arch", ctypes.c_int32), ("n_visible", ctypes.c_int32), ("n_layers", ctypes.c_int32),
                ("widths", ctypes.c_int32 * MAX_LAYERS), ("marshall", ctypes.c_int32),
                ("lat_dim", ctypes.c_int32), ("lat_L", ctypes.c_int32)]


class HamDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dim", ctypes.c_int32), ("L", ctypes.c_int32), ("pbc", ctypes.c_int32),
                ("J", ctypes.c_double), ("h", ctypes.c_double)]


class SampleCfg(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_int64), ("n_sweeps", ctypes.c_int32), ("n_burnin", ctypes.c_int32),
                ("sweep_size", ctypes.c_int32), ("move", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("init_chains", ctypes.c_int32), ("seed", ctypes.c_uint64), ("step_offset", ctypes.c_uint64),
                ("instance_id", ctypes.c_uint32), ("chain_id_offset", ctypes.c_int64),
                ("lanes_per_chain", ctypes.c_int32), ("refresh_sweeps", ctypes.c_int32)]


class SampleJob(ctypes.Structure):
    _fields_ = [("model", ctypes.c_void_p), ("cfg", SampleCfg), ("chain_state", ctypes.c_void_p),
                ("samples", ctypes.c_void_p), ("logpsi", ctypes.c_void_p), ("n_accepted", ctypes.c_void_p),
                ("trace", ctypes.c_void_p)]


class SampleDiag(ctypes.Structure):
    _fields_ = [("stuck_after", ctypes.c_int32), ("nonfinite", ctypes.c_void_p), ("longest_stuck", ctypes.c_void_p),
                ("drift", ctypes.c_void_p), ("total_nonfinite", ctypes.c_uint64), ("chains_stuck", ctypes.c_int64),
                ("max_drift", ctypes.c_float)]


class LaunchPlan(ctypes.Structure):
    _fields_ = [("lanes_per_chain", ctypes.c_int32), ("units_per_lane", ctypes.c_int32),
                ("chains_per_block", ctypes.c_int32), ("table_in_lds", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("tuned_ms", ctypes.c_float)]


LANES_TUNED = -2


class Trace(ctypes.Structure):
    _fields_ = [("n_chains_traced", ctypes.c_int32), ("site", ctypes.c_void_p), ("ubits", ctypes.c_void_p),
                ("delta", ctypes.c_void_p), ("accepted", ctypes.c_void_p)]


_lib = None


class NqsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libnqs status {status}: {msg}")
        self.status = status


def load() -> ctypes.CDLL:
    """Load libnqs.so; raises if the HIP library has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libnqs.so not found at {LIB_PATH}: build it with paper_2601_20782_amd/build.py "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    st = ctypes.c_int
    sig = {
        "nqs_model_create": ([P, P, i64, P], st),
        "nqs_model_set_params": ([P, P, i64], st),
        "nqs_model_set_params_device": ([P, P, i64, P], st),
        "nqs_model_destroy": ([P], st),
        "nqs_model_num_params": ([P], i64),
        "nqs_model_prepare": ([P, i32, P], st),
        "nqs_downcast": ([P, i64, i32, P, P, P], st),
        "nqs_sample": ([P, P, P, P, P, P, P, P], st),
        "nqs_sample_batched": ([P, i32, i32, P], st),
        "nqs_sample_plan": ([P, P, P, P], st),
        "nqs_sample_checked": ([P, P, P, P, P, P, P, P, P], st),
        "nqs_local_energy": ([P, P, P, i64, i32, P, P], st),
        "nqs_energy_stats": ([P, i64, i64, P, P], st),
        "nqs_energy_stats_noalloc": ([P, i64, i64, P, P], st),
        "nqs_logpsi_grad": ([P, P, i64, P, P, P, P, P], st),
        "nqs_forces": ([P, P, i64, i64, P, P, P], st),
        "nqs_gram": ([P, i64, i64, i32, P, P], st),
        "nqs_logpsi_grad_cols": ([P, P, i64, i64, i64, P, P], st),
        "nqs_sample_gram": ([P, P, i64, i64, P, P], st),
        "nqs_sample_gram_factored": ([P, P, i64, P, P], st),
        "nqs_sr_solve": ([P, P, i64, ctypes.c_double, ctypes.c_double, i32, P, P, P, P], st),
        "nqs_sr_solve_complex": ([P, P, P, i64, ctypes.c_double, ctypes.c_double, i32, P, P, P, P], st),
        "nqs_probe_rate": ([i32, i64, P, P, P, P], st),
        "nqs_sr_solve_mixed": ([P, P, i64, ctypes.c_double, i32, ctypes.c_double, i32, P, P, P, P, P, P], st),
        "nqs_sr_update": ([P, P, i64, P, ctypes.c_double, P, P], st),
        "nqs_sample_noisy": ([P, P, ctypes.c_double, ctypes.c_uint64, P, P, P, P, P], st),
        "nqs_local_energy_complex": ([P, P, P, i64, i32, P, P, P], st),
        "nqs_last_error": ([], ctypes.c_char_p),
        "nqs_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != NQS_OK:
        raise NqsError(status, load().nqs_last_error().decode())
