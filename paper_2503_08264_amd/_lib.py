"""ctypes mirror of include/qem.h and the loader of the in-tree libqem.so.

Loading fails loudly when the library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_uint32, c_uint64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libqem.so")

QEM_OK, QEM_E_INVALID, QEM_E_SHAPE, QEM_E_UNSUPPORTED, QEM_E_DEVICE, QEM_E_NONFINITE, QEM_E_STATE = range(7)
STATUS_NAMES = {0: "QEM_OK", 1: "QEM_E_INVALID", 2: "QEM_E_SHAPE", 3: "QEM_E_UNSUPPORTED",
                4: "QEM_E_DEVICE", 5: "QEM_E_NONFINITE", 6: "QEM_E_STATE"}
PREC = {"fp64": 0, "fp32": 1, "bf16exp": 2}
QFAMILY = {"gauss": 0, "gamma": 1, "gamma_ef": 2, "bernoulli": 3, "dirichlet": 4, "categorical": 5}
PRIOR = {"normal": 0, "gamma": 1, "gamma_parents": 2, "normal_logscale": 3, "bernoulli_logit": 4, "dirichlet": 5, "categorical": 6}
OBS = {"gauss": 0, "poisson": 1, "bernoulli_logit": 2, "detection": 3, "categorical": 4, "gauss_mixture": 5}
T_QPARAM, T_MEMA, T_MONE, T_Z, T_U, T_F, T_UT, T_MSG, T_W, T_ROOTL, T_LOGPHAT, T_STATUS, T_PAIR_M, T_PAIR_W, T_FSHIFT = range(15)
DT_F64, DT_F32, DT_U32, DT_BF16 = range(4)
FLAG_NONFINITE, FLAG_VAR_FLOOR, FLAG_GAMMA_MEAN, FLAG_NEG_INF_ROW = 0x1, 0x2, 0x4, 0x8
CREATE_NO_TABLES = 0x1
CREATE_CHAIN_TABLES = 0x2
PHASES = ["sample", "unary", "pairtable", "plate_fwd", "plate_bwd", "chain_fwd", "chain_bwd",
          "tp_fwd", "tp_bwd", "childsum", "root", "moments", "mstep"]


class NodeDesc(ctypes.Structure):
    _fields_ = [("n", c_int32), ("dim", c_int32), ("qfamily", c_int32), ("prior", c_int32),
                ("parent0", c_int32), ("parent1", c_int32), ("parent_index", POINTER(c_int32)),
                ("a", c_double), ("b", c_double), ("var", c_double), ("shape", c_double), ("rate", c_double),
                ("chain_len", c_int32), ("init_b", c_double), ("init_var", c_double),
                ("q0a", c_double), ("q0b", c_double)]


class ObsDesc(ctypes.Structure):
    _fields_ = [("node", c_int32), ("kind", c_int32), ("n_per", c_int32), ("n_cov", c_int32),
                ("coef", c_int32), ("var", c_double), ("x", c_void_p), ("cov", c_void_p)]


class ModelDesc(ctypes.Structure):
    _fields_ = [("n_nodes", c_int32), ("n_obs", c_int32), ("nodes", POINTER(NodeDesc)),
                ("obs", POINTER(ObsDesc))]


class TensorInfo(ctypes.Structure):
    _fields_ = [("offset", c_size_t), ("bytes", c_size_t), ("dtype", c_int32), ("ndim", c_int32),
                ("shape", c_int64 * 4)]


# name -> (restype, argtypes)
SIGNATURES = {
    "qem_create": (c_int32, [POINTER(c_void_p), POINTER(ModelDesc), c_int32, c_int32, c_void_p]),
    "qem_create_ex": (c_int32, [POINTER(c_void_p), POINTER(ModelDesc), c_int32, c_int32, c_uint32, c_void_p]),
    "qem_destroy": (None, [c_void_p]),
    "qem_last_error": (c_char_p, [c_void_p]),
    "qem_workspace_bytes": (c_size_t, [c_void_p]),
    "qem_bind_workspace": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "qem_init": (c_int32, [c_void_p, c_int32]),
    "qem_init_from_q": (c_int32, [c_void_p, c_int32]),
    "qem_tensor": (c_int32, [c_void_p, c_int32, c_int32, POINTER(TensorInfo)]),
    "qem_sample": (c_int32, [c_void_p, c_uint64, c_uint64]),
    "qem_logfactors": (c_int32, [c_void_p]),
    "qem_contract_fwd": (c_int32, [c_void_p]),
    "qem_contract_bwd": (c_int32, [c_void_p, c_void_p]),
    "qem_moments": (c_int32, [c_void_p]),
    "qem_mstep": (c_int32, [c_void_p, c_double]),
    "qem_step": (c_int32, [c_void_p, c_uint64, c_uint64, c_double]),
    "qem_set_ema": (c_int32, [c_void_p, c_double, c_int32]),
    "qem_run": (c_int32, [c_void_p, c_uint64, c_uint64, c_double, c_int32]),
    "qem_read_status": (c_int32, [c_void_p, POINTER(c_uint32), POINTER(c_uint32), POINTER(c_double)]),
    "qem_enc_features": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    "qem_enc_pool": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "qem_enc_features_ctx": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "qem_enc_fwd": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "qem_enc_loss": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "qem_enc_scratch_bytes": (c_size_t, [c_int32]),
    "qem_enc_bwd": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "qem_enc_bwd_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "qem_enc_adam": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_float, c_float,
                              c_float, c_float, c_void_p]),
    "qem_enc_to_bf16": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "qem_enc_apply": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "qem_enc_targets": (c_int32, [c_void_p, c_int32, c_double, c_void_p, c_void_p, c_void_p]),
    "qem_ess": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "qem_enc_apply_residual": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "qem_stream_probe": (c_int32, [c_void_p, c_size_t, c_int32, c_void_p, c_void_p]),
    "qem_timing": (c_int32, [c_void_p, c_int32]),
    "qem_timing_read": (c_int32, [c_void_p, c_int32, c_int32, POINTER(c_double), POINTER(c_int64)]),
}

_LIB = None


class QEMError(RuntimeError):
    pass


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libqem.so (built by paper_2503_08264_amd.build); raise if absent."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise QEMError(f"{path} is missing: build it with `python -m paper_2503_08264_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def check(lib, ctx, status: int, what: str):
    if status != QEM_OK:
        msg = lib.qem_last_error(ctx)
        raise QEMError(f"{what}: {STATUS_NAMES.get(status, status)}: {msg.decode() if msg else ''}")
