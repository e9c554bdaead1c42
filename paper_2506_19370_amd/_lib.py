"""ctypes binding of ``libfcsdnn.so`` (the C ABI declared in include/fcsdnn.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  PyTorch provides device memory (workspaces, fields) and the HIP
stream.  Importing fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# PyTorch first: its HIP runtime (the same soname as ROCm's) is then the one
# the library binds to, so that both share one runtime, its devices and
# streams.  Loaded the other way round, PyTorch runs on the system runtime,
# which it was not built against.
import torch  # noqa: F401,E402

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libfcsdnn.so")

if not os.path.exists(LIBPATH):
    raise ImportError(f"{LIBPATH} is missing: build it with `python -m paper_2506_19370_amd.build`")

lib = ctypes.CDLL(LIBPATH)

c_int32_p = ctypes.POINTER(ctypes.c_int32)
vp = ctypes.c_void_p

FCS_OK, FCS_EINVAL, FCS_EOVERLAP, FCS_ENOMEM, FCS_ENONFINITE, FCS_EHIP, FCS_ESTATE = range(7)
STATUS = {0: "OK", 1: "EINVAL", 2: "EOVERLAP", 3: "ENOMEM", 4: "ENONFINITE", 5: "EHIP", 6: "ESTATE"}
SIDE = {"INTERNAL": 0, "INFLOW": 1, "OUTFLOW": 2, "SLIP": 3, "EXACT": 4, "NOSLIP": 5}
PATCH = {"I": 0, "S": 1, "C1": 2, "C2": 3}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
AV = {"off": 0, "modal": 1, "sdnn": 2, "frozen": 3}
OP = {"d1": 0, "d2": 1, "filter": 2, "smear": 3}
FIELD = {"rho": 0, "mx": 1, "my": 2, "E": 3, "p": 4, "mach": 5, "mu": 6, "tau0": 7, "tau1": 8, "muhat": 9}
SDNN_NPARAM = 64 * 16 + 64 + 64 * 64 + 64 + 3 * 64 + 3


class FcsError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"fcs status {STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("c_mu", ctypes.c_double),
        ("dt_fixed", ctypes.c_double),
        ("fc_d", ctypes.c_int32), ("fc_C", ctypes.c_int32), ("n_f", ctypes.c_int32), ("n_v", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("av_mode", ctypes.c_int32), ("filter", ctypes.c_int32),
        ("use_graph", ctypes.c_int32), ("autotune", ctypes.c_int32), ("visc_all_lines", ctypes.c_int32),
        ("sdnn_weights", ctypes.POINTER(ctypes.c_float)),
        ("vortex", ctypes.c_double * 5),
        ("smear", ctypes.c_int32),
    ]


class PatchDesc(ctypes.Structure):
    _fields_ = [
        ("type", ctypes.c_int32), ("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
        ("x", ctypes.POINTER(ctypes.c_double)), ("y", ctypes.POINTER(ctypes.c_double)),
        ("mask", ctypes.POINTER(ctypes.c_uint8)),
        ("side", ctypes.c_int32 * 4), ("notch", ctypes.c_int32),
        ("inflow", ctypes.c_double * 4),
    ]


class Stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("stages", ctypes.c_int64), ("t", ctypes.c_double),
                ("dt", ctypes.c_double), ("mass", ctypes.c_double), ("energy", ctypes.c_double),
                ("npoints", ctypes.c_int64), ("stage_variant", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def _sig(name, res, args):
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args
    return f


_i = ctypes.c_int32
_i64 = ctypes.c_int64
_d = ctypes.c_double
_sz = ctypes.c_size_t
fcs_version = _sig("fcs_version", ctypes.c_int, [])
fcs_create = _sig("fcs_create", _i, [ctypes.POINTER(Params), _i, ctypes.POINTER(PatchDesc), ctypes.POINTER(vp)])
fcs_workspace_size = _sig("fcs_workspace_size", _i, [vp, ctypes.POINTER(_sz)])
fcs_bind = _sig("fcs_bind", _i, [vp, vp, _sz, vp])
fcs_set_state = _sig("fcs_set_state", _i, [vp, _i, _i, vp, _i])
fcs_set_time = _sig("fcs_set_time", _i, [vp, _d])
fcs_set_tau = _sig("fcs_set_tau", _i, [vp, _i, vp])
fcs_advance = _sig("fcs_advance", _i, [vp, _i64, ctypes.POINTER(_d)])
fcs_get_field = _sig("fcs_get_field", _i, [vp, _i, _i, vp, _i])
fcs_stats = _sig("fcs_stats", _i, [vp, ctypes.POINTER(Stats)])
fcs_autotune_times = _sig("fcs_autotune_times", _i, [vp, _i, ctypes.POINTER(_d)])
fcs_retune = _sig("fcs_retune", _i, [vp])
fcs_set_stage_variant = _sig("fcs_set_stage_variant", _i, [vp, _i])
fcs_profile_stage = _sig("fcs_profile_stage", _i, [vp, _i, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d)])
fcs_profile_enable = _sig("fcs_profile_enable", _i, [vp, _i])
fcs_profile_read = _sig("fcs_profile_read", _i, [vp, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d),
                                                 ctypes.POINTER(_i64), ctypes.POINTER(_d)])
fcs_last_error = _sig("fcs_last_error", ctypes.c_char_p, [vp])
fcs_destroy = _sig("fcs_destroy", None, [vp])
fcs_fc_continuation = _sig("fcs_fc_continuation", _i, [_i, _i, vp, vp])
fcs_fc_operator = _sig("fcs_fc_operator", _i, [_i, _i, _i, _i, vp])
fcs_sweep_create = _sig("fcs_sweep_create", _i, [_i, vp, _i, _i, _i, _i, ctypes.POINTER(vp)])
fcs_sweep_workspace_size = _sig("fcs_sweep_workspace_size", _i, [vp, ctypes.POINTER(_sz)])
fcs_sweep_bind = _sig("fcs_sweep_bind", _i, [vp, vp, _sz, vp])
fcs_sweep_run = _sig("fcs_sweep_run", _i, [vp, vp, vp, vp])
fcs_sweep_profile = _sig("fcs_sweep_profile", _i, [vp, _i, ctypes.POINTER(_d), ctypes.POINTER(_d),
                                                   ctypes.POINTER(_d), ctypes.POINTER(_i64)])
fcs_sweep_points = _sig("fcs_sweep_points", _i, [vp, ctypes.POINTER(_i64)])
fcs_gemm_variant_count = _sig("fcs_gemm_variant_count", _i, [_i])
fcs_gemm_variant_name = _sig("fcs_gemm_variant_name", _i, [_i, _i, ctypes.c_char_p, _i])
fcs_sweep_set_variant = _sig("fcs_sweep_set_variant", _i, [vp, _i])
fcs_sweep_destroy = _sig("fcs_sweep_destroy", None, [vp])
fcs_sweep_autotune = _sig("fcs_sweep_autotune", _i, [vp, vp, vp, vp, vp])
fcs_sdnn_infer = _sig("fcs_sdnn_infer", _i, [vp, vp, _i64, vp, vp, vp])
fcs_modal_infer = _sig("fcs_modal_infer", _i, [vp, _i64, vp, vp])
fcs_sdnn_train_workspace = _sig("fcs_sdnn_train_workspace", _sz, [_i])
fcs_sdnn_train_step = _sig("fcs_sdnn_train_step", _i, [vp, vp, vp, _i, ctypes.c_float, vp, vp, vp, _i, vp, vp, _i,
                                                       vp, _sz, vp])
fcs_sdnn_train_step_noalloc = _sig("fcs_sdnn_train_step_noalloc", _i, [vp, vp, vp, _i, ctypes.c_float, vp, vp, vp,
                                                                       _i, vp, vp, _i, vp])
SDNN_TRAIN_MAX_BATCH = 8192
fcs_lines_workspace = _sig("fcs_lines_workspace", _sz, [_i, _i64])
fcs_lines_apply = _sig("fcs_lines_apply", _i, [_i, _i64, _i, _i, _i, vp, vp, vp, _sz, vp])

EXPORTED = [
    "fcs_version", "fcs_create", "fcs_workspace_size", "fcs_bind", "fcs_set_state", "fcs_set_time",
    "fcs_set_tau", "fcs_advance", "fcs_get_field", "fcs_stats", "fcs_autotune_times", "fcs_retune", "fcs_set_stage_variant", "fcs_profile_stage", "fcs_profile_enable", "fcs_profile_read",
    "fcs_last_error", "fcs_destroy", "fcs_fc_continuation", "fcs_fc_operator", "fcs_sweep_create",
    "fcs_sweep_workspace_size", "fcs_sweep_bind", "fcs_sweep_run", "fcs_sweep_profile", "fcs_sweep_points",
    "fcs_sweep_destroy", "fcs_sweep_autotune", "fcs_sdnn_infer", "fcs_modal_infer", "fcs_sdnn_train_workspace", "fcs_sdnn_train_step",
    "fcs_sdnn_train_step_noalloc", "fcs_lines_workspace", "fcs_lines_apply", "fcs_gemm_variant_count", "fcs_sweep_set_variant",
    "fcs_gemm_variant_name",
]


def check(status, ctx=None):
    if status != FCS_OK:
        msg = fcs_last_error(ctx).decode() if ctx else ""
        raise FcsError(status, msg)


def fc_operator(n: int, d: int, C: int, kind: str = "d1") -> np.ndarray:
    out = np.zeros((n, n))
    check(fcs_fc_operator(n, d, C, OP[kind], out.ctypes.data))
    return out


def gemm_variant_name(precision: str, index: int) -> str:
    buf = ctypes.create_string_buffer(96)
    check(fcs_gemm_variant_name(PREC[precision], int(index), buf, 96))
    return buf.value.decode()


def fc_continuation(d: int, C: int):
    Q = np.zeros((d, d))
    A = np.zeros((C, d))
    check(fcs_fc_continuation(d, C, Q.ctypes.data, A.ctypes.data))
    return Q, A
