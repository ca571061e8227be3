"""ctypes binding of libfbsde.so (the C ABI declared in include/fbsde.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Device buffers are torch tensors (their data_ptr), the stream
is torch's current HIP stream.  Importing works without a GPU (the symbols
are checked), calling a hot entry point without the library raises.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfbsde.so")

OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_HIP, ERR_NOMEM, ERR_NONFINITE = range(6)
SDE = {"gbm_diag": 0, "scaled_bm": 1}
DRV = {"bsb": 0, "hjb": 1, "ac": 2, "linear": 3}
TERM = {"norm2": 0, "loghalf": 1, "inv": 2, "linear": 3}
NET_KIND = {"mlp": 0, "resnet": 1, "u_fc": 2, "u_res": 3, "u_nais": 4}
PREC = {"fp32": 0, "bf16": 1}

EXPORTS = [
    "fbsde_plan_create", "fbsde_plan_destroy", "fbsde_param_count", "fbsde_param_layout", "fbsde_workspace_size",
    "fbsde_forward", "fbsde_forward_backward", "fbsde_adam_step", "fbsde_train_step", "fbsde_prolong",
    "fbsde_sample_normals", "fbsde_terminal_mean", "fbsde_terminal_states",
    "fbsde_profile_enable", "fbsde_profile_read", "fbsde_plan_config", "fbsde_plan_get_config",
    "fbsde_plan_autotune", "fbsde_plan_set_checkpointing", "fbsde_plan_status", "fbsde_batch_create", "fbsde_batch_step", "fbsde_batch_destroy",
    "fbsde_plan_set_unet_loss", "fbsde_unet_forward_backward", "fbsde_unet_nais_project", "fbsde_unet_states",
    "fbsde_plan_set_x0", "fbsde_forward_backward_noalloc",
    "fbsde_status_str", "fbsde_last_error",
]
PROF_NAMES = ["pack", "sde", "forward", "scan", "backward", "wgrad", "reduce", "adam"]


class FbsdeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fbsde status {status}: {msg}")
        self.status = status


class Problem(C.Structure):
    _fields_ = [("d", C.c_int32), ("T", C.c_double), ("x0_host", C.POINTER(C.c_double)),
                ("sde", C.c_int32), ("sde_p", C.c_double * 2),
                ("drv", C.c_int32), ("drv_p", C.c_double * 2),
                ("g", C.c_int32), ("g_p", C.c_double * 2)]


class BatchItem(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("params_dev", C.c_void_p), ("y0_dev", C.c_void_p),
                ("grad_dev", C.c_void_p), ("grad_y0_dev", C.c_void_p), ("loss_dev", C.c_void_p),
                ("m_dev", C.c_void_p), ("v_dev", C.c_void_p), ("m_y0_dev", C.c_void_p),
                ("v_y0_dev", C.c_void_p), ("ws_dev", C.c_void_p), ("seed", C.c_uint64)]


class Net(C.Structure):
    _fields_ = [("kind", C.c_int32), ("width", C.c_int32), ("depth", C.c_int32), ("prec", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libfbsde.so and declare every entry point; raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime: load it first so that this library
    # binds to the same runtime instead of a second copy
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise FbsdeError(ERR_HIP, f"{path} is not built; run __graft_entry__.build()")
    L = C.CDLL(path)
    vp, u64, i64 = C.c_void_p, C.c_uint64, C.c_int64
    L.fbsde_plan_create.argtypes = [C.POINTER(Problem), C.POINTER(Net), C.c_int32, i64, C.POINTER(vp)]
    L.fbsde_plan_set_checkpointing.argtypes = [vp, C.c_int32, i64]
    L.fbsde_plan_status.argtypes = [vp]
    L.fbsde_plan_destroy.argtypes = [vp]
    L.fbsde_plan_destroy.restype = None
    L.fbsde_param_count.argtypes = [vp, C.POINTER(i64)]
    L.fbsde_param_layout.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(C.c_int32)]
    L.fbsde_workspace_size.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.fbsde_forward.argtypes = [vp, vp, vp, u64, u64, vp, vp, vp]
    L.fbsde_forward_backward.argtypes = [vp, vp, vp, vp, vp, vp, u64, u64, vp, vp]
    L.fbsde_adam_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, C.c_double, C.c_double,
                                  C.c_double, C.c_double, C.c_double, vp]
    L.fbsde_train_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, C.c_double, C.c_double,
                                   C.c_double, C.c_double, C.c_double, u64, u64, vp, vp]
    L.fbsde_prolong.argtypes = [vp, vp, vp, vp, vp]
    L.fbsde_sample_normals.argtypes = [vp, u64, u64, vp, vp]
    L.fbsde_terminal_mean.argtypes = [vp, u64, u64, vp, vp, vp]
    L.fbsde_terminal_states.argtypes = [vp, vp, vp, vp, vp]
    L.fbsde_profile_enable.argtypes = [vp, C.c_int32]
    L.fbsde_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i64), C.c_int32]
    L.fbsde_plan_config.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]
    L.fbsde_plan_get_config.argtypes = [vp, C.POINTER(C.c_int32)]
    L.fbsde_plan_autotune.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, C.c_int32]
    L.fbsde_batch_create.argtypes = [C.POINTER(BatchItem), C.c_int32, C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.c_double, vp, C.c_int32, vp, C.POINTER(vp)]
    L.fbsde_batch_step.argtypes = [vp, vp]
    L.fbsde_batch_destroy.argtypes = [vp]
    L.fbsde_batch_destroy.restype = None
    L.fbsde_plan_set_unet_loss.argtypes = [vp, C.c_double, C.c_double]
    L.fbsde_unet_forward_backward.argtypes = [vp, vp, vp, vp, vp, u64, u64, vp, vp]
    L.fbsde_unet_nais_project.argtypes = [vp, vp, C.c_double, vp, vp]
    L.fbsde_unet_states.argtypes = [vp, vp, vp, vp, vp]
    L.fbsde_plan_set_x0.argtypes = [vp, C.POINTER(C.c_double)]
    L.fbsde_forward_backward_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, u64, u64, vp]
    L.fbsde_status_str.argtypes = [C.c_int]
    L.fbsde_status_str.restype = C.c_char_p
    L.fbsde_last_error.argtypes = []
    L.fbsde_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("fbsde_plan_destroy", "fbsde_batch_destroy", "fbsde_status_str", "fbsde_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(status: int) -> None:
    if status != OK:
        L = load()
        raise FbsdeError(status, L.fbsde_last_error().decode())


def make_problem(p: dict):
    """fbsde_problem from a problem dict; returns (struct, keep-alive array)."""
    d = int(p["d"])
    x0 = (C.c_double * d)(*[float(v) for v in p["x0"]])
    s = Problem()
    s.d = d
    s.T = float(p["T"])
    s.x0_host = C.cast(x0, C.POINTER(C.c_double))
    s.sde = SDE[p["sde"]]
    s.sde_p[0], s.sde_p[1] = float(p["sde_s"]), 0.0
    s.drv = DRV[p["drv"]]
    dp = list(p.get("drv_p", [0.0, 0.0])) + [0.0, 0.0]
    s.drv_p[0], s.drv_p[1] = float(dp[0]), float(dp[1])
    s.g = TERM[p["g"]]
    gp = list(p.get("g_p", [0.0, 0.0])) + [0.0, 0.0]
    s.g_p[0], s.g_p[1] = float(gp[0]), float(gp[1])
    return s, x0


def make_net(n: dict) -> Net:
    s = Net()
    s.kind = NET_KIND[n.get("kind", "mlp")]
    s.width = int(n["width"])
    s.depth = int(n.get("depth", 2))
    s.prec = PREC[n.get("prec", "fp32")]
    return s
