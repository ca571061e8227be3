"""ctypes wrapper of the FP64 C oracle (liboracle.so).  TEST INFRASTRUCTURE.

Problem and network descriptions are plain dicts so that callers never need
the product package.  Every routine cites the passage of Güler, Laignelet and
Parpas (arXiv 1910.11623) it follows in ``oracle.h``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

SDE = {"gbm_diag": 0, "scaled_bm": 1}
DRV = {"bsb": 0, "hjb": 1, "ac": 2, "linear": 3}
TERM = {"norm2": 0, "loghalf": 1, "inv": 2, "linear": 3}
NET = {"mlp": 0, "resnet": 1}


def build() -> str:
    """Compile liboracle.so with gcc (plain C99, -O2, no fast-math; OpenMP
    over path chunks, whose sums are combined in a fixed order)."""
    src = os.path.join(HERE, "oracle.c")
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-Wall", "-shared", "-fPIC", "-o", LIB_PATH, src, "-lm"]
    subprocess.check_call(cmd)
    return LIB_PATH


class _Problem(C.Structure):
    _fields_ = [("d", C.c_int), ("T", C.c_double), ("x0", C.POINTER(C.c_double)),
                ("sde", C.c_int), ("sde_s", C.c_double),
                ("drv", C.c_int), ("drv_p", C.c_double * 2),
                ("g", C.c_int), ("g_p", C.c_double * 2)]


class _Net(C.Structure):
    _fields_ = [("kind", C.c_int), ("width", C.c_int), ("depth", C.c_int), ("bf16", C.c_int)]


class _UNet(C.Structure):
    _fields_ = [("arch", C.c_int), ("width", C.c_int), ("depth", C.c_int), ("eps", C.c_double)]


UARCH = {"fc": 0, "res": 1, "nais": 2}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(
                os.path.join(HERE, "oracle.c")):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_param_count.restype = C.c_int64
        L.orc_param_count.argtypes = [C.POINTER(_Problem), C.POINTER(_Net), C.c_int]
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_normals.argtypes = [C.c_uint64, C.c_uint64, C.c_int, C.c_int64, C.c_int, dp]
        L.orc_loss_grad.restype = C.c_int
        L.orc_loss_grad.argtypes = [C.POINTER(_Problem), C.POINTER(_Net), C.c_int, C.c_int64,
                                    dp, C.c_double, dp, C.c_uint64, C.c_uint64,
                                    dp, dp, dp, dp, dp, dp]
        L.orc_paths.restype = C.c_int
        L.orc_paths.argtypes = [C.POINTER(_Problem), C.POINTER(_Net), C.c_int, dp, C.c_double,
                                C.c_uint64, C.c_uint64, C.POINTER(C.c_int64), C.c_int64, dp, dp]
        L.orc_loss_exact_bsb.restype = C.c_int
        L.orc_loss_exact_bsb.argtypes = [C.POINTER(_Problem), C.c_int, C.c_int64, C.c_double, dp,
                                         C.c_uint64, C.c_uint64, C.c_int, dp]
        L.orc_loss_given_z.restype = C.c_int
        L.orc_loss_given_z.argtypes = [C.POINTER(_Problem), C.c_int, C.c_int64, C.c_double, dp, C.c_uint64,
                                       C.c_uint64, dp, C.c_double, dp]
        L.orc_adam.argtypes = [C.c_int64, dp, dp, dp, dp, C.c_int64, C.c_double, C.c_double,
                               C.c_double, C.c_double]
        L.orc_prolong.restype = C.c_int
        L.orc_prolong.argtypes = [C.POINTER(_Problem), C.POINTER(_Net), C.c_int, C.c_int, dp, dp]
        L.orc_round_bf16.restype = C.c_double
        L.orc_round_bf16.argtypes = [C.c_double]
        L.orc_unet_param_count.restype = C.c_int64
        L.orc_unet_param_count.argtypes = [C.POINTER(_Problem), C.POINTER(_UNet)]
        L.orc_unet_loss_grad.restype = C.c_int
        L.orc_unet_loss_grad.argtypes = [C.POINTER(_Problem), C.POINTER(_UNet), C.c_int, C.c_int64, dp, dp,
                                         C.c_uint64, C.c_uint64, C.c_double, dp, dp, dp, dp]
        L.orc_unet_loss_given_uz.restype = C.c_int
        L.orc_unet_loss_given_uz.argtypes = [C.POINTER(_Problem), C.c_int, C.c_int64, dp, C.c_uint64, C.c_uint64,
                                             dp, dp, C.c_double, dp]
        L.orc_unet_eval.restype = C.c_int
        L.orc_unet_eval.argtypes = [C.POINTER(_Problem), C.POINTER(_UNet), dp, C.c_int64, dp, dp, dp, dp]
        L.orc_unet_nais_project.restype = C.c_int
        L.orc_unet_nais_project.argtypes = [C.POINTER(_Problem), C.POINTER(_UNet), dp, C.c_double]
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's path loop (results do not depend on it)."""
    C.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
    lib()


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _problem(p: dict):
    x0 = np.ascontiguousarray(p["x0"], dtype=np.float64)
    s = _Problem()
    s.d = int(p["d"])
    s.T = float(p["T"])
    s.x0 = _ptr(x0)
    s.sde = SDE[p["sde"]]
    s.sde_s = float(p["sde_s"])
    s.drv = DRV[p["drv"]]
    dpv = list(p.get("drv_p", [0.0, 0.0])) + [0.0, 0.0]
    s.drv_p[0], s.drv_p[1] = dpv[0], dpv[1]
    s.g = TERM[p["g"]]
    gpv = list(p.get("g_p", [0.0, 0.0])) + [0.0, 0.0]
    s.g_p[0], s.g_p[1] = gpv[0], gpv[1]
    return s, x0  # keep x0 alive


def _net(n: dict):
    s = _Net()
    s.kind = NET[n.get("kind", "mlp")]
    s.width = int(n["width"])
    s.depth = int(n.get("depth", 2))
    s.bf16 = int(bool(n.get("bf16", False)))
    return s


def param_count(problem: dict, net: dict, N: int) -> int:
    ps, _keep = _problem(problem)
    ns = _net(net)
    return int(lib().orc_param_count(C.byref(ps), C.byref(ns), int(N)))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(o[i]) for i in range(4)]


def normals(seed: int, it: int, N: int, M: int, d: int) -> np.ndarray:
    xi = np.empty((N, M, d), dtype=np.float64)
    lib().orc_normals(C.c_uint64(seed), C.c_uint64(it), N, M, d, _ptr(xi))
    return xi


def loss_grad(problem: dict, net: dict, N: int, M: int, params, y0: float, *, xi=None,
              seed: int = 0, it: int = 0, want_grad: bool = True, want_paths: bool = False):
    """Loss (1/M) sum_m (Y_N - g(X_N))^2 and its gradient (Sec. 2.2)."""
    ps, _keep = _problem(problem)
    ns = _net(net)
    npar = param_count(problem, net, N)
    params = np.ascontiguousarray(params, dtype=np.float64)
    if params.shape != (npar,):
        raise ValueError(f"params must have shape ({npar},), got {params.shape}")
    d = int(problem["d"])
    if xi is not None:
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        if xi.shape != (N, M, d):
            raise ValueError("xi must be [N][M][d]")
    loss = np.zeros(1)
    grad = np.zeros(npar) if want_grad else None
    gy0 = np.zeros(1) if want_grad else None
    XN = np.zeros((M, d)) if want_paths else None
    YN = np.zeros(M) if want_paths else None
    Yp = np.zeros((N + 1, M)) if want_paths else None
    rc = lib().orc_loss_grad(C.byref(ps), C.byref(ns), int(N), int(M), _ptr(params), float(y0),
                             _ptr(xi), C.c_uint64(seed), C.c_uint64(it), _ptr(loss), _ptr(grad),
                             _ptr(gy0), _ptr(XN), _ptr(YN), _ptr(Yp))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    out = {"loss": float(loss[0])}
    if want_grad:
        out["grad"] = grad
        out["grad_y0"] = float(gy0[0])
    if want_paths:
        out.update(XN=XN, YN=YN, Ypath=Yp)
    return out


def paths(problem: dict, net: dict, N: int, params, y0: float, idx, *, seed: int = 0, it: int = 0):
    """Terminal (Y_N, X_N) of the selected path indices of a full batch."""
    ps, _keep = _problem(problem)
    ns = _net(net)
    params = np.ascontiguousarray(params, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    d = int(problem["d"])
    YN = np.zeros(idx.size)
    XN = np.zeros((idx.size, d))
    rc = lib().orc_paths(C.byref(ps), C.byref(ns), int(N), _ptr(params), float(y0), C.c_uint64(seed),
                         C.c_uint64(it), idx.ctypes.data_as(C.POINTER(C.c_int64)), idx.size,
                         _ptr(YN), _ptr(XN))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return YN, XN


def loss_exact_bsb(problem: dict, N: int, M: int, y0: float, *, xi=None, seed=0, it=0, flip=False):
    ps, _keep = _problem(problem)
    d = int(problem["d"])
    if xi is not None:
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        assert xi.shape == (N, M, d)
    loss = np.zeros(1)
    rc = lib().orc_loss_exact_bsb(C.byref(ps), int(N), int(M), float(y0), _ptr(xi),
                                  C.c_uint64(seed), C.c_uint64(it), int(bool(flip)), _ptr(loss))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return float(loss[0])


def loss_given_z(problem: dict, N: int, M: int, y0: float, Z, *, xi=None, seed=0, it=0, drv_sign=1.0):
    """Loss of the Euler scheme driven by the given Z[n][m][i] (no network)."""
    ps, _keep = _problem(problem)
    d = int(problem["d"])
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    if Z.shape != (N, M, d):
        raise ValueError("Z must be [N][M][d]")
    if xi is not None:
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        assert xi.shape == (N, M, d)
    loss = np.zeros(1)
    rc = lib().orc_loss_given_z(C.byref(ps), int(N), int(M), float(y0), _ptr(xi), C.c_uint64(seed),
                                C.c_uint64(it), _ptr(Z), float(drv_sign), _ptr(loss))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return float(loss[0])


def adam(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step t >= 1 on float64 arrays (Kingma & Ba)."""
    for a in (theta, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam(theta.size, _ptr(theta), _ptr(g), _ptr(m), _ptr(v), int(t), lr, b1, b2, eps)


def prolong(problem: dict, net: dict, Nc: int, Nf: int, pc):
    ps, _keep = _problem(problem)
    ns = _net(net)
    pc = np.ascontiguousarray(pc, dtype=np.float64)
    pf = np.zeros(param_count(problem, net, Nf))
    rc = lib().orc_prolong(C.byref(ps), C.byref(ns), int(Nc), int(Nf), _ptr(pc), _ptr(pf))
    if rc != 0:
        raise ValueError("oracle rejected the prolongation")
    return pf


def round_bf16(x: float) -> float:
    return float(lib().orc_round_bf16(float(x)))


# ------------------------------------------------ the paper's own formulation
def _unet(n: dict):
    s = _UNet()
    s.arch = UARCH[n.get("arch", "fc")]
    s.width = int(n["width"])
    s.depth = int(n.get("depth", 3))
    s.eps = float(n.get("eps", 0.01))
    return s


def unet_param_count(problem: dict, net: dict) -> int:
    ps, _keep = _problem(problem)
    return int(lib().orc_unet_param_count(C.byref(ps), C.byref(_unet(net))))


def unet_loss_grad(problem: dict, net: dict, N: int, M: int, params, *, xi=None, seed: int = 0, it: int = 0,
                   kappa: float = 0.0, want_grad: bool = True, want_uz: bool = False):
    """Residual loss of Sec. 2.2 eq. (loss) with Y_n = u(t_n, X_n) and
    Z_n = grad u (one network for every step), the optional terminal-gradient
    penalty kappa |Z_N - grad g(X_N)|^2, and the exact parameter gradient."""
    ps, _keep = _problem(problem)
    ns = _unet(net)
    npar = unet_param_count(problem, net)
    params = np.ascontiguousarray(params, dtype=np.float64)
    if params.shape != (npar,):
        raise ValueError(f"params must have shape ({npar},), got {params.shape}")
    d = int(problem["d"])
    if xi is not None:
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        if xi.shape != (N, M, d):
            raise ValueError("xi must be [N][M][d]")
    loss = np.zeros(1)
    grad = np.zeros(npar) if want_grad else None
    U = np.zeros((N + 1, M)) if want_uz else None
    Z = np.zeros((N + 1, M, d)) if want_uz else None
    rc = lib().orc_unet_loss_grad(C.byref(ps), C.byref(ns), int(N), int(M), _ptr(params), _ptr(xi),
                                  C.c_uint64(seed), C.c_uint64(it), float(kappa), _ptr(loss), _ptr(grad),
                                  _ptr(U), _ptr(Z))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    out = {"loss": float(loss[0])}
    if want_grad:
        out["grad"] = grad
    if want_uz:
        out.update(U=U, Z=Z)
    return out


def unet_loss_given_uz(problem: dict, N: int, M: int, U, Z, *, xi=None, seed=0, it=0, kappa=0.0):
    ps, _keep = _problem(problem)
    d = int(problem["d"])
    U = np.ascontiguousarray(U, dtype=np.float64)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    if U.shape != (N + 1, M) or Z.shape != (N + 1, M, d):
        raise ValueError("U must be [N+1][M] and Z [N+1][M][d]")
    if xi is not None:
        xi = np.ascontiguousarray(xi, dtype=np.float64)
    loss = np.zeros(1)
    rc = lib().orc_unet_loss_given_uz(C.byref(ps), int(N), int(M), _ptr(xi), C.c_uint64(seed), C.c_uint64(it),
                                      _ptr(U), _ptr(Z), float(kappa), _ptr(loss))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return float(loss[0])


def unet_eval(problem: dict, net: dict, params, t, X):
    """u(t, x) and grad_x u(t, x) of the network at the rows (t[i], X[i])."""
    ps, _keep = _problem(problem)
    ns = _unet(net)
    params = np.ascontiguousarray(params, dtype=np.float64)
    t = np.ascontiguousarray(t, dtype=np.float64).ravel()
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(t.size, int(problem["d"]))
    u = np.zeros(t.size)
    Z = np.zeros_like(X)
    rc = lib().orc_unet_eval(C.byref(ps), C.byref(ns), _ptr(params), t.size, _ptr(t), _ptr(X), _ptr(u), _ptr(Z))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return u, Z


def unet_nais_project(problem: dict, net: dict, params, c: float):
    """In-place NAIS projection of every R_k (|R_k^T R_k|_F <= c)."""
    ps, _keep = _problem(problem)
    assert params.dtype == np.float64 and params.flags.c_contiguous
    rc = lib().orc_unet_nais_project(C.byref(ps), C.byref(_unet(net)), _ptr(params), float(c))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
