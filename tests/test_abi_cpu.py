"""CPU-side checks of the C ABI: the library loads, exports every symbol that
include/fbsde.h declares, and rejects invalid arguments on the host before
touching the GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1910_11623_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "fbsde.h")).read()
    return sorted(set(re.findall(r"\b(fbsde_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libfbsde.so not built")
    return B.load()


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTS)


def test_status_strings(lib):
    for s in range(6):
        assert lib.fbsde_status_str(s)


def _create(lib, prob, net, N, M):
    ps, keep = B.make_problem(prob)
    ns = B.make_net(net)
    h = C.c_void_p()
    st = lib.fbsde_plan_create(C.byref(ps), C.byref(ns), N, M, C.byref(h))
    return st, h


BASE = dict(d=3, T=1.0, x0=[1.0, 0.5, 1.0], sde="gbm_diag", sde_s=0.4, drv="bsb", drv_p=[0.05, 0],
            g="norm2", g_p=[0, 0])


@pytest.mark.parametrize("change,expect", [
    (dict(d=0, x0=[]), B.ERR_INVALID),
    (dict(T=0.0), B.ERR_INVALID),
    (dict(T=float("nan")), B.ERR_INVALID),
    (dict(x0=[1.0, float("inf"), 0.0]), B.ERR_INVALID),
])
def test_invalid_problem(lib, change, expect):
    st, h = _create(lib, dict(BASE, **change), dict(width=4, depth=2), 4, 8)
    assert st == expect
    assert not h.value
    assert lib.fbsde_last_error()


@pytest.mark.parametrize("net,N,M,expect", [
    (dict(width=0, depth=2), 4, 8, B.ERR_INVALID),
    (dict(width=4, depth=0), 4, 8, B.ERR_INVALID),
    (dict(width=4, depth=2), 0, 8, B.ERR_INVALID),
    (dict(width=4, depth=2), 4, 0, B.ERR_INVALID),
    (dict(width=4, depth=2), 4, 2 ** 31, B.ERR_INVALID),
    (dict(width=300, depth=2), 4, 8, B.ERR_UNSUPPORTED),
    (dict(width=4, depth=9), 4, 8, B.ERR_UNSUPPORTED),
    (dict(kind="u_fc", width=8, depth=2, prec="bf16"), 4, 8, B.ERR_UNSUPPORTED),   # u-network: fp32 only
    (dict(kind="u_res", width=8, depth=17), 4, 8, B.ERR_UNSUPPORTED),              # at most 16 blocks
    (dict(kind="u_nais", width=8, depth=2), 2 ** 20, 2 ** 10, B.ERR_UNSUPPORTED),  # (N + 1) M >= 2^29 rows
    (dict(kind="u_fc", width=8, depth=0), 4, 8, B.ERR_INVALID),
])
def test_invalid_net_and_sizes(lib, net, N, M, expect):
    st, h = _create(lib, BASE, net, N, M)
    assert st == expect
    assert not h.value


def test_null_plan_calls(lib):
    assert lib.fbsde_forward(None, None, None, 0, 0, None, None, None) == B.ERR_INVALID
    assert lib.fbsde_forward_backward(None, None, None, None, None, None, 0, 0, None, None) == B.ERR_INVALID
    n = C.c_int64()
    assert lib.fbsde_param_count(None, C.byref(n)) == B.ERR_INVALID
    assert lib.fbsde_prolong(None, None, None, None, None) == B.ERR_INVALID
    assert lib.fbsde_plan_set_checkpointing(None, 1, 0) == B.ERR_INVALID
    assert lib.fbsde_plan_status(None) == B.ERR_INVALID
    assert lib.fbsde_unet_forward_backward(None, None, None, None, None, 0, 0, None, None) == B.ERR_INVALID
    assert lib.fbsde_unet_nais_project(None, None, 1.0, None, None) == B.ERR_INVALID
    assert lib.fbsde_unet_states(None, None, None, None, None) == B.ERR_INVALID
    assert lib.fbsde_plan_set_unet_loss(None, 0.0, 0.01) == B.ERR_INVALID
    assert lib.fbsde_plan_set_x0(None, None) == B.ERR_INVALID
