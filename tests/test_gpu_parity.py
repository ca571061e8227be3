"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances:
  fp32 path  loss |L - L*| <= 1e-5 |L*|, gradient per parameter block
             <= 1e-4 normwise and elementwise (max |g - g*| / max |g*|),
             dL/dY0 <= 1e-4 relative
  bf16 path  against the oracle's bf16-emulation mode: loss <= 1e-3,
             gradient <= 1e-2 per block (normwise and elementwise); against
             pure fp64: loss <= 2e-2
  normals    fp32 Box–Muller vs fp64: |dxi| <= 4e-6 (1 + |xi|)
"""
import math

import numpy as np
import pytest
import torch

from oracle import core as O
from oracle import refvalues as RV
from paper_1910_11623_amd import inputs as I

from gpu_common import check_grad, inputs, oracle_net, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1910_11623_amd.plan import Plan


def _problem(name, d):
    if name == "bsb":
        return I.bsb(d)
    if name == "hjb":
        return I.hjb(d)
    return I.allen_cahn(d)


def test_library_is_the_hip_build():
    import paper_1910_11623_amd.binding as B
    lib = B.load()
    assert lib._name.endswith("libfbsde.so")


def test_normals_match_oracle():
    prob = I.bsb(10)
    plan = Plan(prob, dict(width=4, depth=1), 3, 1000)
    xi = plan.sample_normals(seed=12345, it=7).cpu().numpy().astype(np.float64)
    ref = O.normals(12345, 7, 3, 1000, 10)
    err = np.abs(xi - ref) / (1 + np.abs(ref))
    assert err.max() <= 4e-6, err.max()


# (problem, d, width, depth, N, M) — config 0 exactly, plus ragged / degenerate shapes
FP32_CASES = [
    ("bsb", 10, 20, 2, 16, 256),   # BSB d=10 configuration at full size
    ("bsb", 10, 20, 2, 16, 77),    # ragged M
    ("hjb", 12, 24, 2, 5, 130),
    ("ac", 20, 30, 2, 10, 64),
    ("bsb", 1, 3, 1, 3, 5),        # d = 1, one hidden layer
    ("hjb", 7, 9, 3, 4, 33),       # three hidden layers
    ("bsb", 6, 8, 2, 1, 40),       # N = 1: only y0 and z0
    ("bsb", 100, 110, 2, 8, 96),   # d=100, w=110 shape at reduced N, M
    ("hjb", 100, 110, 2, 20, 48),  # HJB d=100 shape at reduced M
    ("hjb", 120, 125, 2, 3, 45),   # 8 x 8 fp32 tiles (reverse sweep loads each layer before its product)
    ("hjb", 3, 5, 2, 3, 100003),   # 1563 one-wave scan workgroups (ragged), 64 gradient splits
    ("ac", 130, 140, 2, 3, 40),    # d, w above 128: 16-tile kernels
    ("hjb", 256, 256, 2, 3, 21),   # largest per-step shape: d = w = 256 (16 x 16 tiles, no padding)
    ("bsb", 5, 8, 2, 40, 50),      # 33 <= N <= 64: the scan's 64-step register form
    ("hjb", 8, 12, 1, 70, 64),     # N > 64: the scan streams c_n and Y_n (HJB: the Y recursion is
    ("hjb", 8, 12, 1, 130, 40),    # stable; Allen-Cahn's y^3 drift amplifies fp32 rounding at long grids)
]


@pytest.mark.parametrize("pname,d,w,L,N,M", FP32_CASES)
def test_fp32_loss_and_gradient(pname, d, w, L, N, M):
    prob = _problem(pname, d)
    net = dict(kind="mlp", width=w, depth=L, prec="fp32")
    p32, p64, y0 = inputs(prob, net, N, seed=3, y0=RV.bsb_y0(d) * 0.95 if pname == "bsb" else 0.5)
    plan = Plan(prob, net, N, M)
    lg, gg, gy = run_gpu(plan, p32, y0, seed=11, it=2)
    ref = run_oracle(prob, net, N, M, p64, y0, seed=11, it=2)
    assert abs(lg - ref["loss"]) <= 1e-5 * abs(ref["loss"]), (lg, ref["loss"])
    assert abs(gy - ref["grad_y0"]) <= 1e-4 * abs(ref["grad_y0"]) + 1e-12
    check_grad(prob, net, N, gg, ref["grad"], 1e-4)


@pytest.mark.parametrize("pname,d,w,N,M", [("hjb", 100, 110, 6, 64), ("bsb", 10, 20, 16, 256),
                                            ("ac", 20, 30, 10, 70),
                                            ("hjb", 80, 90, 5, 100),    # 6 x 6 bf16 tiles
                                            ("hjb", 140, 150, 4, 50),   # 10 x 10 bf16 tiles
                                            ("hjb", 150, 160, 5, 90),   # 12 x 12 bf16 tiles
                                            ("hjb", 200, 210, 4, 40),   # 14 x 14 bf16 tiles
                                            ("hjb", 230, 240, 3, 33),   # 16 x 16 bf16 tiles
                                            ("hjb", 256, 256, 3, 21)])  # largest per-step shape
def test_bf16_loss_and_gradient(pname, d, w, N, M):
    prob = _problem(pname, d)
    net = dict(kind="mlp", width=w, depth=2, prec="bf16")
    p32, p64, y0 = inputs(prob, net, N, seed=5, y0=RV.bsb_y0(d) * 0.95 if pname == "bsb" else 0.5)
    plan = Plan(prob, net, N, M)
    lg, gg, gy = run_gpu(plan, p32, y0, seed=4, it=1)
    emu = run_oracle(prob, net, N, M, p64, y0, seed=4, it=1)
    pure = run_oracle(prob, dict(net, prec="fp32"), N, M, p64, y0, seed=4, it=1)
    assert abs(lg - emu["loss"]) <= 1e-3 * abs(emu["loss"]), (lg, emu["loss"])
    assert abs(lg - pure["loss"]) <= 2e-2 * abs(pure["loss"]), (lg, pure["loss"])
    assert abs(gy - emu["grad_y0"]) <= 1e-3 * abs(emu["grad_y0"]) + 1e-12
    check_grad(prob, net, N, gg, emu["grad"], 1e-2)


def test_forward_only_matches_forward_backward_loss():
    prob = I.hjb(16)
    net = dict(width=20, depth=2)
    p32, _, y0 = inputs(prob, net, 6)
    plan = Plan(prob, net, 6, 100)
    a, _, _ = run_gpu(plan, p32, y0, 1, 1, grad=False)
    b, _, _ = run_gpu(plan, p32, y0, 1, 1, grad=True)
    assert a == b


def test_deterministic_bitwise():
    prob = I.bsb(100)
    net = dict(width=110, depth=2)
    p32, _, y0 = inputs(prob, net, 4)
    plan = Plan(prob, net, 4, 1000)
    l1, g1, y1 = run_gpu(plan, p32, y0, 9, 3)
    l2, g2, y2 = run_gpu(plan, p32, y0, 9, 3)
    assert l1 == l2 and y1 == y2 and np.array_equal(g1, g2)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_full_size_sampled_paths(prec):
    """d=100, w=110, N=32, M=4096 (the BSB throughput configuration) and HJB
    d=100, N=20, M=65536: terminal X_N and Y_N of sampled paths against the
    oracle run on those paths alone."""
    if prec == "fp32":
        prob, N, M = I.bsb(100), 32, 4096
    else:
        prob, N, M = I.hjb(100), 20, 65536
    net = dict(width=110, depth=2, prec=prec)
    p32, p64, y0 = inputs(prob, net, N, seed=1, y0=75.0 if prec == "fp32" else 4.5)
    plan = Plan(prob, net, N, M)
    params = torch.from_numpy(p32).cuda()
    plan.forward(params, torch.tensor(y0, dtype=torch.float64, device="cuda"), 1, 0)
    xN, yN = plan.terminal_states()
    xN, yN = xN.cpu().numpy(), yN.cpu().numpy()
    idx = np.array([0, 1, 15, 16, 63, 64, 1000, M // 2 + 7, M - 2, M - 1])
    yr, xr = O.paths(prob, oracle_net(net), N, p64, y0, idx, seed=1, it=0)
    np.testing.assert_allclose(xN[idx], xr, rtol=2e-5, atol=2e-5)
    tol = 2e-5 if prec == "fp32" else 1e-2
    np.testing.assert_allclose(yN[idx], yr, rtol=tol, atol=tol)
    assert np.isfinite(yN).all()


def test_terminal_mean_matches_oracle():
    prob = I.bsb(10)
    plan = Plan(prob, dict(width=4, depth=1), 16, 300)
    got = float(plan.terminal_mean(5, 0).item())
    p = I.init_params(prob, dict(width=4, depth=1), 16)
    o = O.loss_grad(prob, dict(kind="mlp", width=4, depth=1), 16, 300, p, 0.0, seed=5, it=0,
                    want_grad=False, want_paths=True)
    ref = float((o["XN"] ** 2).sum(1).mean())
    assert got == pytest.approx(ref, rel=1e-5)


def test_adam_matches_oracle():
    prob = I.bsb(10)
    net = dict(width=20, depth=2)
    plan = Plan(prob, net, 4, 8)
    n = plan.n_params
    rng = np.random.default_rng(0)
    th = rng.standard_normal(n).astype(np.float32)
    m = np.zeros(n); v = np.zeros(n)
    th64 = th.astype(np.float64)
    pt = torch.from_numpy(th).cuda(); mt = torch.zeros(n, device="cuda"); vt = torch.zeros(n, device="cuda")
    y = torch.tensor(2.0, dtype=torch.float64, device="cuda")
    my = torch.zeros((), dtype=torch.float64, device="cuda"); vy = torch.zeros_like(my)
    y64 = np.array([2.0]); my64 = np.zeros(1); vy64 = np.zeros(1)
    for t in range(1, 6):
        g = rng.standard_normal(n).astype(np.float32)
        gy = float(rng.standard_normal())
        plan.adam_step(pt, y, torch.from_numpy(g).cuda(), torch.tensor(gy, dtype=torch.float64, device="cuda"),
                       mt, vt, my, vy, t, lr=1e-3, lr_y0=1e-2)
        O.adam(th64, g.astype(np.float64), m, v, t, lr=1e-3)
        O.adam(y64, np.array([gy]), my64, vy64, t, lr=1e-2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(pt.cpu().numpy(), th64, rtol=1e-6, atol=1e-6)
    assert float(y.item()) == pytest.approx(y64[0], rel=1e-14)


def test_prolongation_bitwise():
    prob = I.bsb(10)
    net = dict(width=20, depth=2)
    pc_plan, pf_plan = Plan(prob, net, 4, 8), Plan(prob, net, 8, 8)
    pc = I.init_params(prob, net, 4, seed=2).astype(np.float32)
    pf = pc_plan.prolong_to(pf_plan, torch.from_numpy(pc).cuda()).cpu().numpy()
    ref = O.prolong(prob, oracle_net(net), 4, 8, pc.astype(np.float64))
    assert np.array_equal(pf.astype(np.float64), ref)


def test_autograd_function():
    from paper_1910_11623_amd.plan import FBSDELoss
    prob = I.hjb(8)
    net = dict(width=12, depth=2)
    p32, _, y0 = inputs(prob, net, 4)
    plan = Plan(prob, net, 4, 50)
    params = torch.from_numpy(p32).cuda().requires_grad_(True)
    y = torch.tensor(y0, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = FBSDELoss.apply(params, y, plan, 3, 0)
    (2.0 * loss).backward()
    _, g, gy = plan.forward_backward(params.detach(), y.detach(), 3, 0)
    torch.testing.assert_close(params.grad, 2 * g)
    torch.testing.assert_close(y.grad, 2 * gy)


def test_invalid_arguments_raise():
    import paper_1910_11623_amd.binding as B
    with pytest.raises(B.FbsdeError):
        Plan(I.bsb(300), dict(width=20), 4, 8)   # d above the fused-kernel limit
    plan = Plan(I.bsb(4), dict(width=8), 4, 8)
    with pytest.raises(ValueError):
        plan.forward(torch.zeros(3, device="cuda"), torch.zeros((), dtype=torch.float64, device="cuda"), 0, 0)


@pytest.mark.parametrize("kind", ["mlp", "resnet"])
def test_nonfinite_result_reported_by_next_call(kind):
    """A NaN weight makes the loss and gradient non-finite: the call that
    computes them returns normally (nothing synchronises), the next hot call
    on the plan reports FBSDE_ERR_NONFINITE once, and the one after that
    runs again."""
    import paper_1910_11623_amd.binding as B
    prob = I.bsb(6)
    net = dict(width=16, depth=2) if kind == "mlp" else dict(kind="resnet", width=16, depth=2, prec="bf16")
    plan = Plan(prob, net, 4, 64)
    p = I.init_params(prob, net, 4, seed=0).astype(np.float32)
    y0 = torch.tensor(1.0, dtype=torch.float64, device="cuda")
    good = torch.from_numpy(p).cuda()
    bad = good.clone()
    bad[7] = float("nan")
    plan.forward_backward(good, y0, 1, 0)
    torch.cuda.synchronize()
    plan.forward_backward(good, y0, 1, 1)     # finite: no report
    plan.forward_backward(bad, y0, 1, 2)
    torch.cuda.synchronize()
    with pytest.raises(B.FbsdeError) as ei:
        plan.forward_backward(good, y0, 1, 3)
    assert ei.value.status == B.ERR_NONFINITE
    loss, g, gy = plan.forward_backward(good, y0, 1, 4)
    torch.cuda.synchronize()
    assert np.isfinite(float(loss.item())) and bool(torch.isfinite(g).all().item())
    plan.forward_backward(good, y0, 1, 5)     # still no report
    torch.cuda.synchronize()
    assert plan.finite_since_last_check()
    plan.forward_backward(bad, y0, 1, 6)
    torch.cuda.synchronize()
    assert not plan.finite_since_last_check()  # the status call reports and clears
    assert plan.finite_since_last_check()
