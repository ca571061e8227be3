"""GPU parity of the shared time-conditioned residual network (bf16 MFMA
GEMMs, chunked recompute) against the FP64 oracle's bf16 emulation."""
import numpy as np
import pytest
import torch

from oracle import core as O
from paper_1910_11623_amd import inputs as I

from gpu_common import check_grad, oracle_net, run_gpu

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1910_11623_amd.plan import Plan


def _problem(name, d):
    return {"bsb": I.bsb, "hjb": I.hjb, "ac": I.allen_cahn}[name](d)


# (problem, d, width, blocks, N, M); with 65536-row chunks, M = 20000 makes
# chunks of 3 steps (5 = 3 + 2)
CHUNK = 65536
CASES = [
    ("bsb", 20, 32, 2, 4, 64),
    ("hjb", 37, 40, 1, 3, 130),
    ("ac", 8, 16, 2, 5, 20000),
    ("bsb", 100, 128, 4, 6, 256),
    ("bsb", 1100, 64, 1, 3, 48),  # d > 1024: each SDE thread strides over several 4-dim groups
]


@pytest.mark.parametrize("pname,d,w,B,N,M", CASES)
def test_resnet_loss_and_gradient(pname, d, w, B, N, M):
    prob = _problem(pname, d)
    net = dict(kind="resnet", width=w, depth=B, prec="bf16")
    p = I.init_params(prob, net, N, seed=7, out_scale=0.3).astype(np.float32)
    y0 = 0.9 * float(np.dot(prob["x0"], prob["x0"])) if pname == "bsb" else 0.4
    plan = Plan(prob, net, N, M, chunk_rows=CHUNK)
    lg, gg, gy = run_gpu(plan, p, y0, seed=5, it=1)
    emu = O.loss_grad(prob, oracle_net(net), N, M, p.astype(np.float64), y0, seed=5, it=1)
    pure = O.loss_grad(prob, dict(oracle_net(net), bf16=False), N, M, p.astype(np.float64), y0, seed=5, it=1)
    assert abs(lg - emu["loss"]) <= 1e-3 * abs(emu["loss"]), (lg, emu["loss"])
    assert abs(lg - pure["loss"]) <= 2e-2 * abs(pure["loss"]), (lg, pure["loss"])
    assert abs(gy - emu["grad_y0"]) <= 1e-3 * abs(emu["grad_y0"]) + 1e-12
    check_grad(prob, net, N, gg, emu["grad"], 1e-2)


def test_resnet_prolongation_is_identity_and_deterministic():
    prob = I.hjb(16)
    net = dict(kind="resnet", width=32, depth=2, prec="bf16")
    a, b = Plan(prob, net, 4, 64), Plan(prob, net, 8, 64)
    p = I.init_params(prob, net, 4, seed=1).astype(np.float32)
    q = a.prolong_to(b, torch.from_numpy(p).cuda()).cpu().numpy()
    assert np.array_equal(p, q)
    r1 = run_gpu(b, q, 0.5, 2, 3)
    r2 = run_gpu(b, q, 0.5, 2, 3)
    assert r1[0] == r2[0] and np.array_equal(r1[1], r2[1])


def test_resnet_full_size_sampled_paths():
    """BSB d=1000, width 1024, 4 residual blocks, N=64, M=16384: terminal
    X_N and Y_N of sampled paths against the oracle on those paths alone."""
    prob = I.bsb(1000)
    net = dict(kind="resnet", width=1024, depth=4, prec="bf16")
    N, M = 64, 16384
    p = I.init_params(prob, net, N, seed=0, out_scale=0.1).astype(np.float32)
    y0 = 760.0
    plan = Plan(prob, net, N, M)
    loss = plan.forward(torch.from_numpy(p).cuda(), torch.tensor(y0, dtype=torch.float64, device="cuda"), 1, 0)
    xN, yN = plan.terminal_states()
    xN, yN = xN.cpu().numpy(), yN.cpu().numpy()
    assert np.isfinite(float(loss.item())) and np.isfinite(yN).all()
    idx = np.array([0, 5000, M - 1])
    yr, xr = O.paths(prob, oracle_net(net), N, p.astype(np.float64), y0, idx, seed=1, it=0)
    np.testing.assert_allclose(xN[idx], xr, rtol=2e-5, atol=2e-5)
    np.testing.assert_allclose(yN[idx], yr, rtol=2e-3, atol=2e-3)


# several row chunks each (3 + 2 and 4 + 3 steps)
@pytest.mark.parametrize("pname,d,w,B,N,M", [CASES[2], ("bsb", 50, 64, 2, 7, 16384)])
def test_resnet_kept_activations_match_recompute_bitwise(pname, d, w, B, N, M):
    """Keeping every chunk's activations from the forward pass (no recompute
    in the reverse sweep) gives bitwise the same loss and gradient."""
    prob = _problem(pname, d)
    net = dict(kind="resnet", width=w, depth=B, prec="bf16")
    p = I.init_params(prob, net, N, seed=3, out_scale=0.3).astype(np.float32)
    a = Plan(prob, net, N, M, recompute=True, chunk_rows=CHUNK)
    b = Plan(prob, net, N, M, recompute=False, chunk_rows=CHUNK)
    assert b.ws_bytes > a.ws_bytes
    ra = run_gpu(a, p, 0.4, seed=9, it=2)
    rb = run_gpu(b, p, 0.4, seed=9, it=2)
    assert ra[0] == rb[0] and ra[2] == rb[2]
    assert np.array_equal(ra[1], rb[1])


def test_resnet_chunk_size_changes_only_gradient_summation_order():
    """Chunks of 3 + 2 steps vs one chunk of 5: the same loss bitwise (rows
    are independent in the forward pass); gradients equal up to the fp32
    order of the sums over chunks."""
    prob = _problem("ac", 8)
    net = dict(kind="resnet", width=16, depth=2, prec="bf16")
    N, M = 5, 20000
    p = I.init_params(prob, net, N, seed=4, out_scale=0.3).astype(np.float32)
    a = Plan(prob, net, N, M, chunk_rows=CHUNK)
    b = Plan(prob, net, N, M)
    ra = run_gpu(a, p, 0.4, seed=9, it=2)
    rb = run_gpu(b, p, 0.4, seed=9, it=2)
    assert ra[0] == rb[0]
    np.testing.assert_allclose(ra[1], rb[1], rtol=1e-5, atol=1e-7 * np.abs(rb[1]).max())
    assert abs(ra[2] - rb[2]) <= 1e-12 * max(1.0, abs(rb[2]))


def test_checkpointing_cannot_outgrow_a_reported_workspace():
    import ctypes as C
    import paper_1910_11623_amd.binding as B
    prob = _problem("bsb", 20)
    net = dict(kind="resnet", width=32, depth=2, prec="bf16")
    plan = Plan(prob, net, 8, 4096, chunk_rows=8192)  # checkpointed, workspace already sized
    assert plan.lib.fbsde_plan_set_checkpointing(plan._h, 0, 8192) == B.ERR_INVALID
    assert plan.lib.fbsde_plan_set_checkpointing(plan._h, 1, 8192) == B.OK  # same size: allowed
