"""GPU: activation checkpointing of the per-step MLP.  With recompute on,
the forward pass keeps only one chunk of steps' activations and the reverse
pass recomputes each chunk's from X_n with the same kernels before its
reverse sweep, so loss, dL/dY0 and the gradient must equal those of the plan
that keeps every step's activations bit for bit, for every reverse-kernel
form (fused, separate pair, layer-streamed, global-fragment) and for chunk
counts that do and do not divide N."""
import numpy as np
import pytest
import torch

from paper_1910_11623_amd import inputs as I

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1910_11623_amd.plan import Plan, TrainState

# (problem, d, net, N, M, lds mode, steps per chunk)
CASES = [
    ("bsb", 20, dict(kind="mlp", width=30, depth=2, prec="fp32"), 6, 300, 2, 2),   # fused fp32, 3 chunks
    ("bsb", 20, dict(kind="mlp", width=30, depth=2, prec="fp32"), 6, 300, 2, 4),   # ragged: 4 + 2 steps
    ("hjb", 12, dict(kind="mlp", width=24, depth=2, prec="fp32"), 5, 130, 1, 1),   # separate pair, 1 step
    ("ac", 10, dict(kind="mlp", width=20, depth=2, prec="fp32"), 4, 77, 0, 3),     # weights from global memory
    ("hjb", 7, dict(kind="mlp", width=9, depth=3, prec="fp32"), 4, 33, 2, 2),      # depth 3: the pair
    ("bsb", 24, dict(kind="mlp", width=40, depth=2, prec="bf16"), 5, 200, 2, 2),   # fused bf16
    ("hjb", 150, dict(kind="mlp", width=160, depth=2, prec="bf16"), 4, 90, 2, 3),  # layer-streamed bf16
    ("bsb", 6, dict(kind="mlp", width=8, depth=1, prec="fp32"), 1, 40, 2, 1),      # N = 1: step 0 only
]


def _prob(name, d):
    return {"bsb": I.bsb, "hjb": I.hjb, "ac": I.allen_cahn}[name](d)


@pytest.mark.parametrize("name,d,net,N,M,lds,cs", CASES)
def test_checkpointed_gradient_is_bitwise_equal(name, d, net, N, M, lds, cs):
    prob = _prob(name, d)
    keep = Plan(prob, net, N, M)
    ck = Plan(prob, net, N, M, recompute=True, chunk_rows=cs * M)
    for p in (keep, ck):
        p.config(lds=lds)
    print(f"{name} d={d} N={N} M={M} {net} lds={lds} chunk={cs} steps; workspace {keep.ws_bytes} -> "
          f"{ck.ws_bytes} bytes", flush=True)
    if cs < N:
        assert ck.ws_bytes < keep.ws_bytes
    params = torch.from_numpy(I.init_params(prob, net, N, seed=7, out_scale=0.3).astype(np.float32)).cuda()
    y0 = torch.tensor(10.0 if name == "bsb" else 0.6, dtype=torch.float64, device="cuda")
    for it in (0, 3):
        la, ga, ya = keep.forward_backward(params, y0, 5, it)
        lb, gb, yb = ck.forward_backward(params, y0, 5, it)
        torch.cuda.synchronize()
        assert np.isfinite(la.item())
        assert la.item() == lb.item() and ya.item() == yb.item()
        assert torch.equal(ga, gb)
    # the forward-only loss is unchanged by the chunked forward pass
    assert keep.forward(params, y0, 5, 3).item() == ck.forward(params, y0, 5, 3).item()


def test_checkpointed_training_steps_bitwise():
    """Fused training steps (reduction + Adam) over several iterations."""
    prob = I.bsb(30)
    net = dict(kind="mlp", width=40, depth=2, prec="bf16")
    N, M = 8, 256
    keep = Plan(prob, net, N, M)
    ck = Plan(prob, net, N, M, recompute=True, chunk_rows=3 * M)
    p = I.init_params(prob, net, N, seed=2, out_scale=0.3)
    a, b = TrainState(keep, p, 20.0), TrainState(ck, p, 20.0)
    for k in range(4):
        a.fused_step(11, k, lr=3e-3, lr_y0=0.05)
        b.fused_step(11, k, lr=3e-3, lr_y0=0.05)
    torch.cuda.synchronize()
    for f in ("params", "y0", "grad", "gy0", "loss", "m", "v"):
        assert torch.equal(getattr(a, f), getattr(b, f)), f


def test_checkpointing_after_workspace_query_is_refused_if_larger():
    """Switching back to kept activations needs more workspace than the
    checkpointed plan reported: refused, and the plan keeps working."""
    from paper_1910_11623_amd import binding as B
    prob = I.bsb(10)
    net = dict(kind="mlp", width=20, depth=2, prec="fp32")
    ck = Plan(prob, net, 8, 64, recompute=True, chunk_rows=64)
    with pytest.raises(B.FbsdeError):
        B.check(ck.lib.fbsde_plan_set_checkpointing(ck._h, 0, 0))
    params = torch.from_numpy(I.init_params(prob, net, 8, seed=1).astype(np.float32)).cuda()
    y0 = torch.tensor(5.0, dtype=torch.float64, device="cuda")
    loss, _, _ = ck.forward_backward(params, y0, 1, 0)
    assert np.isfinite(loss.item())


def test_autograd_function_with_checkpointing():
    """The adjoint behind torch.autograd with a checkpointed plan: the same
    gradients as with kept activations."""
    from paper_1910_11623_amd.plan import FBSDELoss
    prob = I.hjb(16)
    net = dict(kind="mlp", width=24, depth=2, prec="fp32")
    N, M = 6, 96
    keep = Plan(prob, net, N, M)
    ck = Plan(prob, net, N, M, recompute=True, chunk_rows=2 * M)
    p0 = torch.from_numpy(I.init_params(prob, net, N, seed=4, out_scale=0.3).astype(np.float32)).cuda()
    grads = []
    for plan in (keep, ck):
        params = p0.clone().requires_grad_(True)
        y = torch.tensor(0.5, dtype=torch.float64, device="cuda", requires_grad=True)
        loss = FBSDELoss.apply(params, y, plan, 2, 1)
        (3.0 * loss).backward()
        grads.append((loss.detach(), params.grad, y.grad))
    assert torch.equal(grads[0][0], grads[1][0])
    assert torch.equal(grads[0][1], grads[1][1])
    assert torch.equal(grads[0][2], grads[1][2])


def test_checkpointed_plans_in_a_batch_graph():
    """Checkpointed instances captured in one hipGraph (their chunk loops
    included): every replay gives the bits of kept-activation eager steps."""
    from paper_1910_11623_amd.plan import Batch
    shapes = [(20, 10), (57, 6)]
    M = 300
    eager, graph, seeds = [], [], []
    for k, (d, N) in enumerate(shapes):
        prob = I.allen_cahn(d)
        net = dict(kind="mlp", width=d + 10, depth=2, prec="bf16")
        p = I.init_params(prob, net, N, seed=k, out_scale=0.05)
        eager.append(TrainState(Plan(prob, net, N, M), p, 0.3))
        graph.append(TrainState(Plan(prob, net, N, M, recompute=True, chunk_rows=4 * M), p, 0.3))
        seeds.append(21 + k)
    batch = Batch(graph, seeds)
    for k in range(3):
        for s, seed in zip(eager, seeds):
            s.eager_step(seed, k)
        junk = torch.randn(1 << 16, device="cuda").sum()  # unrelated eager work between replays
        batch.step()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for a, b in zip(eager, graph):
            assert torch.equal(a.params, b.params), k
            assert torch.equal(a.y0, b.y0), k
            assert torch.equal(a.loss, b.loss), k
