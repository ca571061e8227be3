"""GPU: fbsde_train_step (forward, reverse sweep, gradient reduction fused
with the Adam update) against fbsde_forward_backward followed by
fbsde_adam_step.  Both run the same Adam arithmetic on the same reduced
gradient, so every output must agree bitwise after every step."""
import numpy as np
import pytest
import torch

from paper_1910_11623_amd import binding as B
from paper_1910_11623_amd import inputs as I

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1910_11623_amd.plan import Plan, TrainState, UPlan

FIELDS = ("params", "y0", "grad", "gy0", "loss", "m", "v", "my0", "vy0")


def _same(a, b):
    for f in FIELDS:
        x, y = getattr(a, f).cpu().numpy(), getattr(b, f).cpu().numpy()
        assert np.array_equal(x, y), f
    assert np.all(np.isfinite(a.params.cpu().numpy()))


# per-step MLP fp32 and bf16 (fused and split reverse kernels, ragged sizes),
# a parameter count that is not a multiple of 4 (scalar tail), and the
# shared residual net
CASES = [
    ("bsb", dict(kind="mlp", width=30, depth=2, prec="fp32"), 20, 6, 300),
    ("hjb", dict(kind="mlp", width=17, depth=1, prec="fp32"), 7, 5, 77),
    ("ac", dict(kind="mlp", width=40, depth=2, prec="bf16"), 24, 4, 200),
    ("bsb", dict(kind="resnet", width=32, depth=2, prec="bf16"), 20, 4, 64),
]


@pytest.mark.parametrize("name,net,d,N,M", CASES)
def test_train_step_matches_separate_calls_bitwise(name, net, d, N, M):
    prob = {"bsb": I.bsb, "hjb": I.hjb, "ac": I.allen_cahn}[name](d)
    plan = Plan(prob, net, N, M)
    p = I.init_params(prob, net, N, seed=4, out_scale=0.3)
    print(f"{name} d={d} N={N} M={M} {net} n_params={plan.n_params}", flush=True)
    a, b = TrainState(plan, p, 0.7), TrainState(plan, p, 0.7)
    for k in range(4):
        a.eager_step(9, k, lr=3e-3, lr_y0=0.05)
        b.fused_step(9, k, lr=3e-3, lr_y0=0.05)
        torch.cuda.synchronize()
        _same(a, b)


def test_train_step_split_reverse_pair():
    """LDS mode 1 (separate reverse sweep and weight-gradient kernels)."""
    prob = I.bsb(30)
    net = dict(kind="mlp", width=40, depth=2, prec="fp32")
    plan = Plan(prob, net, 5, 500)
    plan.config(lds=1)
    p = I.init_params(prob, net, 5, seed=2)
    a, b = TrainState(plan, p, 10.0), TrainState(plan, p, 10.0)
    for k in range(3):
        a.eager_step(3, k)
        b.fused_step(3, k)
    torch.cuda.synchronize()
    _same(a, b)


def test_train_step_rejects_u_network_and_bad_arguments():
    prob = I.bsb(4)
    up = UPlan(prob, dict(kind="u_fc", width=16, depth=1), 2, 8)
    z = torch.zeros(up.n_params, dtype=torch.float32, device="cuda")
    s = torch.zeros((), dtype=torch.float64, device="cuda")
    lib = B.load()
    with pytest.raises(B.FbsdeError):
        up_ptr = up._h.value
        B.check(lib.fbsde_train_step(up_ptr, z.data_ptr(), s.data_ptr(), z.data_ptr(), s.data_ptr(), s.data_ptr(),
                                     z.data_ptr(), z.data_ptr(), s.data_ptr(), s.data_ptr(), 1, 1e-3, 1e-3, 0.9,
                                     0.999, 1e-8, 1, 0, up.ws.data_ptr(), None))
    plan = Plan(prob, dict(kind="mlp", width=8, depth=1, prec="fp32"), 3, 16)
    st = TrainState(plan, I.init_params(prob, dict(kind="mlp", width=8, depth=1, prec="fp32"), 3, seed=0), 1.0)
    with pytest.raises(B.FbsdeError):
        plan.train_step(st.params, st.y0, st.grad, st.gy0, st.loss, st.m, st.v, st.my0, st.vy0, 1, 0, 0)
