"""GPU: the fused reverse kernel (reverse sweep and weight gradient of a step
in one kernel, fp32 per-step MLP) against the separate backward and
weight-gradient kernels, which the oracle parity tests pin.  The two forms
walk the same path splits and 16-path chunks with the same MFMA slot
assignment, so loss, dL/dY0 and every gradient entry must agree bitwise."""
import numpy as np
import pytest
import torch

from paper_1910_11623_amd import inputs as I

from gpu_common import check_grad, inputs, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1910_11623_amd.plan import Plan


def _run(plan, p32, y0, seed=5, it=2):
    plan.profile(True)
    out = run_gpu(plan, p32, y0, seed, it)
    prof = plan.profile_read()
    plan.profile(False)
    return out, prof["wgrad"][1]


# (problem, d, width, depth, N, M, precision): every instantiated tile shape
# (fp32 (1, 2), (2, 2), (4, 4), (7, 7); bf16 (2, 2), (4, 4), (6, 6), (8, 8)) at
# depth 1 and 2, the bias column in the last tile column, ragged path counts
# (partial last chunk, uneven splits)
CASES = [
    ("ac", 10, 20, 2, 5, 70, "fp32"),
    ("bsb", 12, 30, 1, 4, 33, "fp32"),
    ("bsb", 20, 24, 2, 6, 200, "fp32"),
    ("hjb", 31, 31, 1, 3, 517, "fp32"),
    ("hjb", 40, 50, 2, 6, 1100, "fp32"),
    ("bsb", 63, 63, 1, 4, 300, "fp32"),
    ("bsb", 100, 110, 2, 4, 1000, "fp32"),
    ("ac", 111, 111, 1, 3, 1030, "fp32"),
    ("ac", 10, 20, 2, 5, 70, "bf16"),
    ("bsb", 31, 17, 1, 4, 45, "bf16"),
    ("hjb", 40, 50, 2, 6, 1100, "bf16"),
    ("bsb", 63, 60, 1, 3, 300, "bf16"),
    ("hjb", 90, 95, 2, 4, 513, "bf16"),
    ("ac", 95, 80, 1, 3, 200, "bf16"),
    ("bsb", 100, 110, 2, 4, 1000, "bf16"),
    ("hjb", 127, 127, 1, 3, 777, "bf16"),
]


def _problem(name, d):
    return {"bsb": I.bsb, "hjb": I.hjb, "ac": I.allen_cahn}[name](d)


@pytest.mark.parametrize("name,d,w,L,N,M,prec", CASES)
def test_fused_reverse_matches_split_kernels_bitwise(name, d, w, L, N, M, prec):
    prob = _problem(name, d)
    net = dict(width=w, depth=L, prec=prec)
    p32, _, y0 = inputs(prob, net, N, seed=3, y0=1.5)
    plan = Plan(prob, net, N, M)
    print(f"{name} d={d} w={w} L={L} N={N} M={M} {prec} config {plan.get_config()}", flush=True)
    fused, nw = _run(plan, p32, y0)
    assert nw == 0, "the default configuration should take the fused reverse kernel"
    plan.config(lds=1)
    split, nw1 = _run(plan, p32, y0)
    assert nw1 > 0
    assert fused[0] == split[0] and fused[2] == split[2]
    assert np.array_equal(fused[1], split[1])
    assert np.all(np.isfinite(fused[1]))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("splits", [1, 3, 32])
def test_fused_reverse_split_counts(splits, prec):
    """Every split count the tuner may pick: same partial-buffer layout as the
    weight-gradient kernel, so the reduction sees identical partials."""
    prob = I.bsb(100)
    net = dict(width=110, depth=2, prec=prec)
    p32, _, y0 = inputs(prob, net, 3, seed=1, y0=70.0)
    plan = Plan(prob, net, 3, 4096)
    plan.config(lds=2, splits=splits)
    fused, nw = _run(plan, p32, y0)
    assert nw == 0
    plan.config(lds=1, splits=splits)
    split, _ = _run(plan, p32, y0)
    assert fused[0] == split[0] and fused[2] == split[2]
    assert np.array_equal(fused[1], split[1])


def test_fused_reverse_against_oracle():
    """Direct oracle parity of the fused path (loss, dL/dY0, every block
    normwise and elementwise) at a ragged size."""
    prob = I.hjb(24)
    net = dict(width=40, depth=2, prec="fp32")
    N, M = 5, 150
    p32, p64, y0 = inputs(prob, net, N, seed=7, y0=0.8)
    plan = Plan(prob, net, N, M)
    (lg, gg, gy), nw = _run(plan, p32, y0, seed=11, it=2)
    assert nw == 0
    ref = run_oracle(prob, net, N, M, p64, y0, seed=11, it=2)
    assert abs(lg - ref["loss"]) <= 1e-5 * abs(ref["loss"]), (lg, ref["loss"])
    assert abs(gy - ref["grad_y0"]) <= 1e-4 * abs(ref["grad_y0"]) + 1e-12
    check_grad(prob, net, N, gg, ref["grad"], 1e-4)


@pytest.mark.parametrize("L,prec,d,w", [(3, "fp32", 20, 30), (3, "bf16", 20, 30), (2, "fp32", 112, 60),
                                        (2, "bf16", 128, 30), (2, "bf16", 140, 150)])
def test_configurations_outside_the_fused_kernel_use_the_split_pair(L, prec, d, w):
    """Depth 3, a bias column past the tiles (d = 112 on 7 fp32 tiles, d = 128
    on 8 bf16 tiles) and shapes beyond 8 tiles keep the separate kernels even
    in LDS mode 2."""
    prob = I.bsb(d)
    net = dict(width=w, depth=L, prec=prec)
    p32, _, y0 = inputs(prob, net, 3, seed=2)
    plan = Plan(prob, net, 3, 64)
    (_, g, _), nw = _run(plan, p32, y0)
    assert nw > 0
    assert np.all(np.isfinite(g))
