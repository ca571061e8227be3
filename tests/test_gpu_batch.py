"""GPU: tuning configurations, the autotuner, and graph-captured batches of
uneven instances against eager execution and against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import core as O
from paper_1910_11623_amd import inputs as I

from gpu_common import blockwise_rel, check_grad, inputs, oracle_net, run_gpu

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1910_11623_amd.plan import Batch, Plan, TrainState


def _fb(plan, p32, y0, seed=3, it=1):
    loss, g, gy = run_gpu(plan, p32, y0, seed, it)
    return loss, g, gy


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_tile_shapes_lds_and_tpw_are_bitwise_identical(prec):
    prob = I.bsb(100)
    net = dict(width=110, depth=2, prec=prec)
    p32, _, y0 = inputs(prob, net, 4, seed=2, y0=75.0)
    plan = Plan(prob, net, 4, 1000)
    ref = _fb(plan, p32, y0)
    ncand = 2
    for shape in range(ncand):
        for lds in (2, 1, 0):  # fused reverse kernel (where it applies), split kernels, global weights
            for tpw in (0, 1, 3):
                try:
                    plan.config(shape=shape, lds=lds, tpw=tpw, splits=0)
                except Exception:
                    continue  # shape not available for this problem
                got = _fb(plan, p32, y0)
                assert got[0] == ref[0] and got[2] == ref[2], (shape, lds, tpw)
                assert np.array_equal(got[1], ref[1]), (shape, lds, tpw)


def test_split_count_changes_only_summation_order():
    prob = I.hjb(40)
    net = dict(width=50, depth=2, prec="fp32")
    p32, _, y0 = inputs(prob, net, 6, seed=4)
    plan = Plan(prob, net, 6, 2048)
    plan.config(splits=4)
    a = _fb(plan, p32, y0)
    plan.config(splits=32)
    b = _fb(plan, p32, y0)
    assert a[0] == b[0] and a[2] == b[2]
    assert np.linalg.norm(a[1] - b[1]) <= 1e-6 * np.linalg.norm(a[1])


def test_autotune_keeps_parity():
    prob = I.allen_cahn(60)
    net = dict(width=70, depth=2, prec="bf16")
    N, M = 5, 512
    p32, p64, y0 = inputs(prob, net, N, seed=6)
    plan = Plan(prob, net, N, M)
    cfg = plan.autotune(torch.from_numpy(p32).cuda(), torch.tensor(y0, dtype=torch.float64, device="cuda"))
    assert cfg["splits"] >= 1 and cfg["tpw"] >= 1
    lg, gg, gy = _fb(plan, p32, y0, seed=2, it=0)
    ref = O.loss_grad(prob, oracle_net(net), N, M, p64, y0, seed=2, it=0)
    assert abs(lg - ref["loss"]) <= 1e-3 * abs(ref["loss"])
    assert max(blockwise_rel(prob, net, N, gg, ref["grad"]).values()) <= 1e-2


def _ac_states(shapes, M, prec, seed0=0):
    out = []
    for k, (d, N) in enumerate(shapes):
        prob = I.allen_cahn(d)
        net = dict(width=d + 10, depth=2, prec=prec)
        plan = Plan(prob, net, N, M)
        p = I.init_params(prob, net, N, seed=seed0 + k, out_scale=0.05).astype(np.float32)
        out.append((prob, net, N, p, plan))
    return out


def test_batch_graph_replays_match_eager_steps():
    shapes = [(20, 10), (57, 20), (130, 5)]
    M, prec, K = 300, "bf16", 4
    insts = _ac_states(shapes, M, prec)
    seeds = [11 + k for k in range(len(insts))]
    eager = [TrainState(plan, p, 0.3) for (_, _, _, p, plan) in insts]
    # graph side: separate plans (separate workspaces) with the same inputs
    insts2 = _ac_states(shapes, M, prec)
    graph = [TrainState(plan, p, 0.3) for (_, _, _, p, plan) in insts2]
    batch = Batch(graph, seeds)
    for k in range(K):
        for s, seed in zip(eager, seeds):
            s.eager_step(seed, k)
        # unrelated eager work between replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        batch.step()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for a, b in zip(eager, graph):
            assert torch.equal(a.params, b.params), k
            assert torch.equal(a.y0, b.y0), k
            assert torch.equal(a.loss, b.loss), k
    assert int(batch.iter.item()) == K


def test_batch_first_step_matches_oracle():
    """Allen–Cahn instances of uneven d and N in one graph: the loss and
    gradient of the first step against the FP64 oracle (bf16 emulation)."""
    shapes = [(23, 10), (96, 20), (171, 40)]
    M, prec = 40, "bf16"
    insts = _ac_states(shapes, M, prec, seed0=5)
    seeds = [3 + k for k in range(len(insts))]
    states = [TrainState(plan, p, 0.2) for (_, _, _, p, plan) in insts]
    batch = Batch(states, seeds)
    batch.step()
    torch.cuda.synchronize()
    for (prob, net, N, p, plan), s, seed in zip(insts, states, seeds):
        ref = O.loss_grad(prob, oracle_net(net), N, M, p.astype(np.float64), 0.2, seed=seed, it=0)
        assert abs(float(s.loss.item()) - ref["loss"]) <= 1e-3 * abs(ref["loss"])
        g = s.grad.cpu().numpy().astype(np.float64)
        check_grad(prob, net, N, g, ref["grad"], 1e-2)


def test_batch_step_reports_a_nonfinite_instance():
    """A NaN weight in one instance: the graph step that computes it runs,
    the next batch step returns FBSDE_ERR_NONFINITE without launching, and
    the step after that runs again."""
    import paper_1910_11623_amd.binding as B
    shapes = [(20, 10), (33, 5)]
    insts = _ac_states(shapes, 64, "bf16")
    states = [TrainState(plan, p, 0.3) for (_, _, _, p, plan) in insts]
    batch = Batch(states, [1, 2])
    batch.step()
    torch.cuda.synchronize()
    states[1].params[5] = float("nan")
    batch.step()
    torch.cuda.synchronize()
    with pytest.raises(B.FbsdeError) as ei:
        batch.step()
    assert ei.value.status == B.ERR_NONFINITE
    assert int(batch.iter.item()) == 2   # the refused step launched nothing
    states[1].params.copy_(torch.from_numpy(insts[1][3]).to(states[1].params.device))
    for t in (states[1].m, states[1].v, states[1].my0, states[1].vy0):
        t.zero_()
    states[1].y0.fill_(0.3)
    batch.step()
    torch.cuda.synchronize()
    assert int(batch.iter.item()) == 3


@pytest.mark.parametrize("prec,d,w,L,N,M", [
    ("bf16", 150, 160, 2, 3, 300),   # 10 x 10 tiles: the whole step fits LDS
    ("bf16", 170, 180, 2, 4, 200),   # 12 x 12: layer-streamed
    ("bf16", 188, 198, 2, 3, 150),   # 14 x 14: layer-streamed
    ("bf16", 230, 240, 1, 3, 100),   # 16 x 16, depth 1: layer-streamed
    ("fp32", 120, 125, 2, 3, 150),   # fp32 8 x 8: layer-streamed
])
def test_layer_streamed_kernels_are_bitwise_identical(prec, d, w, L, N, M):
    """Step networks whose weights do not fit LDS at once run one layer at a
    time through LDS (lds modes 1 and 2); the global-fragment kernels (lds 0)
    give the same bits."""
    prob = I.allen_cahn(d)
    net = dict(width=w, depth=L, prec=prec)
    p32, _, y0 = inputs(prob, net, N, seed=5, y0=0.3)
    plan = Plan(prob, net, N, M)
    print(f"d={d} w={w} L={L} {prec} config {plan.get_config()}", flush=True)
    ref = _fb(plan, p32, y0)
    assert np.all(np.isfinite(ref[1]))
    for lds in (1, 0):
        plan.config(lds=lds)
        got = _fb(plan, p32, y0)
        assert got[0] == ref[0] and got[2] == ref[2], lds
        assert np.array_equal(got[1], ref[1]), lds


def test_layer_streamed_against_oracle():
    """A 14 x 14 bf16 step network (layer-streamed forward and reverse sweep)
    against the oracle's bf16 emulation, every block normwise and
    elementwise."""
    prob = I.allen_cahn(190)
    net = dict(width=200, depth=2, prec="bf16")
    N, M = 3, 96
    p32, p64, y0 = inputs(prob, net, N, seed=8, y0=0.3)
    plan = Plan(prob, net, N, M)
    assert plan.get_config()["ti"] == 14
    lg, gg, gy = run_gpu(plan, p32, y0, 4, 1)
    emu = O.loss_grad(prob, oracle_net(net), N, M, p64, y0, seed=4, it=1)
    assert abs(lg - emu["loss"]) <= 1e-3 * abs(emu["loss"]), (lg, emu["loss"])
    assert abs(gy - emu["grad_y0"]) <= 1e-3 * abs(emu["grad_y0"]) + 1e-12
    check_grad(prob, net, N, gg, emu["grad"], 1e-2)
