"""GPU parity of the paper's own formulation (one u-network, Z = grad u,
per-step residual loss, terminal-gradient penalty; FC, residual and NAIS
blocks) against the FP64 oracle on the same seeded inputs, through the C ABI.

Tolerances (fp32 arithmetic): loss <= 1e-5 relative, u(0, x0) <= 1e-5,
every parameter block's gradient <= 1e-4 normwise and elementwise."""
import numpy as np
import pytest
import torch

from oracle import core as O
from paper_1910_11623_amd import inputs as I

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_1910_11623_amd.plan import UPlan

KIND = {"fc": "u_fc", "res": "u_res", "nais": "u_nais"}


def _problem(name, d):
    return {"bsb": I.bsb, "hjb": I.hjb, "ac": I.allen_cahn}[name](d)


def unet_blocks(d, w, K, arch):
    """(name, slice) of every block of the u-network's flat layout."""
    out, off = [], 0

    def add(name, n):
        nonlocal off
        out.append((name, slice(off, off + n)))
        off += n
    add("W0", w * (d + 1))
    add("b0", w)
    for k in range(1, K + 1):
        add(f"A{k}", w * w)
        if arch == "nais":
            add(f"E{k}", w * (d + 1))
        add(f"b{k}", w)
    add("wo", w)
    add("bo", 1)
    return out


def unet_params(prob, net, seed=0, scale=None):
    """Glorot-uniform weights, zero biases, small output layer (fp32 values)."""
    rng = np.random.default_rng(seed)
    d, w, K = int(prob["d"]), int(net["width"]), int(net["depth"])
    n = O.unet_param_count(prob, dict(arch=net["arch"], width=w, depth=K))
    p = np.zeros(n)
    for name, sl in unet_blocks(d, w, K, net["arch"]):
        m = sl.stop - sl.start
        if name.startswith("W0") or name.startswith("E"):
            a = np.sqrt(6.0 / (w + d + 1))
            p[sl] = rng.uniform(-a, a, m)
        elif name.startswith("A"):
            a = np.sqrt(6.0 / (2 * w)) * (0.5 if net["arch"] == "nais" else 1.0)
            p[sl] = rng.uniform(-a, a, m)
        elif name == "wo":
            p[sl] = rng.uniform(-1, 1, m) * np.sqrt(6.0 / (w + 1))
        elif scale is not None:
            p[sl] = scale * rng.standard_normal(m)
    return p.astype(np.float32)


def run_gpu(plan, p32, seed, it, grad=True):
    params = torch.from_numpy(p32).to(plan.device)
    loss, g, y0 = plan.forward_backward(params, seed, it, grad=grad)
    torch.cuda.synchronize()
    return float(loss.item()), (g.cpu().numpy().astype(np.float64) if grad else None), float(y0.item())


def check(prob, net, N, M, p32, kappa, seed=3, it=1):
    onet = dict(arch=net["arch"], width=net["width"], depth=net["depth"], eps=net.get("eps", 0.01))
    plan = UPlan(prob, dict(kind=KIND[net["arch"]], width=net["width"], depth=net["depth"]), N, M, kappa=kappa,
                 eps=onet["eps"])
    assert plan.n_params == O.unet_param_count(prob, onet)
    print(f"u-network {net} d={prob['d']} N={N} M={M} kappa={kappa}", flush=True)
    lg, gg, y0 = run_gpu(plan, p32, seed, it)
    ref = O.unet_loss_grad(prob, onet, N, M, p32.astype(np.float64), seed=seed, it=it, kappa=kappa, want_uz=True)
    assert abs(lg - ref["loss"]) <= 1e-5 * abs(ref["loss"]), (lg, ref["loss"])
    assert abs(y0 - ref["U"][0, 0]) <= 1e-5 * max(1.0, abs(ref["U"][0, 0])), (y0, ref["U"][0, 0])
    worst, worst_m = ("", 0.0), ("", 0.0)
    for name, sl in unet_blocks(int(prob["d"]), net["width"], net["depth"], net["arch"]):
        a, b = gg[sl], ref["grad"][sl]
        nb = np.linalg.norm(b)
        r = np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)
        mb = np.abs(b).max()
        rm = np.abs(a - b).max() / mb if mb > 0 else np.abs(a - b).max()
        worst = max(worst, (name, r), key=lambda t: t[1])
        worst_m = max(worst_m, (name, rm), key=lambda t: t[1])
    print(f"gradient: worst normwise {worst}, elementwise {worst_m}", flush=True)
    assert worst[1] <= 1e-4, worst
    assert worst_m[1] <= 1e-4, worst_m
    return plan, ref


@pytest.mark.parametrize("arch", ["fc", "res", "nais"])
@pytest.mark.parametrize("pname", ["bsb", "hjb", "ac"])
def test_unet_loss_and_gradient(arch, pname):
    prob = _problem(pname, 5)
    net = dict(arch=arch, width=16, depth=2)
    p = unet_params(prob, net, seed=2, scale=0.1)
    check(prob, net, 4, 40, p, kappa=0.5)


@pytest.mark.parametrize("arch,d,w,K,N,M,kappa", [
    ("fc", 7, 18, 1, 3, 33, 0.0),      # ragged d, w (row stride 20), one block, no penalty
    ("res", 1, 8, 3, 5, 17, 1.0),      # d = 1
    ("fc", 12, 64, 2, 20, 500, 0.3),   # 10500 rows: many row tiles and weight-gradient splits
    ("nais", 9, 24, 3, 6, 70, 0.2),
])
def test_unet_ragged_shapes(arch, d, w, K, N, M, kappa):
    prob = I.hjb(d) if arch != "res" else I.bsb(d)
    net = dict(arch=arch, width=w, depth=K)
    p = unet_params(prob, net, seed=7, scale=0.05)
    check(prob, net, N, M, p, kappa)


def test_unet_paper_configuration():
    """Sec. 4.1 set-up: BSB d = 100, N = 50, M = 100, four fully connected
    layers of width 256 (the input layer and three blocks)."""
    prob = I.bsb(100)
    net = dict(arch="fc", width=256, depth=3)
    p = unet_params(prob, net, seed=0)
    check(prob, net, 50, 100, p, kappa=0.0, seed=1, it=0)


def test_unet_states_match_oracle():
    prob = I.allen_cahn(6)
    net = dict(arch="res", width=12, depth=2)
    p = unet_params(prob, net, seed=4, scale=0.1)
    N, M = 5, 30
    plan, ref = check(prob, net, N, M, p, kappa=0.0)
    u, z = plan.states()
    u, z = u.cpu().numpy(), z.cpu().numpy()
    np.testing.assert_allclose(u, ref["U"].reshape(-1), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(z, ref["Z"].reshape(-1, 6), rtol=1e-4, atol=1e-6)


def test_unet_deterministic_and_forward_only():
    prob = I.hjb(10)
    net = dict(arch="fc", width=32, depth=2)
    p = unet_params(prob, net, seed=1)
    plan = UPlan(prob, dict(kind="u_fc", width=32, depth=2), 8, 300, kappa=0.2)
    a = run_gpu(plan, p, 5, 2)
    b = run_gpu(plan, p, 5, 2)
    c = run_gpu(plan, p, 5, 2, grad=False)
    assert a[0] == b[0] == c[0] and a[2] == b[2] == c[2]
    assert np.array_equal(a[1], b[1])


def test_unet_nais_projection_matches_oracle():
    prob = I.bsb(4)
    net = dict(arch="nais", width=20, depth=3, eps=0.01)
    p = unet_params(prob, net, seed=3, scale=0.1)
    # make the first block infeasible, leave the others as drawn
    sl = unet_blocks(4, 20, 3, "nais")[2][1]
    p[sl] *= 3.0
    plan = UPlan(prob, dict(kind="u_nais", width=20, depth=3), 2, 8)
    t = torch.from_numpy(p).cuda()
    plan.nais_project(t, 0.98)
    torch.cuda.synchronize()
    got = t.cpu().numpy().astype(np.float64)
    ref = p.astype(np.float64)
    O.unet_nais_project(prob, net, ref, 0.98)
    np.testing.assert_allclose(got, ref, rtol=2e-6, atol=1e-7)


def test_unet_adam_matches_oracle():
    prob = I.bsb(5)
    plan = UPlan(prob, dict(kind="u_res", width=8, depth=2), 4, 16)
    n = plan.n_params
    rng = np.random.default_rng(0)
    th = rng.standard_normal(n).astype(np.float32)
    th64, m, v = th.astype(np.float64), np.zeros(n), np.zeros(n)
    pt = torch.from_numpy(th).cuda()
    mt, vt = torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    for t in range(1, 6):
        g = rng.standard_normal(n).astype(np.float32)
        plan.adam_step(pt, torch.from_numpy(g).cuda(), mt, vt, t, lr=1e-3)
        O.adam(th64, g.astype(np.float64), m, v, t, lr=1e-3)
    torch.cuda.synchronize()
    np.testing.assert_allclose(pt.cpu().numpy(), th64, rtol=1e-6, atol=1e-6)


def test_unet_invalid_calls():
    import paper_1910_11623_amd.binding as B
    prob = I.bsb(3)
    plan = UPlan(prob, dict(kind="u_fc", width=8, depth=1), 2, 4)
    params = torch.zeros(plan.n_params, device="cuda")
    y0 = torch.zeros((), dtype=torch.float64, device="cuda")
    out = torch.zeros((), dtype=torch.float64, device="cuda")
    # the Deep-BSDE entry points refuse a u-network plan
    st = plan.lib.fbsde_forward(plan._h, params.data_ptr(), y0.data_ptr(), 0, 0, out.data_ptr(),
                                plan.ws.data_ptr(), None)
    assert st == B.ERR_UNSUPPORTED
    with pytest.raises(B.FbsdeError):
        plan.nais_project(params, 1.0)  # not a NAIS plan


def test_unet_evaluation_from_a_perturbed_initial_condition():
    """Sec. 4 generalisation experiment: the network trained at x0 is
    evaluated on paths from x0' without re-optimisation.  After
    fbsde_plan_set_x0 the forward pass (no gradient) gives u and Z along the
    new paths: against the oracle run on the problem with x0'."""
    prob = I.bsb(8)
    net = dict(arch="nais", width=24, depth=2)
    p = unet_params(prob, net, seed=9, scale=0.05)
    N, M = 6, 50
    plan = UPlan(prob, dict(kind="u_nais", width=24, depth=2), N, M)
    rng = np.random.default_rng(2)
    x1 = np.asarray(prob["x0"]) * (1.0 + 0.2 * rng.standard_normal(8))
    plan.set_x0(x1)
    lg, _, y0 = run_gpu(plan, p, 4, 3, grad=False)
    u, z = plan.states()
    u, z = u.cpu().numpy(), z.cpu().numpy()
    prob1 = dict(prob, x0=x1)
    ref = O.unet_loss_grad(prob1, dict(net, eps=0.01), N, M, p.astype(np.float64), seed=4, it=3, want_grad=False,
                           want_uz=True)
    assert abs(lg - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    np.testing.assert_allclose(u, ref["U"].reshape(-1), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(z, ref["Z"].reshape(-1, 8), rtol=1e-4, atol=1e-6)
    assert y0 == pytest.approx(ref["U"][0, 0], rel=1e-5)
