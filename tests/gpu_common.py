"""Helpers shared by the GPU parity tests: run the library and the oracle on
the same seeded inputs and compare."""
from __future__ import annotations

import numpy as np
import torch

from oracle import core as O
from paper_1910_11623_amd import inputs as I


def blocks(problem: dict, net: dict, N: int):
    """(name, slice) of every parameter block of the flat layout."""
    d = int(problem["d"])
    out = []
    off = 0
    if net.get("kind", "mlp") == "mlp":
        out.append(("z0", slice(0, d)))
        off = d
        nets = range(1, N)
    else:
        nets = [0]
    for n in nets:
        for k, (o, i) in enumerate(I._layers(d, net)):
            out.append((f"W{k}@{n}", slice(off, off + o * i)))
            off += o * i
            out.append((f"b{k}@{n}", slice(off, off + o)))
            off += o
    return out


def oracle_net(net: dict) -> dict:
    return dict(kind=net.get("kind", "mlp"), width=net["width"], depth=net.get("depth", 2),
                bf16=net.get("prec", "fp32") == "bf16")


def inputs(problem, net, N, seed=0, y0=None, z0_scale=0.1):
    """fp32 parameters (as the library sees them) and the same values in fp64."""
    p = I.init_params(problem, net, N, seed=seed)
    d = int(problem["d"])
    if net.get("kind", "mlp") == "mlp":
        rng = np.random.default_rng(seed + 100)
        p[:d] = z0_scale * rng.standard_normal(d)
    p32 = p.astype(np.float32)
    if y0 is None:
        y0 = 1.0
    return p32, p32.astype(np.float64), float(y0)


def run_gpu(plan, p32, y0, seed, it, grad=True):
    dev = plan.device
    params = torch.from_numpy(p32).to(dev)
    y = torch.tensor(y0, dtype=torch.float64, device=dev)
    if grad:
        loss, g, gy = plan.forward_backward(params, y, seed, it)
        torch.cuda.synchronize()
        return float(loss.item()), g.cpu().numpy().astype(np.float64), float(gy.item())
    loss = plan.forward(params, y, seed, it)
    torch.cuda.synchronize()
    return float(loss.item()), None, None


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def blockwise_rel(problem, net, N, g, gref):
    return {name: rel(g[s], gref[s]) for name, s in blocks(problem, net, N)}


def run_oracle(problem, net, N, M, p64, y0, seed, it, grad=True):
    return O.loss_grad(problem, oracle_net(net), N, M, p64, y0, seed=seed, it=it, want_grad=grad)


def maxrel(a, b):
    """max |a - b| / max |b| (elementwise error on the block's own scale)."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = float(np.abs(b).max()) if b.size else 0.0
    err = float(np.abs(a - b).max()) if b.size else 0.0
    return err / den if den > 0 else err


def blockwise_maxrel(problem, net, N, g, gref):
    return {name: maxrel(g[s], gref[s]) for name, s in blocks(problem, net, N)}


def check_grad(problem, net, N, g, gref, tol):
    """Every parameter block's gradient within `tol`, normwise
    (|g - g*| / |g*|) and elementwise (max |g - g*| / max |g*|)."""
    br = blockwise_rel(problem, net, N, g, gref)
    bm = blockwise_maxrel(problem, net, N, g, gref)
    worst = max(br.items(), key=lambda kv: kv[1])
    worst_m = max(bm.items(), key=lambda kv: kv[1])
    print(f"gradient: worst normwise {worst[0]} {worst[1]:.2e}, worst elementwise {worst_m[0]} {worst_m[1]:.2e}",
          flush=True)
    assert worst[1] <= tol, ("normwise", worst)
    assert worst_m[1] <= tol, ("elementwise", worst_m)
