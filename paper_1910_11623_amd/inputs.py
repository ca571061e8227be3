"""Seeded synthetic inputs shared by the library's callers and the tests.

This module holds no arithmetic of the method: it only describes the paper's
benchmark problems (Sec. 4: Black–Scholes–Barenblatt, Hamilton–Jacobi–Bellman,
Allen–Cahn) as plain parameter dicts, and draws initial network weights
(Glorot-uniform, zero biases) from numpy's PCG64 generator.  The Brownian
increments are not drawn here: each side implements the counter-based Philox
generator from its published definition.
"""
from __future__ import annotations

import math

import numpy as np


def bsb_x0(d: int) -> np.ndarray:
    """x0 = (1, 0.5, 1, 0.5, ...) for the Black–Scholes–Barenblatt problem."""
    return np.array([1.0 if i % 2 == 0 else 0.5 for i in range(d)])


def bsb(d: int = 100, T: float = 1.0, r: float = 0.05, sigma: float = 0.4) -> dict:
    """Black–Scholes–Barenblatt (Sec. 4): sigma(x) dW = sigma x (.) dW,
    driver r (y - z.x), g(x) = |x|^2."""
    return dict(name="bsb", d=d, T=T, x0=bsb_x0(d), sde="gbm_diag", sde_s=sigma,
                drv="bsb", drv_p=[r, 0.0], g="norm2", g_p=[0.0, 0.0])


def hjb(d: int = 100, T: float = 1.0, lam: float = 1.0) -> dict:
    """Hamilton–Jacobi–Bellman (Sec. 4): X = x0 + sqrt(2) W, x0 = 0,
    driver lam |z|^2, g(x) = ln((1 + |x|^2) / 2)."""
    return dict(name="hjb", d=d, T=T, x0=np.zeros(d), sde="scaled_bm", sde_s=math.sqrt(2.0),
                drv="hjb", drv_p=[lam, 0.0], g="loghalf", g_p=[0.0, 0.0])


def allen_cahn(d: int = 20, T: float = 0.3) -> dict:
    """Allen–Cahn (Sec. 4): X = x0 + sqrt(2) W, x0 = 0, driver y^3 - y,
    g(x) = 1 / (2 + 0.4 |x|^2)."""
    return dict(name="ac", d=d, T=T, x0=np.zeros(d), sde="scaled_bm", sde_s=math.sqrt(2.0),
                drv="ac", drv_p=[0.0, 0.0], g="inv", g_p=[2.0, 0.4])


def mlp_net(width: int, depth: int = 2) -> dict:
    return dict(kind="mlp", width=width, depth=depth)


def resnet_net(width: int, blocks: int = 4) -> dict:
    return dict(kind="resnet", width=width, depth=blocks)


def _layers(d: int, net: dict):
    """(out, in) shapes of the dense layers of one network, in layout order."""
    w, L = int(net["width"]), int(net.get("depth", 2))
    if net.get("kind", "mlp") == "mlp":
        return [(w, d)] + [(w, w)] * (L - 1) + [(d, w)]
    return [(w, d + 1)] + [(w, w)] * L + [(d, w)]


def init_params(problem: dict, net: dict, N: int, seed: int = 0,
                out_scale: float = 1.0) -> np.ndarray:
    """Glorot-uniform weights, zero biases, z0 = 0, in the flat layout
    (row-major W[out][in] followed by b[out], layer after layer, step after
    step; the per-step form starts with z0[d])."""
    rng = np.random.default_rng(seed)
    d = int(problem["d"])
    parts = []
    nets = 1
    if net.get("kind", "mlp") == "mlp":
        parts.append(np.zeros(d))
        nets = N - 1
    for _ in range(nets):
        lay = _layers(d, net)
        for k, (o, i) in enumerate(lay):
            a = math.sqrt(6.0 / (o + i))
            W = rng.uniform(-a, a, size=(o, i))
            if k == len(lay) - 1:
                W = W * out_scale
            parts.append(W.ravel())
            parts.append(np.zeros(o))
    return np.concatenate(parts) if parts else np.zeros(0)


def param_count(problem: dict, net: dict, N: int) -> int:
    d = int(problem["d"])
    per = sum(o * i + o for (o, i) in _layers(d, net))
    if net.get("kind", "mlp") == "mlp":
        return d + (N - 1) * per
    return per


def allen_cahn_batch(n: int = 32, seed: int = 2019):
    """(d, N) of n Allen–Cahn instances: d uniform on the integers 20..200,
    N uniform on {10, 20, 40}; width w = d + 10 (two hidden layers)."""
    rng = np.random.default_rng(seed)
    ds = rng.integers(20, 201, size=n)
    Ns = rng.choice([10, 20, 40], size=n)
    return [(int(d), int(N)) for d, N in zip(ds, Ns)]


def unet_blocks(d: int, net: dict):
    """(name, rows, cols) of the blocks of the u-network's flat layout
    (arch "fc" | "res" | "nais", depth K blocks after the input layer)."""
    w, K, arch = int(net["width"]), int(net.get("depth", 3)), net.get("arch", "fc")
    out = [("W0", w, d + 1), ("b0", w, 1)]
    for k in range(1, K + 1):
        out.append((f"R{k}" if arch == "nais" else f"A{k}", w, w))
        if arch == "nais":
            out.append((f"E{k}", w, d + 1))
        out.append((f"b{k}", w, 1))
    out += [("wo", 1, w), ("bo", 1, 1)]
    return out


def init_unet_params(problem: dict, net: dict, seed: int = 0, out_scale: float = 1.0) -> np.ndarray:
    """Glorot-uniform weight blocks, zero biases (the u-network of the
    paper's own formulation); NAIS R_k at half the Glorot range."""
    rng = np.random.default_rng(seed)
    d = int(problem["d"])
    parts = []
    for name, r, c in unet_blocks(d, net):
        if name.startswith("b"):
            parts.append(np.zeros(r * c))
            continue
        fan = (r + c) if name != "wo" else (c + 1)
        a = math.sqrt(6.0 / fan)
        if name.startswith("R"):
            a *= 0.5
        if name == "wo":
            a *= out_scale
        parts.append(rng.uniform(-a, a, size=r * c))
    return np.concatenate(parts)
