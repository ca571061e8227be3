"""Training driver: Adam on the library's fused forward + reverse sweep, with
the multilevel warm start of Sec. 3.2 (time grids N, 2N, 4N, ...; the
parameters of each level initialise the next through fbsde_prolong).

Every hot step is a library call on torch's current stream; Y0 and the loss
are logged on the device each iteration and read back once per level, so
the loop never synchronises the host inside a level.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import torch

from . import inputs as I
from .plan import Plan


@dataclasses.dataclass
class Level:
    N: int
    iters: int


@dataclasses.dataclass
class History:
    N: np.ndarray          # time steps of the level of every iteration
    y0: np.ndarray         # Y0 after every iteration
    loss: np.ndarray       # loss of every iteration (before its update)
    t: np.ndarray          # seconds since the first timed iteration, at its end
    level_seconds: list
    params: torch.Tensor
    y0_final: float


def multilevel_schedule(levels, iters_per_level) -> list:
    if isinstance(iters_per_level, int):
        iters_per_level = [iters_per_level] * len(levels)
    return [Level(int(n), int(k)) for n, k in zip(levels, iters_per_level)]


def train(problem: dict, net: dict, M: int, schedule: list, *, lr: float = 1e-3, lr_y0: float = 1e-2,
          seed: int = 1, init_seed: int = 0, y0_init: float | None = None,
          params_init: np.ndarray | None = None, device: str = "cuda", plans: dict | None = None,
          warmup: int = 0) -> History:
    """Adam over the levels of `schedule` (a list of Level).  y0 starts at the
    pilot mean of g(X_N) on the first level unless y0_init is given.  Adam
    moments restart at every level.  `warmup` untimed iterations run on the
    first level (on a copy of the parameters) before the clock starts."""
    plans = {} if plans is None else plans

    def plan_for(N):
        if N not in plans:
            plans[N] = Plan(problem, net, N, M, device=device)
        return plans[N]

    lv0 = schedule[0]
    P0 = plan_for(lv0.N)
    if params_init is None:
        params_init = I.init_params(problem, net, lv0.N, seed=init_seed)
    params = torch.from_numpy(np.asarray(params_init, dtype=np.float32)).to(P0.device)
    if y0_init is None:
        y0_init = float(P0.terminal_mean(seed ^ 0x5A5A, 0).item())
    y0 = torch.tensor(float(y0_init), dtype=torch.float64, device=P0.device)

    if warmup > 0:
        _run_level(P0, params.clone(), y0.clone(), warmup, lr, lr_y0, seed + 7919, None, None, 0)
    torch.cuda.synchronize()

    Ns, ys, ls, ts, level_seconds = [], [], [], [], []
    t_start = time.perf_counter()
    t_prev = 0.0
    it0 = 0
    for li, lv in enumerate(schedule):
        P = plan_for(lv.N)
        if li > 0:
            Pc = plan_for(schedule[li - 1].N)
            if P.N != 2 * Pc.N:
                raise ValueError("multilevel schedule must double N at every level")
            params = Pc.prolong_to(P, params)
        ylog = torch.empty(lv.iters, dtype=torch.float64, device=P.device)
        llog = torch.empty(lv.iters, dtype=torch.float64, device=P.device)
        params, y0 = _run_level(P, params, y0, lv.iters, lr, lr_y0, seed, ylog, llog, it0)
        torch.cuda.synchronize()
        t_now = time.perf_counter() - t_start
        dt_level = t_now - t_prev
        level_seconds.append(dt_level)
        Ns.append(np.full(lv.iters, lv.N))
        ys.append(ylog.cpu().numpy())
        ls.append(llog.cpu().numpy())
        ts.append(t_prev + dt_level * (np.arange(1, lv.iters + 1) / lv.iters))
        t_prev = t_now
        it0 += lv.iters
    return History(N=np.concatenate(Ns), y0=np.concatenate(ys), loss=np.concatenate(ls),
                   t=np.concatenate(ts), level_seconds=level_seconds, params=params,
                   y0_final=float(y0.item()))


def _run_level(P: Plan, params, y0, iters, lr, lr_y0, seed, ylog, llog, it0):
    dev = P.device
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    my = torch.zeros((), dtype=torch.float64, device=dev)
    vy = torch.zeros((), dtype=torch.float64, device=dev)
    loss = torch.empty((), dtype=torch.float64, device=dev)
    grad = torch.empty_like(params)
    gy = torch.empty((), dtype=torch.float64, device=dev)
    for k in range(iters):
        P.forward_backward(params, y0, seed, it0 + k, out=(loss, grad, gy))
        P.adam_step(params, y0, grad, gy, m, v, my, vy, k + 1, lr=lr, lr_y0=lr_y0)
        if llog is not None:
            llog[k].copy_(loss, non_blocking=True)
            ylog[k].copy_(y0, non_blocking=True)
    return params, y0


def time_to_accuracy(h: History, target: float, rel: float = 0.01, hold: int = 100,
                     finest_N: int | None = None) -> float | None:
    """Seconds until the first iteration on the finest level from which Y0
    stays within `rel` of `target` for the next `hold` iterations (None if
    never)."""
    finest_N = int(h.N.max()) if finest_N is None else finest_N
    ok = (np.abs(h.y0 / target - 1.0) <= rel) & (h.N == finest_N)
    n = len(ok)
    for i in range(n - hold + 1):
        if ok[i:i + hold].all():
            return float(h.t[i])
    return None
