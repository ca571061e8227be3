"""Training driver: Adam on the library's fused forward + reverse sweep, with
the multilevel warm start of Sec. 3.2 (time grids N, 2N, 4N, ...; the
parameters of each level initialise the next through fbsde_prolong).

Every hot step is a library call on torch's current stream; Y0 and the loss
are logged on the device each iteration and read back once per level, so
the loop never synchronises the host inside a level (the optional early
level switch reads Y0 back once per check window).
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import torch

from . import inputs as I
from .plan import Plan, UPlan


@dataclasses.dataclass
class Level:
    N: int
    iters: int   # iteration budget of the level (the most it runs)


@dataclasses.dataclass
class History:
    N: np.ndarray          # time steps of the level of every iteration
    y0: np.ndarray         # Y0 after every iteration
    loss: np.ndarray       # loss of every iteration (before its update)
    t: np.ndarray          # seconds since the first timed iteration, at its end
    level_seconds: list
    params: torch.Tensor
    y0_final: float
    level_iters: list = dataclasses.field(default_factory=list)  # iterations each level ran


def multilevel_schedule(levels, iters_per_level) -> list:
    if isinstance(iters_per_level, int):
        iters_per_level = [iters_per_level] * len(levels)
    return [Level(int(n), int(k)) for n, k in zip(levels, iters_per_level)]


def train(problem: dict, net: dict, M: int, schedule: list, *, lr: float = 1e-3, lr_y0: float = 1e-2,
          seed: int = 1, init_seed: int = 0, y0_init: float | None = None,
          params_init: np.ndarray | None = None, device: str = "cuda", plans: dict | None = None,
          warmup: int = 0, switch_rel: float | None = None, switch_window: int = 100) -> History:
    """Adam over the levels of `schedule` (a list of Level).  y0 starts at the
    pilot mean of g(X_N) on the first level unless y0_init is given.  Adam
    moments restart at every level.  `warmup` untimed iterations run on the
    first level (on a copy of the parameters) before the clock starts.

    Level switch: every level but the last runs its whole budget, unless
    `switch_rel` is given; then it also ends as soon as Y0 has changed by
    less than `switch_rel` (relative) over the last `switch_window`
    iterations, checked once per window (the only host synchronisation)."""
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
        st = _AdamState(params)
        _run_iters(P0, params.clone(), y0.clone(), st, 0, warmup, lr, lr_y0, seed + 7919, None, None, 0)
    torch.cuda.synchronize()

    Ns, ys, ls, ts, level_seconds, level_iters = [], [], [], [], [], []
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
        st = _AdamState(params)
        last = li == len(schedule) - 1
        if switch_rel is None or last:
            _run_iters(P, params, y0, st, 0, lv.iters, lr, lr_y0, seed, ylog, llog, it0)
            done = lv.iters
        else:
            done = 0
            while done < lv.iters:
                k = min(switch_window, lv.iters - done)
                _run_iters(P, params, y0, st, done, k, lr, lr_y0, seed, ylog, llog, it0)
                done += k
                if done >= 2 * switch_window:
                    a_, b_ = ylog[done - 1 - switch_window].item(), ylog[done - 1].item()
                    if abs(b_ - a_) <= switch_rel * abs(b_):
                        break
        torch.cuda.synchronize()
        t_now = time.perf_counter() - t_start
        dt_level = t_now - t_prev
        level_seconds.append(dt_level)
        level_iters.append(done)
        Ns.append(np.full(done, lv.N))
        ys.append(ylog[:done].cpu().numpy())
        ls.append(llog[:done].cpu().numpy())
        ts.append(t_prev + dt_level * (np.arange(1, done + 1) / done))
        t_prev = t_now
        it0 += done
    return History(N=np.concatenate(Ns), y0=np.concatenate(ys), loss=np.concatenate(ls),
                   t=np.concatenate(ts), level_seconds=level_seconds, params=params,
                   y0_final=float(y0.item()), level_iters=level_iters)


class _AdamState:
    """Adam moments of one level (zero at the level's start)."""

    def __init__(self, params):
        dev = params.device
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.my = torch.zeros((), dtype=torch.float64, device=dev)
        self.vy = torch.zeros((), dtype=torch.float64, device=dev)
        self.loss = torch.empty((), dtype=torch.float64, device=dev)
        self.grad = torch.empty_like(params)
        self.gy = torch.empty((), dtype=torch.float64, device=dev)


def _run_iters(P: Plan, params, y0, st: _AdamState, k0, iters, lr, lr_y0, seed, ylog, llog, it0):
    """Iterations k0 .. k0 + iters - 1 of a level (Adam step count k + 1),
    updating params and y0 in place."""
    for k in range(k0, k0 + iters):
        # forward_backward + adam_step as one call (same bits)
        P.train_step(params, y0, st.grad, st.gy, st.loss, st.m, st.v, st.my, st.vy, seed, it0 + k, k + 1, lr=lr,
                     lr_y0=lr_y0)
        if llog is not None:
            llog[k].copy_(st.loss, non_blocking=True)
            ylog[k].copy_(y0, non_blocking=True)


def first_accurate_iteration(h: History, target: float, rel: float = 0.01, hold: int = 100,
                             finest_N: int | None = None) -> int | None:
    """Index (over all levels) of the first iteration on the finest level
    from which Y0 stays within `rel` of `target` for the next `hold`
    iterations (None if never)."""
    finest_N = int(h.N.max()) if finest_N is None else finest_N
    ok = (np.abs(h.y0 / target - 1.0) <= rel) & (h.N == finest_N)
    n = len(ok)
    for i in range(n - hold + 1):
        if ok[i:i + hold].all():
            return i
    return None


def time_to_accuracy(h: History, target: float, rel: float = 0.01, hold: int = 100,
                     finest_N: int | None = None) -> float | None:
    """Seconds until the first iteration on the finest level from which Y0
    stays within `rel` of `target` for the next `hold` iterations (None if
    never)."""
    i = first_accurate_iteration(h, target, rel, hold, finest_N)
    return None if i is None else float(h.t[i])


def train_unet(problem: dict, net: dict, M: int, schedule: list, *, lr: float = 1e-3, seed: int = 1,
               init_seed: int = 0, params_init: np.ndarray | None = None, kappa: float = 0.0,
               eps: float = 0.01, nais_c: float | None = None, device: str = "cuda", plans: dict | None = None,
               warmup: int = 0, switch_rel: float | None = None, switch_window: int = 100) -> History:
    """Adam on the paper's own formulation (one u-network, residual loss):
    net = dict(kind="u_fc" | "u_res" | "u_nais", width, depth).  Y0 = u(0, x0)
    is logged every iteration.  The network is shared by every step, so the
    multilevel warm start carries it over unchanged; Adam moments restart at
    every level.  NAIS: after every Adam step each R_k is projected onto
    |R_k^T R_k|_F <= nais_c (default 1 - 2 eps).  Level switch as in train."""
    plans = {} if plans is None else plans
    arch = {"u_fc": "fc", "u_res": "res", "u_nais": "nais"}[net["kind"]]
    if arch == "nais" and nais_c is None:
        nais_c = 1.0 - 2.0 * eps

    def plan_for(N):
        if N not in plans:
            plans[N] = UPlan(problem, net, N, M, kappa=kappa, eps=eps, device=device)
        return plans[N]

    P0 = plan_for(schedule[0].N)
    if params_init is None:
        params_init = I.init_unet_params(problem, dict(net, arch=arch), seed=init_seed)
    params = torch.from_numpy(np.asarray(params_init, dtype=np.float32)).to(P0.device)

    def run(P, st, k0, iters, ylog, llog, it0):
        for k in range(k0, k0 + iters):
            P.forward_backward(params, seed, it0 + k, out=(st.loss, st.grad, st.y))
            P.adam_step(params, st.grad, st.m, st.v, k + 1, lr=lr)
            if arch == "nais":
                P.nais_project(params, nais_c)
            if ylog is not None:
                llog[k].copy_(st.loss, non_blocking=True)
                ylog[k].copy_(st.y, non_blocking=True)

    class _St:
        def __init__(self, p):
            self.m, self.v = torch.zeros_like(p), torch.zeros_like(p)
            self.grad = torch.empty_like(p)
            self.loss = torch.empty((), dtype=torch.float64, device=p.device)
            self.y = torch.empty((), dtype=torch.float64, device=p.device)

    if warmup > 0:
        keep = params.clone()
        run(P0, _St(params), 0, warmup, None, None, 0)
        params.copy_(keep)
    torch.cuda.synchronize()
    Ns, ys, ls, ts, level_seconds, level_iters = [], [], [], [], [], []
    t_start = time.perf_counter()
    t_prev = 0.0
    it0 = 0
    last_y = float("nan")
    for li, lv in enumerate(schedule):
        P = plan_for(lv.N)
        ylog = torch.empty(lv.iters, dtype=torch.float64, device=P.device)
        llog = torch.empty(lv.iters, dtype=torch.float64, device=P.device)
        st = _St(params)
        if switch_rel is None or li == len(schedule) - 1:
            run(P, st, 0, lv.iters, ylog, llog, it0)
            done = lv.iters
        else:
            done = 0
            while done < lv.iters:
                k = min(switch_window, lv.iters - done)
                run(P, st, done, k, ylog, llog, it0)
                done += k
                if done >= 2 * switch_window:
                    a_, b_ = ylog[done - 1 - switch_window].item(), ylog[done - 1].item()
                    if abs(b_ - a_) <= switch_rel * abs(b_):
                        break
        torch.cuda.synchronize()
        t_now = time.perf_counter() - t_start
        dt_level = t_now - t_prev
        level_seconds.append(dt_level)
        level_iters.append(done)
        Ns.append(np.full(done, lv.N))
        ys.append(ylog[:done].cpu().numpy())
        ls.append(llog[:done].cpu().numpy())
        ts.append(t_prev + dt_level * (np.arange(1, done + 1) / done))
        t_prev = t_now
        it0 += done
        last_y = float(ys[-1][-1])
    return History(N=np.concatenate(Ns), y0=np.concatenate(ys), loss=np.concatenate(ls),
                   t=np.concatenate(ts), level_seconds=level_seconds, params=params, y0_final=last_y,
                   level_iters=level_iters)


def first_accurate_mean_iteration(h: History, target: float, rel: float = 0.01, window: int = 100,
                                  hold: int = 500, finest_N: int | None = None) -> int | None:
    """Index of the first iteration on the finest level at which the mean of
    Y0 over the trailing `window` finest-level iterations is within `rel` of
    `target` and stays so for the next `hold` iterations (None if never).
    For noisy Y0 trajectories (the paper's formulation at M = 100 paths,
    where Y0 = u(0, x0) moves with every Adam step)."""
    finest_N = int(h.N.max()) if finest_N is None else finest_N
    idx = np.nonzero(h.N == finest_N)[0]
    if idx.size < window:
        return None
    y = h.y0[idx]
    c = np.cumsum(np.concatenate([[0.0], y]))
    mean = (c[window:] - c[:-window]) / window          # mean[k] = mean of y[k .. k + window)
    ok = np.abs(mean / target - 1.0) <= rel
    for k in range(len(ok) - hold):
        if ok[k:k + hold + 1].all():
            return int(idx[k + window - 1])
    return None
