#!/usr/bin/env python3
"""Throughput and time-to-accuracy of the deep-FBSDE hot path on one GPU.

Workload (the throughput configuration): Black–Scholes–Barenblatt, d = 100,
T = 1, r = 0.05, sigma = 0.4, x0 = (1, 0.5, ...), M = 4096 paths, N = 32
steps, one MLP per step (2 hidden tanh layers of width 110), fp32.  A step is
one training iteration: Philox increments, Euler–Maruyama paths, every
network, the Y recursion, the loss, the reverse sweep and Adam.

Printed: one JSON line with path-steps/s, the dominant kernel against its
roofline (HIP events on the launch stream), the FP64 CPU oracle timed on a
bounded sample of the same workload, and the time until Y0 is within 1% of
the closed form exp((r + sigma^2) T) |x0|^2 = 77.1049, single level and
multilevel (4 -> 8 -> 16 -> 32 steps), for the library and for a plain FP32
PyTorch-eager implementation of the same method.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "train path-steps/s (fwd+bwd) at d=100; time to Y0 within 1% vs plain FP32"
D, W, DEPTH, N, M = 100, 110, 2, 32, 4096
PEAK_FP32_MFMA = 157.3   # TFLOP/s, MI355X dense fp32 matrix
PEAK_BF16_MFMA = 2500.0  # TFLOP/s, MI355X dense bf16 matrix
PEAK_HBM = 8000.0        # GB/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_flops(net_prec: str, d: int, w: int, L: int, n_steps: int, paths: int) -> dict:
    """Algorithmic flops per launch of the MFMA kernels (useful work only:
    no padding, 2 flops per multiply-add, 1 per bias add)."""
    rows = paths * (n_steps - 1)
    fwd = 2 * (w * d + (L - 1) * w * w + d * w) * rows
    bwd = 2 * (w * d + (L - 1) * w * w) * rows
    wgrad = (2 * (w * d + (L - 1) * w * w + d * w) + (L * w + d)) * rows + d * paths
    return {"forward": fwd, "backward": bwd, "wgrad": wgrad, "reverse": bwd + wgrad}


def step_net_params(d: int, w: int, L: int) -> int:
    """Weights and biases of one step's MLP (d -> w -> ... -> w -> d)."""
    return w * (d + 1) + (L - 1) * w * (w + 1) + d * (w + 1)


def kernel_alg_bytes(net_prec: str, d: int, w: int, L: int, n_steps: int, paths: int) -> dict:
    """Algorithmic HBM bytes per launch of the MFMA kernels on the method's
    own basis: the step networks' weights once per pass (in the GEMM
    precision; the weight gradient written once in fp32) and two fp32
    scalars per path-step (Y_n or c_n, lambda), the Brownian increments and
    hence X_n being regenerable from their counters.  Whatever an
    implementation keeps between its kernels (X_n, activations, deltas) is
    not algorithmic: the counter traffic over these bytes measures it."""
    esz = 4 if net_prec == "fp32" else 2
    rows = paths * (n_steps - 1)
    nw = (n_steps - 1) * step_net_params(d, w, L)
    per_row = 8
    return {"forward": esz * nw + per_row * rows,
            "backward": esz * nw + per_row * rows,
            "wgrad": 4 * nw + per_row * rows,
            "reverse": esz * nw + 4 * nw + per_row * rows}


def _quantiles(xs) -> dict:
    a = np.sort(np.asarray(xs, dtype=np.float64))
    return {"n": int(a.size), "median": round(float(np.median(a)), 5),
            "p10": round(float(np.percentile(a, 10)), 5), "p90": round(float(np.percentile(a, 90)), 5),
            "mean": round(float(a.mean()), 5)}


def time_library(prec: str, steps: int, warmup: int, min_samples: int = 100):
    """Training steps of the throughput configuration: the mean over exactly
    `steps` timed steps (HIP events around the whole region), then the
    median / p10 / p90 of at least `min_samples` single steps (one event
    pair per step, a separate run), then per-kernel durations from the
    library's own HIP events on its launch stream."""
    import torch
    from paper_1910_11623_amd import inputs as I
    from paper_1910_11623_amd.plan import Plan

    prob = I.bsb(D)
    net = dict(kind="mlp", width=W, depth=DEPTH, prec=prec)
    plan = Plan(prob, net, N, M)
    params = torch.from_numpy(I.init_params(prob, net, N, seed=0).astype(np.float32)).cuda()
    y0 = torch.tensor(73.0, dtype=torch.float64, device="cuda")
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    my, vy = torch.zeros_like(y0), torch.zeros_like(y0)
    out = (torch.empty((), dtype=torch.float64, device="cuda"), torch.empty_like(params),
           torch.empty((), dtype=torch.float64, device="cuda"))
    k_next = [0]

    def step():  # forward + reverse sweep + Adam (fbsde_train_step: the reduction applies the update)
        k = k_next[0]
        plan.train_step(params, y0, out[1], out[2], out[0], m, v, my, vy, 1, k, k + 1, lr=1e-3, lr_y0=1e-2)
        k_next[0] = k + 1

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps

    ns = max(min_samples, steps)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(ns + 1)]
    ev[0].record()
    for i in range(ns):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    stats = _quantiles([ev[i].elapsed_time(ev[i + 1]) for i in range(ns)])

    # per-kernel durations, HIP events recorded by the library around each launch
    plan.profile(True)
    nprof = max(20, min(steps, 200))
    for _ in range(nprof):
        step()
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    kern = {k: (t / c if c else 0.0) for k, (t, c) in prof.items()}
    finite = bool(torch.isfinite(out[0]).item())
    return ms, stats, kern, finite


def bsb_closed_form_y0(d: int, T: float = 1.0, r: float = 0.05, sigma: float = 0.4) -> float:
    """u(0, x0) = exp((r + sigma^2) T) |x0|^2 of the Black-Scholes-Barenblatt
    problem (Sec. 4), x0 = (1, 0.5, 1, 0.5, ...)."""
    x0sq = sum(1.0 if i % 2 == 0 else 0.25 for i in range(d))
    return math.exp((r + sigma * sigma) * T) * x0sq


def resnet_multilevel_leg(levels=(8, 16, 32, 64), iters=(300, 300, 300, 600), lr_y0: float = 0.1):
    """BSB d=1000, M=16384, shared residual net (width 1024, 4 blocks, bf16,
    kept activations) trained through the multilevel schedule N = 8 -> 16 ->
    32 -> 64 (the shared net carries over unchanged): seconds per level,
    ms per iteration and the final Y0 against the closed form."""
    import torch
    from paper_1910_11623_amd import inputs as I
    from paper_1910_11623_amd.plan import Plan
    from paper_1910_11623_amd.train import multilevel_schedule, train

    d, Mr = 1000, 16384
    prob = I.bsb(d)
    net = dict(kind="resnet", width=1024, depth=4, prec="bf16")
    plans = {n: Plan(prob, net, n, Mr, recompute=False) for n in levels}
    p0 = I.init_params(prob, net, levels[0], seed=0, out_scale=0.1)
    target = bsb_closed_form_y0(d)
    h = train(prob, net, Mr, multilevel_schedule(levels, iters), lr=1e-3, lr_y0=lr_y0, seed=1,
              params_init=p0, plans=plans, warmup=3)
    torch.cuda.synchronize()
    y_last = h.y0[-100:]
    return {"levels": list(levels), "iters": list(iters), "lr_y0": lr_y0,
            "level_seconds": [round(t, 3) for t in h.level_seconds],
            "ms_per_iter": [round(1e3 * t / k, 3) for t, k in zip(h.level_seconds, iters)],
            "y0_start": round(float(h.y0[0]), 4), "y0_final": round(h.y0_final, 4),
            "y0_mean_last100": round(float(np.mean(y_last)), 4), "target": round(target, 4),
            "rel_err_final": round(abs(h.y0_final / target - 1.0), 5),
            "loss_first": float(h.loss[0]), "loss_last": float(h.loss[-1])}


def measured_traffic(kernel: str, prec: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain-copy calibration),
    or None when the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "bsb_d100_traffic.json")
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256"):
        return None
    t = rec.get("per_launch", {}).get(f"{kernel}_{prec}")
    return None if t is None else int(round(t["read_bytes"] + t["write_bytes"]))


# Kernel-name prefix -> the roofline keys the bench uses
_TRAFFIC_KEYS = {"k_pack": "pack", "k_pack_sde": "sde", "k_sde": "sde", "k_forward": "forward", "k_scan": "scan",
                 "k_backward": "backward", "k_wgrad": "wgrad", "k_reverse": "reverse", "k_reverse_bf": "reverse",
                 "k_reduce": "reduce", "k_reduce_adam": "reduce", "k_adam": "adam"}


def reverse_kernels(kern_ms: dict) -> dict:
    """Per-launch milliseconds keyed by the MFMA kernels that ran: the fused
    reverse kernel (timed in the library's backward slot, no weight-gradient
    launches) is reported as "reverse", carrying both flop counts."""
    k = dict(kern_ms)
    if k.get("wgrad", 0.0) == 0.0 and k.get("backward", 0.0) > 0.0:
        k["reverse"] = k.pop("backward")
        k.pop("wgrad", None)
    return k


def _counter_means(path: str, counter: str) -> dict:
    """{kernel name: mean over its dispatches of `counter`} from a rocprofv3
    --pmc CSV directory (values of one dispatch summed over dimensions)."""
    import csv
    import glob
    per = {}
    files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    for fn in files:
        for r in csv.DictReader(open(fn)):
            if r.get("Counter_Name") != counter:
                continue
            key = (r["Kernel_Name"], r.get("Dispatch_Id", r.get("Correlation_Id")))
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    sums = {}
    for (name, _), v in per.items():
        t = sums.setdefault(name, [0.0, 0])
        t[0] += v
        t[1] += 1
    return {k: v[0] / v[1] for k, v in sums.items()}


def summarize_traffic(fetch32: str, write32: str, fetch16: str, write16: str, copyf: str, copyw: str) -> dict:
    """HBM bytes per launch of the hot-path kernels from FETCH_SIZE and
    WRITE_SIZE runs (KiB per dispatch), each scaled so that a plain copy of
    known size reads and writes exactly its bytes; keyed by the bench's
    kernel names and tagged with the hash of the kernel source."""
    import hashlib
    n = (1 << 30)
    cf = max(_counter_means(copyf, "FETCH_SIZE").items(), key=lambda kv: kv[1])[1]
    cw = max(_counter_means(copyw, "WRITE_SIZE").items(), key=lambda kv: kv[1])[1]
    fscale, wscale = n / (cf * 1024.0), n / (cw * 1024.0)
    src = "paper_1910_11623_amd/csrc/kernels.hip"
    out = {"source": src, "source_sha256": hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest(),
           "workload": f"BSB d={D} N={N} M={M} per-step MLP {W}x{DEPTH}", "fetch_scale": fscale,
           "write_scale": wscale, "per_launch": {}}
    for prec, fd, wd in (("fp32", fetch32, write32), ("bf16", fetch16, write16)):
        fm, wm = _counter_means(fd, "FETCH_SIZE"), _counter_means(wd, "WRITE_SIZE")
        for name, v in fm.items():
            short = name.split("(")[0].replace("void ", "").split("<")[0].split("::")[-1]
            key = _TRAFFIC_KEYS.get(short)
            if key is None:
                continue
            out["per_launch"][f"{key}_{prec}"] = {"read_bytes": v * 1024.0 * fscale,
                                                  "write_bytes": wm.get(name, 0.0) * 1024.0 * wscale,
                                                  "kernel": name.split("(")[0].replace("void fbsde::", "")}
    return out


def roofline_entry(prec: str, kern_ms: dict):
    """Roofline of the dominant MFMA kernel (the longest of forward, reverse
    sweep and weight gradient, or the fused reverse kernel that does both of
    the latter): its algorithmic flops per launch over its
    average launch duration, against the dense matrix peak of its own dtype
    (157.3 TFLOP/s fp32, 2.5 PFLOP/s bf16).  On the method's byte basis
    (weights once per pass, X_n and two scalars per path-step) every one of
    these kernels sits far above the ridge point, so the matrix peak is the
    bound.  `traffic` is the counter-measured HBM bytes per launch and
    `traffic_ratio` its multiple of the algorithmic bytes."""
    kern_ms = reverse_kernels(kern_ms)
    flops = {k: v for k, v in kernel_flops(prec, D, W, DEPTH, N, M).items() if k in kern_ms}
    nbytes = kernel_alg_bytes(prec, D, W, DEPTH, N, M)
    dom = max(flops, key=lambda k: kern_ms.get(k, 0.0))
    t = kern_ms[dom] * 1e-3
    peak = PEAK_FP32_MFMA if prec == "fp32" else PEAK_BF16_MFMA
    traffic = measured_traffic(dom, prec)
    achieved = flops[dom] / t / 1e12
    return dom, {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                 "frac": round(achieved / peak, 4), "traffic": traffic,
                 "algorithmic_bytes": int(nbytes[dom]),
                 "traffic_ratio": None if traffic is None else round(traffic / nbytes[dom], 2),
                 "kernel_ms": round(kern_ms[dom], 5)}


def step_roofline(prec: str, ms: float) -> dict:
    """The whole training step on the same basis: algorithmic flops of the
    forward, reverse sweep and weight gradients over the step time, against
    the matrix peak of the dtype."""
    f = kernel_flops(prec, D, W, DEPTH, N, M)
    fl = f["forward"] + f["backward"] + f["wgrad"]
    peak = PEAK_FP32_MFMA if prec == "fp32" else PEAK_BF16_MFMA
    return {"flops": int(fl), "achieved": round(fl / (ms * 1e-3) / 1e12, 3), "peak": peak,
            "frac": round(fl / (ms * 1e-3) / 1e12 / peak, 4)}


def _host_cpu() -> dict:
    """Core count the process may use and the CPU model of the host."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = min(avail, int(omp)) if omp and omp.isdigit() and int(omp) > 0 else avail
    return {"nproc": os.cpu_count(), "affinity": avail, "omp_num_threads": omp, "threads": threads,
            "model": model}


def _oracle_rate(threads: int, target_s: float):
    """Path-steps/s of the FP64 C oracle (forward + reverse sweep of the
    throughput configuration) on `threads` OpenMP threads, over a sample of
    about `target_s` seconds: a prefix of the paths, or whole batches of
    successive iterations when one batch takes less than that."""
    from oracle import core as O
    from paper_1910_11623_amd import inputs as I

    O.set_threads(threads)
    prob = I.bsb(D)
    net = dict(kind="mlp", width=W, depth=DEPTH)
    p = I.init_params(prob, net, N, seed=0)
    probe = 64 * threads
    t0 = time.perf_counter()
    O.loss_grad(prob, net, N, probe, p, 73.0, seed=1, it=0)
    per_path = max((time.perf_counter() - t0) / probe, 1e-7)
    ms = int(max(probe, min(M, round(target_s / per_path / 64) * 64)))
    reps = int(max(1, min(16, round(target_s / (per_path * M))))) if ms >= M else 1
    ms = min(ms, M)
    t0 = time.perf_counter()
    for it in range(reps):
        O.loss_grad(prob, net, N, ms, p, 73.0, seed=1, it=it)
    dt = time.perf_counter() - t0
    what = f"{ms} of {M} paths" if reps == 1 else f"all {M} paths, {reps} iterations"
    return reps * ms * N / dt, f"{what} ({dt:.1f} s)"


def cpu_baseline(target_s: float = 10.0):
    """The FP64 C oracle on the host: with OpenMP over path chunks on every
    core this process may use (the reported value), and on one thread."""
    host = _host_cpu()
    v_all, what_all = _oracle_rate(host["threads"], target_s)
    v_one, what_one = _oracle_rate(1, target_s)
    return {"value": round(v_all, 2), "unit": "path-steps/s", "cores": host["threads"], "kind": "oracle",
            "sample": f"forward + reverse sweep at N={N}, d={D}, width {W}x{DEPTH}: {what_all} on "
                      f"{host['threads']} threads; single thread {what_one}",
            "single_thread_value": round(v_one, 2), "host": host}


# ------------------------------------------------------- plain FP32 eager
def eager_model(prob, N_, params_flat, y0, device):
    import torch
    import torch.nn as nn

    d = prob["d"]

    class DeepBSDE(nn.Module):
        def __init__(self):
            super().__init__()
            self.y0 = nn.Parameter(torch.tensor(float(y0), dtype=torch.float32))
            self.z0 = nn.Parameter(torch.tensor(params_flat[:d], dtype=torch.float32))
            self.nets = nn.ModuleList()
            off = d
            for _ in range(1, N_):
                layers = []
                for k, (o, i) in enumerate([(W, d)] + [(W, W)] * (DEPTH - 1) + [(d, W)]):
                    lin = nn.Linear(i, o)
                    lin.weight.data = torch.tensor(params_flat[off:off + o * i].reshape(o, i), dtype=torch.float32)
                    off += o * i
                    lin.bias.data = torch.tensor(params_flat[off:off + o], dtype=torch.float32)
                    off += o
                    layers.append(lin)
                    if k < DEPTH:
                        layers.append(nn.Tanh())
                self.nets.append(nn.Sequential(*layers))
            self.register_buffer("x0", torch.tensor(prob["x0"], dtype=torch.float32))

        def forward(self, paths):
            r, s = prob["drv_p"][0], prob["sde_s"]
            dt = prob["T"] / N_
            X = self.x0.expand(paths, d)
            Y = self.y0.expand(paths)
            for n in range(N_):
                Z = self.z0.expand(paths, d) if n == 0 else self.nets[n - 1](X)
                dW = torch.randn(paths, d, device=X.device) * math.sqrt(dt)
                sdw = s * X * dW
                Y = Y + r * (Y - (Z * X).sum(1)) * dt + (Z * sdw).sum(1)
                X = X + sdw
            return ((Y - (X * X).sum(1)) ** 2).mean()

    return DeepBSDE().to(device)


def eager_prolong(model_c, prob, Nf, device):
    import torch
    params = [model_c.z0.detach().cpu().numpy()]
    Nc = len(model_c.nets) + 1
    for j in range(1, Nf):
        c = min(max(j // 2, 1), Nc - 1)
        for lyr in model_c.nets[c - 1]:
            if hasattr(lyr, "weight"):
                params.append(lyr.weight.detach().cpu().numpy().ravel())
                params.append(lyr.bias.detach().cpu().numpy())
    flat = np.concatenate(params)
    return eager_model(prob, Nf, flat, float(model_c.y0.item()), device)


def eager_run(levels, iters, y0_init, check_every=100, target=None, max_seconds=90.0, lr_y0=1e-2):
    """Plain FP32 eager training with the same schedule as the library's
    legs; stops once Y0 has held within 1% for 100 finest-level iterations.
    Returns (ms/step at the finest level, seconds to 1%, final Y0,
    iteration index of the first accurate iteration)."""
    import torch
    from paper_1910_11623_amd import inputs as I

    torch.backends.cuda.matmul.allow_tf32 = False
    torch.backends.cudnn.allow_tf32 = False
    prob = I.bsb(D)
    p0 = I.init_params(prob, dict(kind="mlp", width=W, depth=DEPTH), levels[0], seed=0)
    torch.manual_seed(1)
    model = eager_model(prob, levels[0], p0, y0_init, "cuda")
    # untimed warmup on a copy
    wm = eager_model(prob, levels[0], p0, y0_init, "cuda")
    wopt = torch.optim.Adam(wm.parameters(), lr=1e-3)
    for _ in range(3):
        wopt.zero_grad(set_to_none=True)
        wm(M).backward()
        wopt.step()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ys, ts, Ns = [], [], []
    ms_fine = None
    for li, Nl in enumerate(levels):
        if li > 0:
            model = eager_prolong(model, prob, Nl, "cuda")
        opt = torch.optim.Adam([{"params": [model.y0], "lr": lr_y0},
                                {"params": [p for n_, p in model.named_parameters() if n_ != "y0"], "lr": 1e-3}])
        ylog = torch.empty(iters[li], device="cuda")
        lv_t0 = time.perf_counter()
        done = 0
        for k in range(iters[li]):
            opt.zero_grad(set_to_none=True)
            model(M).backward()
            opt.step()
            ylog[k] = model.y0.detach()
            done = k + 1
            if (k + 1) % check_every == 0:
                torch.cuda.synchronize()
                if time.perf_counter() - t_start > max_seconds:
                    break
                if Nl == levels[-1] and target is not None:
                    yk = ylog[:done].cpu().numpy()
                    if _tta(yk, np.arange(done, dtype=np.float64), np.full(done, Nl), target, Nl) is not None:
                        break
        torch.cuda.synchronize()
        lv_dt = time.perf_counter() - lv_t0
        t_prev = ts[-1][-1] if ts else 0.0
        ys.append(ylog[:done].cpu().numpy())
        ts.append(t_prev + lv_dt * np.arange(1, done + 1) / done)
        Ns.append(np.full(done, Nl))
        if Nl == levels[-1]:
            ms_fine = lv_dt / done * 1e3
        if time.perf_counter() - t_start > max_seconds:
            break
    y, t, Nn = np.concatenate(ys), np.concatenate(ts), np.concatenate(Ns)
    i = _tta(y, np.arange(len(y), dtype=np.float64), Nn, target, levels[-1])
    tta = None if i is None else float(t[int(i)])
    return ms_fine, tta, float(y[-1]) if len(y) else None, None if i is None else int(i)


def _tta(y, t, Nn, target, finest, rel=0.01, hold=100):
    ok = (np.abs(y / target - 1.0) <= rel) & (Nn == finest)
    for i in range(len(ok) - hold + 1):
        if ok[i:i + hold].all():
            return float(t[i])
    return None


LR_Y0_TTA = 0.1     # y0's Adam rate in the time-to-accuracy legs (networks: 1e-3)
SINGLE = ([32], [3000])
MULTI = ([4, 8, 16, 32], [600, 600, 600, 1500])
MULTI_SWITCH = ([4, 8, 16, 32], [1500, 1500, 1500, 1500])
SWITCH_REL = 1e-3


def tta_library(prec, levels, iters, y0_init, target, switch_rel=None):
    """One training run of the library through a schedule: seconds and
    iterations until Y0 holds within 1% of the target on the finest level."""
    from paper_1910_11623_amd import inputs as I
    from paper_1910_11623_amd.train import first_accurate_iteration, multilevel_schedule, train

    prob = I.bsb(D)
    net = dict(kind="mlp", width=W, depth=DEPTH, prec=prec)
    h = train(prob, net, M, multilevel_schedule(levels, iters), lr=1e-3, lr_y0=LR_Y0_TTA, seed=1, init_seed=0,
              y0_init=y0_init, warmup=5, switch_rel=switch_rel)
    i = first_accurate_iteration(h, target)
    return {"seconds": None if i is None else round(float(h.t[i]), 4),
            "iterations": i, "level_iters": h.level_iters,
            "level_seconds": [round(t, 4) for t in h.level_seconds],
            "y0_final": round(h.y0_final, 4), "run_seconds": round(float(h.t[-1]), 4)}


def tta_legs(target: float, eager: bool = True) -> dict:
    """Time to Y0 within 1% of the closed form (held for 100 iterations on
    the N = 32 grid), from y0 = 73: the library in fp32 and bf16, single
    level, multilevel with fixed per-level budgets and multilevel with the
    early switch; the plain FP32 PyTorch-eager form single level and
    multilevel with the fixed budgets."""
    y0_init = 73.0
    out = {"target_y0": target, "y0_start": y0_init, "lr": 1e-3, "lr_y0": LR_Y0_TTA,
           "single_level": {"levels": SINGLE[0], "iters": SINGLE[1]},
           "multilevel": {"levels": MULTI[0], "iters": MULTI[1]},
           "multilevel_early_switch": {"levels": MULTI_SWITCH[0], "max_iters": MULTI_SWITCH[1],
                                       "switch_rel": SWITCH_REL, "window": 100}}
    for prec in ("fp32", "bf16"):
        r = {"single_level": tta_library(prec, *SINGLE, y0_init, target),
             "multilevel": tta_library(prec, *MULTI, y0_init, target),
             "multilevel_early_switch": tta_library(prec, *MULTI_SWITCH, y0_init, target, switch_rel=SWITCH_REL)}
        out[f"library_{prec}"] = r
        log(f"time to 1% ({prec}): " + ", ".join(f"{k} {v['seconds']} s / {v['iterations']} it" for k, v in r.items()))
    if eager:
        e_single = eager_run(*SINGLE, y0_init, target=target, lr_y0=LR_Y0_TTA)
        e_multi = eager_run(*MULTI, y0_init, target=target, lr_y0=LR_Y0_TTA)
        out["eager_fp32"] = {
            "ms_per_step": None if e_single[0] is None else round(e_single[0], 4),
            "single_level": {"seconds": e_single[1], "iterations": e_single[3], "y0_final": e_single[2]},
            "multilevel": {"seconds": e_multi[1], "iterations": e_multi[3], "y0_final": e_multi[2]}}
        log(f"eager: {e_single[0]} ms/step, time to 1% single {e_single[1]} s, multilevel {e_multi[1]} s")
    return out


# ----------------------------------------- the paper's own formulation
PAPER_D, PAPER_W, PAPER_K, PAPER_N, PAPER_M = 100, 256, 3, 50, 100


def unet_flops_per_row(d: int, w: int, K: int) -> int:
    """Algorithmic flops of one row (one path at one grid point) of a
    training step of the u-network: per block product (w x w) the forward,
    the input-gradient sweep, the second-order sweep, the reverse sweep and
    two weight-gradient terms (12 w^2); the input layer (d x w) the same
    minus the reverse product into x (10 d w); the output dot products."""
    return 12 * K * w * w + 10 * d * w + 4 * w


def eager_unet_step_ms(N_: int, M_: int, steps: int = 20, warmup: int = 3) -> float:
    """Plain FP32 PyTorch-eager form of the same formulation (Z by autograd
    with create_graph, residual loss, double backward, torch Adam)."""
    import torch
    from paper_1910_11623_amd import inputs as I

    torch.backends.cuda.matmul.allow_tf32 = False
    prob = I.bsb(PAPER_D)
    d, w, K = PAPER_D, PAPER_W, PAPER_K
    layers = [torch.nn.Linear(d + 1, w)] + [torch.nn.Linear(w, w) for _ in range(K)] + [torch.nn.Linear(w, 1)]
    net = torch.nn.ModuleList(layers).cuda()
    opt = torch.optim.Adam(net.parameters(), lr=1e-3)
    r, s_ = prob["drv_p"][0], prob["sde_s"]
    dt = prob["T"] / N_
    x0 = torch.tensor(prob["x0"], dtype=torch.float32, device="cuda")
    t = (torch.arange(N_ + 1, device="cuda", dtype=torch.float32) * dt).repeat_interleave(M_)[:, None]

    def step():
        dW = torch.randn(N_, M_, d, device="cuda") * math.sqrt(dt)
        X = [x0.expand(M_, d)]
        for n in range(N_):
            X.append(X[-1] * (1 + s_ * dW[n]))
        Xa = torch.cat(X, 0).requires_grad_(True)
        h = torch.cat([Xa, t], 1)
        for k, lin in enumerate(net):
            h = lin(h)
            if k < len(net) - 1:
                h = torch.tanh(h)
        u = h[:, 0]
        (Z,) = torch.autograd.grad(u.sum(), Xa, create_graph=True)
        U, Zr, Xr = u.view(N_ + 1, M_), Z.view(N_ + 1, M_, d), Xa.view(N_ + 1, M_, d)
        S = s_ * Xr[:-1] * dW
        phi = r * (U[:-1] - (Zr[:-1] * Xr[:-1]).sum(2))
        res = U[1:] - U[:-1] - phi * dt - (Zr[:-1] * S).sum(2)
        L = ((res ** 2).sum() + ((U[-1] - (Xr[-1] ** 2).sum(1)) ** 2).sum()) / M_
        opt.zero_grad(set_to_none=True)
        L.backward()
        opt.step()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


TTA_U_ITERS = 12000


def paper_leg(steps: int = 100, tta: bool = True, archs=("u_fc", "u_res", "u_nais")):
    """The paper's own formulation (Sec. 2.2 eq. (loss), Sec. 4.1 set-up):
    BSB d = 100, one u-network with four fully connected tanh layers of
    width 256 (input layer + 3 blocks), Z = grad u, residual loss, fp32.
    Training steps at the paper's M = 100, N = 50 and at M = 4096, N = 32;
    time until u(0, x0) holds within 1% of the closed form, single level
    (N = 32) against the multilevel schedule 2 -> 4 -> 8 -> 16 -> 32 of
    Sec. 3.2; the plain FP32 PyTorch-eager form of the same method."""
    import torch
    from paper_1910_11623_amd import inputs as I
    from paper_1910_11623_amd.plan import UPlan
    from paper_1910_11623_amd.train import first_accurate_mean_iteration, multilevel_schedule, train_unet

    prob = I.bsb(PAPER_D)
    net = dict(kind="u_fc", width=PAPER_W, depth=PAPER_K)
    out = {"network": f"u-network, {PAPER_K + 1} fully connected tanh layers x {PAPER_W}, fp32",
           "flops_per_row": unet_flops_per_row(PAPER_D, PAPER_W, PAPER_K)}
    for (Nn, Mm) in ((PAPER_N, PAPER_M), (32, 4096)):
        plan = UPlan(prob, net, Nn, Mm)
        p = torch.from_numpy(I.init_unet_params(prob, dict(arch="fc", width=PAPER_W, depth=PAPER_K),
                                                seed=0).astype(np.float32)).cuda()
        m, v = torch.zeros_like(p), torch.zeros_like(p)
        o = (torch.empty((), dtype=torch.float64, device="cuda"), torch.empty_like(p),
             torch.empty((), dtype=torch.float64, device="cuda"))

        def step(k):
            plan.forward_backward(p, 1, k, out=o)
            plan.adam_step(p, o[1], m, v, k + 1)
        for k in range(5):
            step(k)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record()
        for k in range(steps):
            step(5 + k)
            ev[k + 1].record()
        torch.cuda.synchronize()
        q = _quantiles([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
        ms = q["median"]
        rows = (Nn + 1) * Mm
        tf = out["flops_per_row"] * rows / (ms * 1e-3) / 1e12
        out[f"M{Mm}_N{Nn}"] = {"step_ms": q, "path_steps_per_s": round(Mm * Nn / (ms * 1e-3), 1),
                               "tflops": round(tf, 2), "frac_fp32_peak": round(tf / PEAK_FP32_MFMA, 4),
                               "finite": bool(torch.isfinite(o[0]).item())}
        log(f"paper formulation M={Mm} N={Nn}: {ms:.4f} ms/step, {tf:.1f} TFLOP/s")
    try:
        out["eager_fp32_M100_N50_ms_per_step"] = round(eager_unet_step_ms(PAPER_N, PAPER_M), 4)
    except Exception as e:  # the comparator is context; the leg keeps its own numbers
        out["eager_fp32_M100_N50_ms_per_step"] = f"failed: {e}"
    if tta:
        target = bsb_closed_form_y0(PAPER_D)
        res = {}
        for kind in archs:
            k_net = dict(kind=kind, width=PAPER_W, depth=PAPER_K)
            for name, sched, sw in (("single_level", multilevel_schedule([32], [TTA_U_ITERS]), None),
                                    ("multilevel_early_switch",
                                     multilevel_schedule([2, 4, 8, 16, 32], [4000] * 4 + [TTA_U_ITERS]), SWITCH_REL)):
                h = train_unet(prob, k_net, PAPER_M, sched, lr=1e-3, seed=1, init_seed=0, warmup=3, switch_rel=sw)
                i = first_accurate_mean_iteration(h, target)
                fin = h.y0[h.N == 32][-1000:]
                res[f"{kind}_{name}"] = {
                    "seconds": None if i is None else round(float(h.t[i]), 4), "iterations": i,
                    "level_iters": h.level_iters, "y0_mean_last1000": round(float(np.mean(fin)), 4),
                    "y0_rel_err_last1000": round(float(abs(np.mean(fin) / target - 1.0)), 5),
                    "y0_std_last1000": round(float(np.std(fin)), 4),
                    "loss_mean_last1000": round(float(np.mean(h.loss[h.N == 32][-1000:])), 4),
                    "run_seconds": round(float(h.t[-1]), 3)}
                log(f"paper formulation {kind} {name}: {res[f'{kind}_{name}']}")
        out["time_to_1pct"] = dict(res, target_y0=round(target, 4), M=PAPER_M, lr=1e-3,
                                   criterion="first finest-level iteration whose trailing 100-iteration mean of "
                                             "u(0, x0) is within 1% of the closed form and stays so for 500 more")
    return out


def generalisation_leg(iters: int = 8000, deltas=(0.0, 0.05, 0.1, 0.2, 0.4), N_: int = 32, M_: int = 100,
                       n_dirs: int = 4):
    """Sec. 4 generalisation experiment: u-networks of the three block types
    (fully connected, residual, NAIS), trained at x0 with the same budget,
    evaluated without re-optimisation on paths from perturbed initial
    conditions x0 + delta |x0| e (e a random unit direction): the mean over
    paths and grid points of |u(t_n, X_n) - u*(t_n, X_n)| / u*(t_n, X_n)
    against the closed form u* = exp((r + sigma^2)(T - t)) |x|^2."""
    import torch
    from paper_1910_11623_amd import inputs as I
    from paper_1910_11623_amd.plan import UPlan
    from paper_1910_11623_amd.train import multilevel_schedule, train_unet

    prob = I.bsb(PAPER_D)
    r, sg, T = prob["drv_p"][0], prob["sde_s"], prob["T"]
    x0 = np.asarray(prob["x0"], dtype=np.float64)
    rng = np.random.default_rng(11)
    dirs = rng.standard_normal((n_dirs, PAPER_D))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    out = {"iters": iters, "N": N_, "M": M_, "deltas": list(deltas), "width": PAPER_W, "blocks": PAPER_K}
    for kind in ("u_fc", "u_res", "u_nais"):
        net = dict(kind=kind, width=PAPER_W, depth=PAPER_K)
        t0 = time.perf_counter()
        h = train_unet(prob, net, M_, multilevel_schedule([N_], [iters]), lr=1e-3, seed=1, init_seed=0)
        train_s = time.perf_counter() - t0
        ev = UPlan(prob, net, N_, M_)
        errs = []
        for delta in deltas:
            e_d = []
            for k in range(n_dirs if delta > 0 else 1):
                xs = x0 + delta * np.linalg.norm(x0) * dirs[k]
                ev.set_x0(xs)
                ev.forward_backward(h.params, 7, 1000 + k, grad=False)
                u, _ = ev.states()
                torch.cuda.synchronize()
                u = u.cpu().numpy().astype(np.float64).reshape(N_ + 1, M_)
                # the paths of the evaluation, for the closed form
                xi = ev.sample_normals(7, 1000 + k).cpu().numpy().astype(np.float64)
                X = np.broadcast_to(xs, (M_, PAPER_D)).copy()
                rel = []
                for n in range(N_ + 1):
                    us = math.exp((r + sg * sg) * (T - n * T / N_)) * (X * X).sum(1)
                    rel.append(np.abs(u[n] - us) / us)
                    if n < N_:
                        X = X * (1.0 + sg * math.sqrt(T / N_) * xi[n])
                e_d.append(float(np.mean(rel)))
            errs.append(round(float(np.mean(e_d)), 5))
        out[kind] = {"mean_rel_error": errs, "train_seconds": round(train_s, 2),
                     "y0_final": round(h.y0_final, 4), "loss_final": float(h.loss[-1])}
        log(f"generalisation {kind}: {errs}")
    return out


def batch_leg(steps: int = 20):
    """32 Allen–Cahn instances (d uniform on 20..200, N in {10, 20, 40},
    M = 8192, width d + 10, bf16): one training step of every instance per
    step, eager (separate calls) vs one graph launch, untuned vs autotuned."""
    import torch
    from paper_1910_11623_amd import inputs as I
    from paper_1910_11623_amd.plan import Batch, Plan, TrainState

    shapes = I.allen_cahn_batch(32, 2019)
    Mb = 8192
    LR_AC = 1e-4  # the untrained cubic driver diverges on extreme paths at 1e-3
    states, seeds, init = [], [], []
    for k, (d, Nk) in enumerate(shapes):
        prob = I.allen_cahn(d)
        net = dict(kind="mlp", width=d + 10, depth=2, prec="bf16")
        plan = Plan(prob, net, Nk, Mb)
        p = I.init_params(prob, net, Nk, seed=k, out_scale=0.05)
        y0 = float(plan.terminal_mean(0x5A5A + k, 0).item())
        states.append(TrainState(plan, p, y0))
        init.append((states[-1].params.clone(), y0))
        seeds.append(1 + k)
    work = sum(Mb * Nk for _, Nk in shapes)

    def reset():
        # every phase trains from the same initial state with Adam's step
        # count starting at 1, so the three phases do identical work
        for s, (p, y0) in zip(states, init):
            s.params.copy_(p)
            s.y0.fill_(y0)
            for t in (s.m, s.v, s.my0, s.vy0):
                t.zero_()

    def timed(fn, n):
        reset()
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    it = [0]

    def eager():
        for s, seed in zip(states, seeds):
            s.fused_step(seed, it[0], lr=LR_AC)
        it[0] += 1

    def all_finite():
        # every loss and gradient of the phase (the plans' device-side checks), then the state
        torch.cuda.synchronize()
        flags = [s.plan.finite_since_last_check() for s in states]
        return all(flags) and all(bool(torch.isfinite(s.loss).item() and torch.isfinite(s.y0).item())
                                  for s in states)

    ms_eager = timed(eager, steps)
    finite = all_finite()
    reset()
    b = Batch(states, seeds, lr=LR_AC)
    ms_graph = timed(b.step, steps)
    finite = all_finite() and finite
    del b
    reset()
    bt = Batch(states, seeds, lr=LR_AC, autotune=True)  # tunes on the initial state
    all_finite()  # the tuner's own calls are not part of the measurement
    ms_tuned = timed(bt.step, steps)
    cfgs = [s.plan.get_config() for s in states]
    finite = all_finite() and finite
    del bt
    return {"instances": len(shapes), "paths": Mb, "shapes_d_N": shapes, "prec": "bf16",
            "path_steps_per_step": work,
            "eager_ms": round(ms_eager, 4), "graph_ms": round(ms_graph, 4), "graph_tuned_ms": round(ms_tuned, 4),
            "graph_tuned_path_steps_per_s": round(work / (ms_tuned * 1e-3), 1),
            "eager_path_steps_per_s": round(work / (ms_eager * 1e-3), 1),
            "tuned_shapes": sorted({(c["ti"], c["tw"], c["lds"], c["splits"]) for c in cfgs}),
            "finite": finite}


def hjb_leg(steps: int = 20):
    """HJB d=100, N=20, M=65536, width 110x2: ms per training step, fp32 and bf16."""
    import torch
    from paper_1910_11623_amd import inputs as I
    from paper_1910_11623_amd.plan import Plan, TrainState

    out = {}
    for prec in ("fp32", "bf16"):
        prob = I.hjb(100)
        net = dict(kind="mlp", width=110, depth=2, prec=prec)
        plan = Plan(prob, net, 20, 65536)
        s = TrainState(plan, I.init_params(prob, net, 20, seed=0), 4.6)
        for k in range(3):
            s.fused_step(1, k)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(steps):
            s.fused_step(1, 3 + k)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[prec] = {"ms_per_step": round(ms, 4), "path_steps_per_s": round(65536 * 20 / (ms * 1e-3), 1)}
    return out


def mlp_checkpoint_leg(steps: int = 20, chunk_steps: int = 8):
    """HJB d=100, N=20, M=65536, width 110x2, fp32 and bf16: training steps
    with activation checkpointing (chunks of `chunk_steps` steps, recomputed
    in the reverse pass) against every step's activations kept: ms per step,
    workspace, and whether the trained parameters are the same bits."""
    import torch
    from paper_1910_11623_amd import inputs as I
    from paper_1910_11623_amd.plan import Plan, TrainState

    N, Mh = 20, 65536
    out = {"chunk_steps": chunk_steps}
    for prec in ("fp32", "bf16"):
        prob = I.hjb(100)
        net = dict(kind="mlp", width=110, depth=2, prec=prec)
        res = {}
        for ck in (False, True):
            plan = Plan(prob, net, N, Mh, recompute=ck, chunk_rows=chunk_steps * Mh if ck else 0)
            s = TrainState(plan, I.init_params(prob, net, N, seed=0), 4.6)
            for k in range(3):
                s.fused_step(1, k)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for k in range(steps):
                s.fused_step(1, 3 + k)
            e1.record()
            torch.cuda.synchronize()
            res[ck] = (e0.elapsed_time(e1) / steps, plan.ws_bytes / 2**30, s.params.clone())
            del plan, s
        out[prec] = {"kept_ms_per_step": round(res[False][0], 4), "kept_workspace_gib": round(res[False][1], 3),
                     "checkpointed_ms_per_step": round(res[True][0], 4),
                     "checkpointed_workspace_gib": round(res[True][1], 3),
                     "same_bits": bool(torch.equal(res[False][2], res[True][2]))}
    return out


def resnet_leg(steps: int = 3, recompute: bool = True):
    """BSB d=1000, N=64, M=16384, shared residual network (width 1024,
    4 blocks, t as input), bf16 MFMA; the reverse sweep recomputes each row
    chunk's activations (checkpointing) or reads the ones the forward pass
    kept: ms per training step and MFMA TFLOP/s of the forward and reverse
    phases (the recompute's flops count only when it runs)."""
    import torch
    from paper_1910_11623_amd import inputs as I
    from paper_1910_11623_amd.plan import Plan, TrainState

    d, w, B, Nr, Mr = 1000, 1024, 4, 64, 16384
    prob = I.bsb(d)
    net = dict(kind="resnet", width=w, depth=B, prec="bf16")
    plan = Plan(prob, net, Nr, Mr, recompute=recompute)
    s = TrainState(plan, I.init_params(prob, net, Nr, seed=0, out_scale=0.1), 760.0)
    s.fused_step(1, 0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        s.fused_step(1, 1 + k)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    plan.profile(True)
    for k in range(steps):
        s.fused_step(1, 10 + k)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    rows = Nr * Mr
    fwd_flops = 2.0 * (w * d + B * w * w + d * w) * rows
    recompute_flops = 2.0 * (w * d + B * w * w) * rows if recompute else 0.0
    bwd_flops = recompute_flops + (2.0 * w * d + 2.0 * B * w * w +
                                   2.0 * (d * (w + 1) + B * w * (w + 1) + w * (d + 2))) * rows
    t_f = prof["forward"][0] / max(prof["forward"][1], 1) * 1e-3
    t_b = prof["backward"][0] / max(prof["backward"][1], 1) * 1e-3
    return {"recompute": bool(recompute), "workspace_gib": round(plan.ws_bytes / 2**30, 2),
            "ms_per_step": round(ms, 3), "path_steps_per_s": round(rows / (ms * 1e-3), 1),
            "step_mfma_tflops": round((fwd_flops + bwd_flops) / (ms * 1e-3) / 1e12, 1),
            "forward_ms": round(t_f * 1e3, 3), "backward_ms": round(t_b * 1e3, 3),
            "forward_tflops": round(fwd_flops / t_f / 1e12, 1), "backward_tflops": round(bwd_flops / t_b / 1e12, 1),
            "bf16_peak_tflops": PEAK_BF16_MFMA,
            "finite": bool(torch.isfinite(s.loss).item())}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tta", action="store_true", help="skip the time-to-accuracy legs")
    ap.add_argument("--no-eager", action="store_true", help="skip the PyTorch-eager comparator")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched Allen-Cahn and HJB legs")
    ap.add_argument("--prec", choices=["fp32", "bf16", "both"], default="both",
                    help="which library precision(s) to time")
    ap.add_argument("--only", choices=["batch", "hjb", "mlp_checkpoint", "resnet", "resnet_kept",
                                       "resnet_multilevel", "paper", "generalisation"],
                    help="run just one of the extra legs and print its JSON")
    ap.add_argument("--summarize-traffic", nargs=6, metavar="DIR",
                    help="rocprofv3 --pmc output dirs: FETCH_SIZE fp32, WRITE_SIZE fp32, FETCH_SIZE bf16, "
                         "WRITE_SIZE bf16, FETCH_SIZE and WRITE_SIZE of --copy-calibration; writes "
                         "profiles/bsb_d100_traffic.json")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.summarize_traffic:
        rec = summarize_traffic(*args.summarize_traffic)
        with open(os.path.join(ROOT, "profiles", "bsb_d100_traffic.json"), "w") as fo:
            json.dump(rec, fo, indent=1)
        print(json.dumps(rec["per_launch"]), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only; there is no multi-GPU path in this library.", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log(f"device {torch.cuda.get_device_name(0)}")
    if args.copy_calibration:
        n = (1 << 30) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}), flush=True)
        return
    if args.only:
        leg = {"batch": batch_leg, "hjb": hjb_leg, "resnet": resnet_leg,
               "resnet_kept": lambda: resnet_leg(recompute=False),
               "resnet_multilevel": resnet_multilevel_leg, "paper": lambda: paper_leg(tta=not args.no_tta),
               "generalisation": generalisation_leg, "mlp_checkpoint": mlp_checkpoint_leg}[args.only]
        print(json.dumps({args.only: leg()}), flush=True)
        return
    if args.prec == "bf16":
        ms_bf, st_bf, kern_bf, _ = time_library("bf16", args.steps, args.warmup)
        log(f"bf16 only: {ms_bf:.4f} ms/step {st_bf}; kernels " + ", ".join(f"{k}={v:.4f}" for k, v in kern_bf.items()))
        return
    ms, stats, kern, finite = time_library("fp32", args.steps, args.warmup)
    value = M * N / (ms * 1e-3)
    log(f"fp32: {ms:.4f} ms/step ({stats}), {value:.4e} path-steps/s; kernels (ms/launch) "
        + ", ".join(f"{k}={v:.4f}" for k, v in kern.items()))
    dom, roof = roofline_entry("fp32", kern)
    log(f"dominant kernel {dom}: {roof['achieved']} TFLOP/s of {roof['peak']}")
    if args.prec == "fp32":
        print(json.dumps({"ms_per_step": ms, "step_ms": stats, "kernels_ms_per_launch": kern, "roofline": roof,
                          "roofline_kernel": dom}), flush=True)
        return
    ms_bf, stats_bf, kern_bf, _ = time_library("bf16", args.steps, args.warmup)
    dom_bf, roof_bf = roofline_entry("bf16", kern_bf)
    log(f"bf16: {ms_bf:.4f} ms/step ({stats_bf}); dominant {dom_bf} {roof_bf['achieved']} {roof_bf['unit']} "
        f"({100 * roof_bf['frac']:.1f}% of the bf16 matrix peak)")

    target = bsb_closed_form_y0(D)
    tta = tta_legs(target, eager=not args.no_eager) if not args.no_tta else None

    extra = {}
    if not args.no_extra:
        extra["batched_allen_cahn_32"] = batch_leg()
        log(f"batched AC x32: eager {extra['batched_allen_cahn_32']['eager_ms']} ms, graph "
            f"{extra['batched_allen_cahn_32']['graph_ms']} ms, tuned graph {extra['batched_allen_cahn_32']['graph_tuned_ms']} ms")
        extra["hjb_d100_M65536"] = hjb_leg()
        log(f"HJB d=100 M=65536: {extra['hjb_d100_M65536']}")
        extra["mlp_checkpoint_hjb_d100"] = mlp_checkpoint_leg()
        log(f"per-step MLP checkpointing, HJB d=100 M=65536: {extra['mlp_checkpoint_hjb_d100']}")
        extra["resnet_bsb_d1000"] = resnet_leg(recompute=True)
        log(f"ResNet BSB d=1000 (recompute): {extra['resnet_bsb_d1000']}")
        extra["resnet_bsb_d1000_kept"] = resnet_leg(recompute=False)
        log(f"ResNet BSB d=1000 (activations kept): {extra['resnet_bsb_d1000_kept']}")
        extra["paper_formulation_bsb_d100"] = paper_leg(tta=not args.no_tta)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline()
        log(f"cpu oracle: {cpu['value']} path-steps/s ({cpu['sample']})")

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "path-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"Black-Scholes-Barenblatt d={D} T=1 N={N} M={M}, per-step MLP "
                               f"{W}x{DEPTH} tanh, fp32, Adam; one step = fwd + reverse sweep + Adam",
                   "global_batch": M, "seq_len": N, "parallelism": "none"},
        "roofline": roof,
        "roofline_kernel": f"k_{dom}<fp32>",
        "cpu_baseline": cpu,
        "step_ms": stats,
        "step_roofline": step_roofline("fp32", ms),
        "kernels_ms_per_launch": {k: round(v, 5) for k, v in kern.items()},
        "finite": finite,
        "bf16": {"ms_per_step": round(ms_bf, 5), "value": round(M * N / (ms_bf * 1e-3), 1),
                 "step_ms": stats_bf, "step_roofline": step_roofline("bf16", ms_bf),
                 "roofline": roof_bf, "roofline_kernel": f"k_{dom_bf}<bf16>",
                 "kernels_ms_per_launch": {k: round(v, 5) for k, v in kern_bf.items()}},
        "time_to_1pct": tta,
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
