"""Plan objects over the C ABI, with torch tensors as device memory.

``Plan`` owns one fbsde_plan and one workspace tensor; every method is one
call into libfbsde.so on torch's current HIP stream.  ``FBSDELoss`` exposes
the fused forward + hand-written reverse sweep as a torch.autograd.Function.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import binding as B


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Plan:
    """One (problem, network, N, M) configuration of the hot path."""

    def __init__(self, problem: dict, net: dict, N: int, M: int, device: str | torch.device = "cuda",
                 recompute: bool | None = None, chunk_rows: int = 0):
        """Activation checkpointing (fbsde_plan_set_checkpointing).  Shared
        residual network: `recompute` (default True) recomputes each chunk's
        activations in the reverse sweep, False keeps them all (larger
        workspace).  Per-step MLP: `recompute` (default False) True keeps one
        chunk's activations and recomputes the rest (same bits).
        `chunk_rows` sets the rows per chunk of whole steps (0: the
        library's default)."""
        self.lib = B.load()
        self.problem, self.net, self.N, self.M = problem, dict(net), int(N), int(M)
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        with torch.cuda.device(self.device):
            ps, keep = B.make_problem(problem)
            ns = B.make_net(self.net)
            h = C.c_void_p()
            B.check(self.lib.fbsde_plan_create(C.byref(ps), C.byref(ns), self.N, self.M, C.byref(h)))
            self._h = h
            del keep
            n = C.c_int64()
            B.check(self.lib.fbsde_param_count(self._h, C.byref(n)))
            self.n_params = int(n.value)
            kind = self.net.get("kind")
            self.recompute = (recompute is None or bool(recompute)) if kind == "resnet" else bool(recompute)
            if kind == "resnet" or (kind == "mlp" and self.recompute):
                B.check(self.lib.fbsde_plan_set_checkpointing(self._h, int(self.recompute), int(chunk_rows)))
            sz = C.c_size_t()
            B.check(self.lib.fbsde_workspace_size(self._h, C.byref(sz)))
            self.ws_bytes = int(sz.value)
            # +256 so that the workspace can be aligned to 256 bytes
            self._ws_raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self._ws_raw.data_ptr()) % 256
            self.ws = self._ws_raw[off:off + self.ws_bytes]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                self.lib.fbsde_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    # ---------------------------------------------------------------- calls
    def param_layout(self) -> list:
        """[(offset, rows, cols)] of every block of the flat parameter layout
        (z0, then W and b of every dense layer), from fbsde_param_layout."""
        nb = C.c_int64()
        B.check(self.lib.fbsde_param_layout(self._h, None, C.byref(nb), None, None))
        offs = (C.c_int64 * (nb.value + 1))()
        shp = (C.c_int32 * (2 * nb.value))()
        B.check(self.lib.fbsde_param_layout(self._h, None, None, offs, shp))
        return [(int(offs[k]), int(shp[2 * k]), int(shp[2 * k + 1])) for k in range(nb.value)]

    def _check_params(self, params: torch.Tensor):
        if params.dtype != torch.float32 or params.numel() != self.n_params or not params.is_contiguous():
            raise ValueError(f"params must be a contiguous fp32 tensor of {self.n_params} elements")
        if params.device != self.device:
            raise ValueError("params must live on the plan's device")

    def forward(self, params: torch.Tensor, y0: torch.Tensor, seed: int, it: int,
                loss: torch.Tensor | None = None) -> torch.Tensor:
        self._check_params(params)
        if loss is None:
            loss = torch.empty((), dtype=torch.float64, device=self.device)
        B.check(self.lib.fbsde_forward(self._h, _ptr(params), _ptr(y0), seed, it, _ptr(loss),
                                       _ptr(self.ws), _stream()))
        return loss

    def forward_backward(self, params: torch.Tensor, y0: torch.Tensor, seed: int, it: int,
                         out: tuple | None = None):
        """Returns (loss fp64 scalar, grad fp32 [n_params], grad_y0 fp64 scalar)."""
        self._check_params(params)
        if out is None:
            loss = torch.empty((), dtype=torch.float64, device=self.device)
            grad = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
            gy0 = torch.empty((), dtype=torch.float64, device=self.device)
        else:
            loss, grad, gy0 = out
        B.check(self.lib.fbsde_forward_backward(self._h, _ptr(params), _ptr(y0), _ptr(grad), _ptr(gy0),
                                                _ptr(loss), seed, it, _ptr(self.ws), _stream()))
        return loss, grad, gy0

    def adam_step(self, params, y0, grad, gy0, m, v, my0, vy0, t: int, lr: float = 1e-3,
                  lr_y0: float | None = None, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        B.check(self.lib.fbsde_adam_step(self._h, _ptr(params), _ptr(y0), _ptr(grad), _ptr(gy0), _ptr(m),
                                         _ptr(v), _ptr(my0), _ptr(vy0), int(t), float(lr),
                                         float(lr if lr_y0 is None else lr_y0), float(b1), float(b2),
                                         float(eps), _stream()))

    def train_step(self, params, y0, grad, gy0, loss, m, v, my0, vy0, seed: int, it: int, t: int,
                   lr: float = 1e-3, lr_y0: float | None = None, b1: float = 0.9, b2: float = 0.999,
                   eps: float = 1e-8):
        """forward_backward of iteration `it` then adam_step with step count t,
        the reduction and the update in one launch (same bits)."""
        self._check_params(params)
        B.check(self.lib.fbsde_train_step(self._h, _ptr(params), _ptr(y0), _ptr(grad), _ptr(gy0), _ptr(loss),
                                          _ptr(m), _ptr(v), _ptr(my0), _ptr(vy0), int(t), float(lr),
                                          float(lr if lr_y0 is None else lr_y0), float(b1), float(b2),
                                          float(eps), seed, it, _ptr(self.ws), _stream()))

    def prolong_to(self, fine: "Plan", params: torch.Tensor) -> torch.Tensor:
        self._check_params(params)
        out = torch.empty(fine.n_params, dtype=torch.float32, device=self.device)
        B.check(self.lib.fbsde_prolong(self._h, fine._h, _ptr(params), _ptr(out), _stream()))
        return out

    def sample_normals(self, seed: int, it: int) -> torch.Tensor:
        xi = torch.empty((self.N, self.M, int(self.problem["d"])), dtype=torch.float32, device=self.device)
        B.check(self.lib.fbsde_sample_normals(self._h, seed, it, _ptr(xi), _stream()))
        return xi

    def terminal_mean(self, seed: int, it: int) -> torch.Tensor:
        out = torch.empty((), dtype=torch.float64, device=self.device)
        B.check(self.lib.fbsde_terminal_mean(self._h, seed, it, _ptr(out), _ptr(self.ws), _stream()))
        return out

    def terminal_states(self):
        d = int(self.problem["d"])
        xN = torch.empty((self.M, d), dtype=torch.float32, device=self.device)
        yN = torch.empty(self.M, dtype=torch.float32, device=self.device)
        B.check(self.lib.fbsde_terminal_states(self._h, _ptr(self.ws), _ptr(xN), _ptr(yN), _stream()))
        return xN, yN


    def profile(self, enable: bool = True):
        B.check(self.lib.fbsde_profile_enable(self._h, int(bool(enable))))

    def profile_read(self) -> dict:
        """{kernel name: (total ms, launches)} since the previous read."""
        n = len(B.PROF_NAMES)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        B.check(self.lib.fbsde_profile_read(self._h, ms, cnt, n))
        return {B.PROF_NAMES[i]: (float(ms[i]), int(cnt[i])) for i in range(n)}


    # -------------------------------------------------------------- tuning
    def config(self, shape: int = 0, lds=2, tpw: int = 0, splits: int = 0):
        """lds: 0 weights read from global memory, 1 staged in LDS, 2 staged in
        LDS with the fused reverse kernel where it applies (True = 2, False = 0)."""
        mode = (2 if lds else 0) if isinstance(lds, bool) else int(lds)
        B.check(self.lib.fbsde_plan_config(self._h, int(shape), mode, int(tpw), int(splits)))

    def finite_since_last_check(self) -> bool:
        """Whether every loss and gradient since the last report was finite
        (clears the report; synchronise first to cover queued work)."""
        st = self.lib.fbsde_plan_status(self._h)
        if st == B.ERR_NONFINITE:
            return False
        B.check(st)
        return True

    def get_config(self) -> dict:
        c = (C.c_int32 * 6)()
        B.check(self.lib.fbsde_plan_get_config(self._h, c))
        return dict(shape=c[0], ti=c[1], tw=c[2], lds=int(c[3]), tpw=c[4], splits=c[5])

    def autotune(self, params: torch.Tensor, y0: torch.Tensor, reps: int = 3) -> dict:
        self._check_params(params)
        grad = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        gy0 = torch.empty((), dtype=torch.float64, device=self.device)
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        B.check(self.lib.fbsde_plan_autotune(self._h, _ptr(params), _ptr(y0), _ptr(grad), _ptr(gy0),
                                             _ptr(loss), _ptr(self.ws), _stream(), int(reps)))
        return self.get_config()


class UPlan(Plan):
    """The paper's own formulation (one network u(t, x) for every step,
    Z = grad u, per-step residual loss): net = dict(kind="u_fc" | "u_res" |
    "u_nais", width, depth = blocks after the input layer), fp32.  kappa is
    the weight of the terminal-gradient penalty, eps the NAIS shift."""

    def __init__(self, problem: dict, net: dict, N: int, M: int, kappa: float = 0.0, eps: float = 0.01,
                 device: str | torch.device = "cuda"):
        net = dict(net, prec="fp32")
        super().__init__(problem, net, N, M, device=device)
        B.check(self.lib.fbsde_plan_set_unet_loss(self._h, float(kappa), float(eps)))
        self.kappa, self.eps = float(kappa), float(eps)

    def forward_backward(self, params: torch.Tensor, seed: int, it: int, out: tuple | None = None,
                         grad: bool = True):
        """Returns (loss fp64 scalar, grad fp32 [n_params] or None, u(0, x0) fp64 scalar)."""
        self._check_params(params)
        if out is None:
            loss = torch.empty((), dtype=torch.float64, device=self.device)
            g = torch.empty(self.n_params, dtype=torch.float32, device=self.device) if grad else None
            y0 = torch.empty((), dtype=torch.float64, device=self.device)
        else:
            loss, g, y0 = out
        B.check(self.lib.fbsde_unet_forward_backward(self._h, _ptr(params), _ptr(g), _ptr(loss), _ptr(y0),
                                                     seed, it, _ptr(self.ws), _stream()))
        return loss, g, y0

    def adam_step(self, params, grad, m, v, t: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
                  eps: float = 1e-8):
        B.check(self.lib.fbsde_adam_step(self._h, _ptr(params), None, _ptr(grad), None, _ptr(m), _ptr(v), None,
                                         None, int(t), float(lr), float(lr), float(b1), float(b2), float(eps),
                                         _stream()))

    def nais_project(self, params: torch.Tensor, c: float):
        self._check_params(params)
        B.check(self.lib.fbsde_unet_nais_project(self._h, _ptr(params), float(c), _ptr(self.ws), _stream()))

    def states(self):
        """(u [(N+1) M], Z [(N+1) M][d]) of the last call, row n M + m."""
        R = (self.N + 1) * self.M
        u = torch.empty(R, dtype=torch.float32, device=self.device)
        z = torch.empty((R, int(self.problem["d"])), dtype=torch.float32, device=self.device)
        B.check(self.lib.fbsde_unet_states(self._h, _ptr(self.ws), _ptr(u), _ptr(z), _stream()))
        return u, z

    def set_x0(self, x0):
        import ctypes as C_
        arr = (C_.c_double * int(self.problem["d"]))(*[float(v) for v in x0])
        B.check(self.lib.fbsde_plan_set_x0(self._h, arr))


class TrainState:
    """Parameters, y0 and Adam state of one instance, as device tensors."""

    def __init__(self, plan: Plan, params, y0: float):
        dev = plan.device
        self.plan = plan
        self.params = torch.as_tensor(params, dtype=torch.float32).to(dev).contiguous()
        self.y0 = torch.tensor(float(y0), dtype=torch.float64, device=dev)
        self.grad = torch.zeros_like(self.params)
        self.gy0 = torch.zeros((), dtype=torch.float64, device=dev)
        self.loss = torch.zeros((), dtype=torch.float64, device=dev)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.my0 = torch.zeros((), dtype=torch.float64, device=dev)
        self.vy0 = torch.zeros((), dtype=torch.float64, device=dev)

    def eager_step(self, seed: int, it: int, lr=1e-3, lr_y0=1e-2, b1=0.9, b2=0.999, eps=1e-8):
        """The same training step the batch graph runs, as separate calls."""
        self.plan.forward_backward(self.params, self.y0, seed, it, out=(self.loss, self.grad, self.gy0))
        self.plan.adam_step(self.params, self.y0, self.grad, self.gy0, self.m, self.v, self.my0, self.vy0,
                            it + 1, lr=lr, lr_y0=lr_y0, b1=b1, b2=b2, eps=eps)

    def fused_step(self, seed: int, it: int, lr=1e-3, lr_y0=1e-2, b1=0.9, b2=0.999, eps=1e-8):
        """eager_step as one library call (fbsde_train_step): the same bits."""
        self.plan.train_step(self.params, self.y0, self.grad, self.gy0, self.loss, self.m, self.v, self.my0,
                             self.vy0, seed, it, it + 1, lr=lr, lr_y0=lr_y0, b1=b1, b2=b2, eps=eps)


class Batch:
    """Independent instances advanced by one hipGraph launch per step (the
    iteration index lives in a device counter, starting at `it0`)."""

    def __init__(self, states: list, seeds: list, lr=1e-3, lr_y0=1e-2, b1=0.9, b2=0.999, eps=1e-8,
                 autotune: bool = False, it0: int = 0):
        self.lib = B.load()
        self.states = states
        dev = states[0].plan.device
        self.iter = torch.tensor([it0], dtype=torch.int64, device=dev)
        items = (B.BatchItem * len(states))()
        for i, (s, seed) in enumerate(zip(states, seeds)):
            it = items[i]
            it.plan = s.plan._h.value
            it.params_dev, it.y0_dev = s.params.data_ptr(), s.y0.data_ptr()
            it.grad_dev, it.grad_y0_dev, it.loss_dev = s.grad.data_ptr(), s.gy0.data_ptr(), s.loss.data_ptr()
            it.m_dev, it.v_dev = s.m.data_ptr(), s.v.data_ptr()
            it.m_y0_dev, it.v_y0_dev = s.my0.data_ptr(), s.vy0.data_ptr()
            it.ws_dev = s.plan.ws.data_ptr()
            it.seed = int(seed)
        self._items = items
        h = C.c_void_p()
        B.check(self.lib.fbsde_batch_create(items, len(states), lr, lr_y0, b1, b2, eps, self.iter.data_ptr(),
                                            int(bool(autotune)), _stream(), C.byref(h)))
        self._h = h

    def step(self):
        B.check(self.lib.fbsde_batch_step(self._h, _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                self.lib.fbsde_batch_destroy(h)
            except Exception:
                pass
            self._h = None


class FBSDELoss(torch.autograd.Function):
    """loss = FBSDELoss.apply(params, y0, plan, seed, it).

    The forward call runs the fused forward and the hand-written reverse
    sweep at once (the loss and its gradient come from one pass over the
    paths); backward only scales the stored gradient."""

    @staticmethod
    def forward(ctx, params, y0, plan: Plan, seed: int, it: int):
        loss, grad, gy0 = plan.forward_backward(params.detach(), y0.detach(), seed, it)
        ctx.save_for_backward(grad, gy0)
        return loss

    @staticmethod
    def backward(ctx, gout):
        grad, gy0 = ctx.saved_tensors
        return grad * gout.to(grad.dtype), gy0 * gout, None, None, None
