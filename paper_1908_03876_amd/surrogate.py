"""Learned form: a convolutional surrogate of the control-to-state map,
trained on pairs the MRT solver itself generates, proposing warm starts and
line-search steps to the adjoint-based gradient loop (Section 3.2.1), while
every accepted step is verified by a true MRT solve.

The paper's conclusion suggests pairing the method with a reduced-order
model to cut cost further; here that model is a 4-layer periodic 3x3 CNN
(32 channels, BF16 weights, FP32 accumulation) whose forward, backward and
Adam steps run in libmrt.so.  The reactions screen the response of u(T) to
the control within a few nodes, so a 9 x 9 receptive field captures it, the
network is fully convolutional, trains on crops and runs at any lattice
size.  Python here only marshals data, draws seeded random numbers and
combines a handful of scalars.
"""
from __future__ import annotations

import math
import time
from typing import Dict, List, Optional

import numpy as np
import torch

from . import abi
from . import inputs as I
from .batched import Batch
from .solver import DeviceProblem, GradientIteration, Tape

SHAPES = [(32, 1), (32, 32), (32, 32), (1, 32)]  # (cout, cin) per layer


class Surrogate:
    """c -> u(T) - u_base, fields float [B, H, W] on the device."""

    def __init__(self, max_batch: int, max_h: int, max_w: int,
                 in_scale: float = 0.2, out_scale: float = 0.1, seed: int = 0,
                 device="cuda:0"):
        self.device = torch.device(device)
        self.in_scale, self.out_scale = in_scale, out_scale
        self.max_batch, self.max_h, self.max_w = max_batch, max_h, max_w
        self.handle = abi.mrt_srg_create(32, max_batch, max_h, max_w, in_scale, out_scale)
        self.init_params(seed)

    # -- parameters
    def init_params(self, seed: int) -> None:
        rng = np.random.default_rng(seed)
        for layer, (o, c) in enumerate(SHAPES):
            w = rng.normal(0.0, 1.0 / math.sqrt(9 * c), (o, c, 3, 3))
            self.set_param(layer, 0, w)
            self.set_param(layer, 1, np.zeros(o))
        abi.mrt_srg_sync(self.handle)
        torch.cuda.synchronize(self.device)

    def set_param(self, layer: int, kind: int, arr) -> None:
        t = torch.tensor(np.asarray(arr, dtype=np.float32).ravel(), device=self.device)
        abi.mrt_srg_copy_param(self.handle, layer, kind, True, t)
        torch.cuda.current_stream(self.device).synchronize()

    def get_param(self, layer: int, kind: int) -> np.ndarray:
        _, n = abi.mrt_srg_param(self.handle, layer, kind)
        t = torch.empty(n, dtype=torch.float32, device=self.device)
        abi.mrt_srg_copy_param(self.handle, layer, kind, False, t)
        return t.cpu().numpy().astype(np.float64)

    def params(self) -> List[tuple]:
        out = []
        for layer, (o, c) in enumerate(SHAPES):
            out.append((self.get_param(layer, 0).reshape(o, c, 3, 3), self.get_param(layer, 1)))
        return out

    def load(self, params) -> None:
        for layer, (w, b) in enumerate(params):
            self.set_param(layer, 0, w)
            self.set_param(layer, 1, b)
        abi.mrt_srg_sync(self.handle)

    # -- evaluation
    def forward(self, x: torch.Tensor) -> torch.Tensor:
        x = x.contiguous()
        B, H, W = x.shape
        y = torch.empty_like(x)
        abi.mrt_srg_forward(self.handle, x, y, B, H, W)
        return y

    def input_grad(self, x: torch.Tensor, dy: torch.Tensor) -> torch.Tensor:
        """dL/dx for L with dL/dy = dy (runs the forward on x first)."""
        x = x.contiguous()
        B, H, W = x.shape
        y = torch.empty_like(x)
        dx = torch.empty_like(x)
        abi.mrt_srg_forward(self.handle, x, y, B, H, W)
        abi.mrt_srg_backward(self.handle, x, dy.contiguous(), dx, False, B, H, W)
        return dx

    def loss(self, x: torch.Tensor, y: torch.Tensor, border: int = 0,
             sub: Optional[torch.Tensor] = None) -> float:
        """Interior MSE of the surrogate on x against y (minus the field sub
        when given, the same for every sample)."""
        x = x.contiguous()
        B, H, W = x.shape
        if sub is not None:
            assert H == W, "baseline subtraction needs square fields"
            t = torch.empty_like(x)
            idx = torch.arange(B, dtype=torch.int32, device=self.device)
            zero = torch.zeros(B, dtype=torch.int32, device=self.device)
            abi.mrt_srg_gather(y.contiguous(), H, idx, zero, zero, t, B, H, W,
                               sub=sub.contiguous())
            y = t
        return abi.mrt_srg_loss(self.handle, x, y.contiguous(), B, H, W, border)

    # -- use in the optimisation loop
    def objective(self, x: torch.Tensor, u_base, u_target, alpha: float, grad: bool = False):
        """Surrogate costs 1/2 |u_base + S(x_b) - u_t|^2 + alpha/2 |x_b|^2 of
        the fields x_b, and their input gradients when grad is set."""
        x = x.contiguous()
        B, H, W = x.shape
        dx = torch.empty_like(x) if grad else None
        J = abi.mrt_srg_objective(self.handle, x, u_base.contiguous(), u_target.contiguous(),
                                  alpha, B, H, W, want_J=True, dx=dx)
        return (J, dx) if grad else J

    def score_steps(self, c, E, lambdas, u_base, u_target, alpha: float) -> List[float]:
        """Surrogate costs of the controls c - lambda_k E."""
        H, W = c.shape
        return abi.mrt_srg_score_steps(self.handle, c.contiguous(), E.contiguous(), lambdas,
                                       u_base.contiguous(), u_target.contiguous(), alpha, H, W)

    def warm_start(self, u_base, u_target, alpha: float, iters: int = 300, lr: float = 0.05,
                   c0: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Control minimising the surrogate cost (Adam on the control, the
        gradients through the network), from c0 (default 0)."""
        H, W = u_target.shape
        c = torch.zeros((H, W), dtype=torch.float32, device=self.device) if c0 is None \
            else c0.clone().contiguous()
        abi.mrt_srg_warm_start(self.handle, u_base.contiguous(), u_target.contiguous(), alpha,
                               H, W, iters, lr, c)
        return c

    # -- training
    def train(self, controls: torch.Tensor, responses: torch.Tensor, steps: int,
              batch: int = 32, crop: int = 64, border: int = 4, lr: float = 2e-3,
              seed: int = 0, log_every: int = 100,
              u_base: Optional[torch.Tensor] = None) -> List[float]:
        """Adam on random periodic crops of (control, response) pairs, cosine
        learning-rate decay; the targets are the responses minus u_base when
        given.  Returns the logged training losses."""
        n, L, _ = controls.shape
        rng = np.random.default_rng(seed)
        x = torch.empty((batch, crop, crop), dtype=torch.float32, device=self.device)
        y = torch.empty_like(x)
        hist = []
        for s in range(steps):
            idx = torch.tensor(rng.integers(0, n, batch), dtype=torch.int32, device=self.device)
            oy = torch.tensor(rng.integers(0, L, batch), dtype=torch.int32, device=self.device)
            ox = torch.tensor(rng.integers(0, L, batch), dtype=torch.int32, device=self.device)
            abi.mrt_srg_gather(controls, L, idx, oy, ox, x, batch, crop, crop)
            abi.mrt_srg_gather(responses, L, idx, oy, ox, y, batch, crop, crop, sub=u_base)
            lr_s = lr * 0.5 * (1.0 + math.cos(math.pi * s / steps))
            want = (s % log_every == 0) or s == steps - 1
            loss = abi.mrt_srg_train_step(self.handle, x, y, batch, crop, crop, border,
                                          max(lr_s, lr * 1e-3), want_loss=want)
            if want:
                hist.append(loss)
        return hist

    def close(self) -> None:
        if getattr(self, "handle", None):
            abi.mrt_srg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ training data

def render_bumps(n: int, L: int, rng: np.random.Generator, device,
                 kmin=1, kmax=8, smin=4.0, smax=32.0, amax=5.0) -> torch.Tensor:
    """n periodic controls, each a sum of K ~ U{kmin..kmax} Gaussian bumps
    (uniform centres, sigma ~ U[smin, smax], amplitude ~ U[-amax, amax]).
    The random draws are seeded numpy; the sums are evaluated on the device."""
    out = torch.zeros((n, L, L), dtype=torch.float32, device=device)
    ax = torch.arange(L, dtype=torch.float32, device=device)
    for i in range(n):
        k = int(rng.integers(kmin, kmax + 1))
        cx, cy = rng.uniform(0, L, k), rng.uniform(0, L, k)
        sig, amp = rng.uniform(smin, smax, k), rng.uniform(-amax, amax, k)
        for j in range(k):
            dx = (ax - float(cx[j])).abs()
            dx = torch.minimum(dx, L - dx)
            dy = (ax - float(cy[j])).abs()
            dy = torch.minimum(dy, L - dy)
            out[i] += float(amp[j]) * torch.exp(-(dy[:, None] ** 2 + dx[None, :] ** 2)
                                                / (2.0 * float(sig[j]) ** 2))
    return out


def physics(L: int, nsteps: int) -> "I.Problem":
    """The learned problem family: the periodic isotropic physics on a periodic L x L lattice,
    u0 = 1, v0 = 0."""
    p = I.periodic_isotropic(L=L, nsteps=nsteps)
    return p.copy(u0=np.ones((L, L)), v0=np.zeros((L, L)), control=np.zeros((L, L)))


def generate_pairs(n: int, L: int, nsteps: int, seed: int, per_launch: int = 96,
                   device="cuda:0", smax: float = 32.0) -> Dict[str, torch.Tensor]:
    """(control, u(T)) pairs from forward MRT solves of the batched engine
    (one persistent launch per group of `per_launch` controls), and the
    uncontrolled u(T) = u_base.  The network learns u(T) - u_base."""
    dev = torch.device(device)
    rng = np.random.default_rng(seed)
    base = physics(L, nsteps)
    m = min(per_launch, n)
    b = Batch([base] * m, dtype=torch.float32, ckpt_every=-1, device=dev)
    # u_base: the uncontrolled solution
    abi.mrt_batch_forward(b.handle)
    u_base = b.get(0, "uN").clone()
    controls = render_bumps(n, L, rng, dev, smax=smax)
    responses = torch.empty_like(controls)
    for s in range(0, n, m):
        cnt = min(m, n - s)
        for k in range(cnt):
            abi.mrt_batch_copy(b.handle, k, abi.MRT_FIELD_CONTROL, True, controls[s + k])
        abi.mrt_batch_forward(b.handle)
        for k in range(cnt):
            abi.mrt_batch_copy(b.handle, k, abi.MRT_FIELD_UN, False, responses[s + k])
    torch.cuda.synchronize(dev)
    b.close()
    return {"controls": controls, "responses": responses, "u_base": u_base}


# ------------------------------------------------------- optimisation loops

class ControlProblem:
    """One control problem on the device with counters of MRT solves."""

    def __init__(self, prob, dtype=torch.float32, device="cuda:0"):
        self.prob = prob
        self.dp = DeviceProblem(prob, dtype=dtype, device=device)
        self.it = GradientIteration(self.dp, ckpt_every=-1)
        self.ftape = Tape(self.dp, 0)
        self.uN = self.dp.empty_field()
        self.trial = self.dp.empty_field()
        self.n_forward = 0
        self.n_adjoint = 0
        assert self.dp.pitch == self.dp.nx, "square lattices with nx a multiple of 64"

    def cost(self, c: torch.Tensor) -> float:
        dp = self.dp
        abi.mrt_forward(dp.struct, self.ftape.handle, dp.u0, dp.v0, c, None, self.uN, None)
        r = abi.cost_gradient(dp.struct, self.ftape.handle, self.uN, dp.u_target, c)
        self.n_forward += 1
        return r["J"]

    def step(self, c: torch.Tensor, E: torch.Tensor, lam: float) -> None:
        """c <- c - lam E in place (gd_step with a given step size)."""
        abi.gd_step(self.dp.struct, self.ftape.handle, c, E, zeta=lam, want_zeta=False)

    def trial_cost(self, c: torch.Tensor, E: torch.Tensor, lam: float) -> float:
        """J(c - lam E), one MRT forward."""
        self.trial.copy_(c)
        self.step(self.trial, E, lam)
        return self.cost(self.trial)

    def gradient(self, c: torch.Tensor):
        """J, E = grad J, ||E||_inf and ||E||_2 at c (one MRT + AMRT)."""
        r = self.it.gradient(control=c)
        self.n_forward += 1
        self.n_adjoint += 1
        return r["J"], self.it.grad.clone(), r["grad_inf"], r["grad_l2"]

    def close(self):
        self.it.close()
        self.ftape.close()


def line_search(cp: ControlProblem, c, E, J0, lam0, max_expand=20, golden=6):
    """Line minimisation of J(c - lam E) (Remark after Step 6: zeta_k =
    argmin J(f - lam E)): bracket by doubling from lam0, then a golden-
    section refinement with `golden` more MRT forwards.  Returns (lam, J)."""
    f = {0.0: J0}

    def J(lam):
        if lam not in f:
            f[lam] = cp.trial_cost(c, E, lam)
        return f[lam]

    a, b = 0.0, lam0
    if J(b) >= J0:
        for _ in range(8):  # shrink until a decrease
            b *= 0.25
            if J(b) < J0:
                break
        else:
            return 0.0, J0
    cc = 2.0 * b
    for _ in range(max_expand):
        if J(cc) >= J(b):
            break
        a, b, cc = b, cc, 2.0 * cc
    gr = (math.sqrt(5.0) - 1.0) / 2.0
    lo, hi = a, cc
    x1, x2 = hi - gr * (hi - lo), lo + gr * (hi - lo)
    for _ in range(golden // 2):
        if J(x1) < J(x2):
            hi, x2 = x2, x1
            x1 = hi - gr * (hi - lo)
        else:
            lo, x1 = x1, x2
            x2 = lo + gr * (hi - lo)
    lam = min(f, key=f.get)
    return lam, f[lam]


def optimize_plain(cp: ControlProblem, iters: int, c0=None) -> dict:
    """Gradient iterations with the exact line search."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c = (cp.dp.field(None) if c0 is None else c0.clone())
    hist = []
    J = None
    for _ in range(iters):
        J, E, einf, _ = cp.gradient(c)
        hist.append(J)
        lam, Jn = line_search(cp, c, E, J, min(1.0, 1.0 / max(einf, 1e-300)))
        cp.step(c, E, lam)
        J = Jn
    hist.append(J)
    torch.cuda.synchronize()
    return {"J": J, "hist": hist, "control": c, "time": time.perf_counter() - t0,
            "forwards": cp.n_forward, "adjoints": cp.n_adjoint}


def optimize_assisted(cp: ControlProblem, srg: Surrogate, u_base, target_J: float,
                      max_iters: int = 50, n_cand: int = 16, warm_iters: int = 300) -> dict:
    """Surrogate-assisted gradient loop: warm start from the surrogate, then
    per iteration one MRT+AMRT gradient, surrogate-scored step candidates in
    one batched inference, and one MRT forward that verifies the chosen step
    (Armijo, c1 = 1e-4); a rejected proposal falls back to the exact line
    search.  Stops once J <= target_J."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nx = cp.dp.nx
    ut = cp.dp.u_target[:, :nx]
    alpha = cp.prob.alpha
    c = srg.warm_start(u_base, ut, alpha, iters=warm_iters)
    J = cp.cost(c)
    hist = [J]
    accepted = fallbacks = 0
    for _ in range(max_iters):
        if J <= target_J:
            break
        J, E, einf, e2 = cp.gradient(c)
        lam0 = min(1.0, 1.0 / max(einf, 1e-300))
        lams = [lam0 * 2.0 ** k for k in range(-2, n_cand - 2)]
        # surrogate costs of the candidates and of c itself (lambda = 0):
        # the predicted change is added to the true J
        pj = srg.score_steps(c, E, lams + [0.0], u_base, ut, alpha)
        pred = [pj[k] - pj[-1] + J for k in range(n_cand)]
        lam = lams[int(np.argmin(pred))]
        Jn = cp.trial_cost(c, E, lam)
        if Jn <= J - 1e-4 * lam * e2 * e2:
            accepted += 1
        else:
            fallbacks += 1
            lam, Jn = line_search(cp, c, E, J, lam0)
        cp.step(c, E, lam)
        J = Jn
        hist.append(J)
    torch.cuda.synchronize()
    return {"J": J, "hist": hist, "control": c, "time": time.perf_counter() - t0,
            "forwards": cp.n_forward, "adjoints": cp.n_adjoint,
            "accepted": accepted, "fallbacks": fallbacks}


def hidden_target_problem(L: int, nsteps: int, seed: int, device="cuda:0",
                          amax: float = 3.0, smin: float = 6.0, smax: float = 24.0):
    """A reachable target: u_target = u(T) of a hidden seeded bump control
    (computed with one MRT forward)."""
    dev = torch.device(device)
    rng = np.random.default_rng(seed)
    hidden = render_bumps(1, L, rng, dev, kmin=2, kmax=5, smin=smin, smax=smax, amax=amax)[0]
    p = physics(L, nsteps)
    dp = DeviceProblem(p, device=dev)
    t = Tape(dp, 0)
    uN = dp.empty_field()
    abi.mrt_forward(dp.struct, t.handle, dp.u0, dp.v0, hidden.contiguous(), None, uN, None)
    torch.cuda.synchronize(dev)
    target = dp.host(uN)
    t.close()
    return p.copy(u_target=target), hidden
