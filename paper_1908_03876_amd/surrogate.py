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
        """y = S(x)."""
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

    def zero_response_base(self, u_base: torch.Tensor) -> torch.Tensor:
        """u_base - S(0): the base field corrected by the network's response to
        the zero control (a small constant where it should be exactly zero),
        so that the model's control response, like the true one, vanishes at
        c = 0.  Without it a warm start spreads a spurious control over every
        flat region of the lattice to cancel the offset."""
        z = torch.zeros((1,) + tuple(u_base.shape), dtype=torch.float32, device=self.device)
        return (u_base - self.forward(z)[0]).contiguous()

    def warm_start_bb(self, u_base, u_target, alpha: float, iters: int = 100,
                      step0: float = 0.5, c0: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Control minimising the surrogate cost by steepest descent with
        Barzilai-Borwein steps (one step length for the whole field, so flat
        regions where the surrogate's gradient is only noise stay put), from
        c0 (default 0); the iterate of least surrogate cost."""
        H, W = u_target.shape
        c = torch.zeros((H, W), dtype=torch.float32, device=self.device) if c0 is None \
            else c0.clone().contiguous()
        abi.mrt_srg_warm_start_bb(self.handle, u_base.contiguous(), u_target.contiguous(),
                                  alpha, H, W, iters, step0, c)
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

def draw_bumps(n: int, L: int, rng: np.random.Generator, kmin=1, kmax=8, smin=4.0,
               smax=32.0, amax=5.0):
    """Seeded parameters of n controls, each a sum of K ~ U{kmin..kmax}
    Gaussian bumps (uniform centres, sigma ~ U[smin, smax], amplitude ~
    U[-amax, amax]), as [n, kmax] arrays (unused slots have amplitude 0)."""
    cx, cy = np.zeros((n, kmax)), np.zeros((n, kmax))
    sig, amp = np.ones((n, kmax)), np.zeros((n, kmax))
    for i in range(n):
        k = int(rng.integers(kmin, kmax + 1))
        cx[i, :k], cy[i, :k] = rng.uniform(0, L, k), rng.uniform(0, L, k)
        sig[i, :k], amp[i, :k] = rng.uniform(smin, smax, k), rng.uniform(-amax, amax, k)
    return cx, cy, sig, amp


def render_bumps(n: int, L: int, rng: np.random.Generator, device,
                 kmin=1, kmax=8, smin=4.0, smax=32.0, amax=5.0,
                 chunk: int = 512) -> torch.Tensor:
    """n periodic controls of draw_bumps on an L x L lattice, evaluated on the
    device: a periodic Gaussian factors into a row and a column profile, so
    a control is sum_k a_k g_k(y) h_k(x), one small batched product per chunk
    of controls."""
    cx, cy, sig, amp = draw_bumps(n, L, rng, kmin, kmax, smin, smax, amax)
    out = torch.empty((n, L, L), dtype=torch.float32, device=device)
    ax = torch.arange(L, dtype=torch.float32, device=device)

    def profile(centre, s2):
        d = (ax[None, None, :] - centre[:, :, None]).abs()
        d = torch.minimum(d, L - d)
        return torch.exp(-(d * d) / s2[:, :, None])

    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        T = lambda a: torch.tensor(a[s:e], dtype=torch.float32, device=device)
        s2 = 2.0 * T(sig) ** 2
        gy = (profile(T(cy), s2) * T(amp)[:, :, None]).transpose(1, 2).contiguous()
        gx = profile(T(cx), s2).contiguous()
        torch.bmm(gy, gx, out=out[s:e])
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
    uncontrolled u(T) = u_base.  The network learns u(T) - u_base.  Also
    returns the seconds spent rendering the controls, copying them in and
    out of the batch, and in the MRT launches, with the latter's rate."""
    dev = torch.device(device)
    rng = np.random.default_rng(seed)
    base = physics(L, nsteps)
    m = min(per_launch, n)
    b = Batch([base] * m, dtype=torch.float32, ckpt_every=-1, device=dev)
    # u_base: the uncontrolled solution
    abi.mrt_batch_forward(b.handle)
    u_base = b.get(0, "uN").clone()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    controls = render_bumps(n, L, rng, dev, smax=smax)
    torch.cuda.synchronize(dev)
    t_render = time.perf_counter() - t0
    responses = torch.empty_like(controls)
    t_copy = t_solve = 0.0
    for s in range(0, n, m):
        cnt = min(m, n - s)
        ta = time.perf_counter()
        for k in range(cnt):
            abi.mrt_batch_copy(b.handle, k, abi.MRT_FIELD_CONTROL, True, controls[s + k])
        torch.cuda.synchronize(dev)
        tb = time.perf_counter()
        abi.mrt_batch_forward(b.handle)
        torch.cuda.synchronize(dev)
        tc = time.perf_counter()
        for k in range(cnt):
            abi.mrt_batch_copy(b.handle, k, abi.MRT_FIELD_UN, False, responses[s + k])
        torch.cuda.synchronize(dev)
        t_copy += (tb - ta) + (time.perf_counter() - tc)
        t_solve += tc - tb
    b.close()
    launches = (n + m - 1) // m
    return {"controls": controls, "responses": responses, "u_base": u_base,
            "render_s": t_render, "copy_s": t_copy, "solve_s": t_solve,
            "solve_glups": launches * m * L * L * nsteps / max(t_solve, 1e-9) / 1e9}


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
        self.n_tlm = 0
        assert self.dp.pitch == self.dp.nx, "square lattices with nx a multiple of 64"

    @property
    def solves(self) -> int:
        """MRT sweeps so far (forward, adjoint and tangent-linear)."""
        return self.n_forward + self.n_adjoint + self.n_tlm

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

    def recorded_cost(self, c: torch.Tensor) -> float:
        """J(c) from one MRT forward that also records the adjoint tape, so
        that adjoint_gradient(c) can follow without another forward."""
        self.it.forward(c)
        self.n_forward += 1
        return self.it.cost(c)["J"]

    def adjoint_gradient(self, c: torch.Tensor):
        """E, ||E||_inf, ||E||_2 at c from the AMRT of the last
        recorded_cost(c) (the same tensor c)."""
        dp, t = self.dp, self.it.tape.handle
        abi.amrt_adjoint(dp.struct, t, dp.u0, dp.v0, c, self.it.seed, None, self.it.gacc,
                         None, None)
        r = abi.cost_gradient(dp.struct, t, self.it.uN, dp.u_target, c, self.it.gacc, None,
                              self.it.grad)
        self.n_adjoint += 1
        return self.it.grad.clone(), r["grad_inf"], r["grad_l2"]

    def lma_step(self, c: torch.Tensor) -> float:
        """LMA step size (Section 2.4) at c after gradient(c): one
        tangent-linear solve."""
        self.n_tlm += 1
        return self.it.lma_zeta(control=c)

    def close(self):
        self.it.close()
        self.ftape.close()


def line_search(cp: ControlProblem, c, E, J0, lam0, max_bracket=8, golden=4):
    """Line minimisation of J(c - lam E) (Remark after Step 6: zeta_k =
    argmin J(f - lam E)), with true MRT forwards: from the first trial lam0
    (the previous iteration's step, or the heuristic one at the start),
    shrink or expand by factors of 4 until J(lam) is bracketed, then
    `golden` golden-section forwards in the bracket.  In the usual case (the
    previous step still decreases J and four times it does not) that is six
    forwards.  Returns (lam, J)."""
    f = {0.0: J0}

    def J(lam):
        if lam not in f:
            f[lam] = cp.trial_cost(c, E, lam)
        return f[lam]

    a, b = 0.0, lam0
    if J(b) >= J0:
        for _ in range(max_bracket):  # shrink until a decrease
            b *= 0.25
            if J(b) < J0:
                break
        else:
            return 0.0, J0
        cc = 4.0 * b
    else:
        cc = 4.0 * b
        for _ in range(max_bracket):
            if J(cc) >= J(b):
                break
            a, b, cc = b, cc, 4.0 * cc
    gr = (math.sqrt(5.0) - 1.0) / 2.0
    lo, hi = a, cc
    x1, x2 = hi - gr * (hi - lo), lo + gr * (hi - lo)
    f1, f2 = J(x1), J(x2)
    for _ in range(max(golden - 2, 0)):
        if f1 < f2:
            hi, x2, f2 = x2, x1, f1
            x1 = hi - gr * (hi - lo)
            f1 = J(x1)
        else:
            lo, x1, f1 = x1, x2, f2
            x2 = lo + gr * (hi - lo)
            f2 = J(x2)
    lam = min(f, key=f.get)
    return lam, f[lam]


def _clock(t0: float) -> float:
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def _result(cp: ControlProblem, hist, c, t0, **extra) -> dict:
    out = {"J": hist[-1][1], "hist": [h[1] for h in hist], "times": [h[0] for h in hist],
           "control": c, "time": _clock(t0), "forwards": cp.n_forward,
           "adjoints": cp.n_adjoint, "tlms": cp.n_tlm, "solves": cp.solves}
    out.update(extra)
    return out


def optimize_plain(cp: ControlProblem, iters: int, c0=None) -> dict:
    """Gradient iterations with the golden-section line search, its first
    trial the previous iteration's step.  hist/times: J at each iterate and
    the wall time at which it was known."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c = (cp.dp.field(None) if c0 is None else c0.clone())
    hist, lam = [], None
    J = None
    for _ in range(iters):
        J, E, einf, _ = cp.gradient(c)
        if not hist:
            hist.append((_clock(t0), J))
        lam0 = min(1.0, 1.0 / max(einf, 1e-300)) if not lam else lam
        lam, J = line_search(cp, c, E, J, lam0)
        cp.step(c, E, lam)
        hist.append((_clock(t0), J))
    return _result(cp, hist, c, t0)


def optimize_lma(cp: ControlProblem, iters: int, c0=None) -> dict:
    """Gradient iterations with the LMA step (one gradient and one
    tangent-linear solve per iteration, no line search)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c = (cp.dp.field(None) if c0 is None else c0.clone())
    hist = []
    for _ in range(iters):
        J, E, _, _ = cp.gradient(c)
        hist.append((_clock(t0), J))
        z = cp.lma_step(c)
        cp.step(c, E, z)
    hist.append((_clock(t0), cp.cost(c)))
    return _result(cp, hist, c, t0)


def optimize_cg(cp: ControlProblem, iters: int, rule: str = "PR") -> dict:
    """Nonlinear conjugate gradients (Section 2.4, Remark after Step 6) with
    the Wolfe line search whose first trial is the LMA step along D, from
    the problem's control."""
    from .optim import ConjugateGradient
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cg = ConjugateGradient(cp.dp, rule=rule, ckpt_every=-1)
    hist = [(_clock(t0), cg.start())]
    for _ in range(iters):
        hist.append((_clock(t0), cg.iterate()["J"]))
    cp.n_forward += cg.evals
    cp.n_adjoint += cg.evals
    cp.n_tlm += cg.tlms
    c = cg.control.clone()
    out = _result(cp, hist, c, t0)
    cg.close()
    return out


def optimize_assisted(cp: ControlProblem, srg: Surrogate, u_base, target_J: float,
                      max_iters: int = 50, warm_iters: int = 100) -> dict:
    """Surrogate-assisted gradient loop: warm start from the surrogate
    (Barzilai-Borwein steps on the surrogate cost), then per iteration one
    AMRT gradient E, the step along -E from the surrogate's curvature
    (SurrogateSteps, slope -|E|^2) and one MRT forward that verifies it
    (Armijo, c1 = 1e-4) and records the tape for the next gradient; a
    rejected step falls back to the exact line search.  Stops once
    J <= target_J."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nx = cp.dp.nx
    ut = cp.dp.u_target[:, :nx]
    alpha = cp.prob.alpha
    u_base = srg.zero_response_base(u_base)
    steps = SurrogateSteps(srg, u_base, ut, alpha)
    c = srg.warm_start_bb(u_base, ut, alpha, iters=warm_iters)
    buf = torch.empty_like(c)
    J = cp.recorded_cost(c)
    hist = [(_clock(t0), J)]
    accepted = fallbacks = 0
    lam_prev = None
    for _ in range(max_iters):
        if J <= target_J:
            break
        E, einf, e2 = cp.adjoint_gradient(c)
        h = lam_prev if lam_prev else 1.0 / math.sqrt(max(e2 * e2 / cp.it.tape.n_fluid,
                                                          1e-300))
        # along D = -E: score c + z D = c - z E, i.e. pass E with the sign
        # folded into the slope (phi'(0) = -|E|^2) and the points -h, 0, h
        lam = steps.step(c, E, -e2 * e2, h)
        lam0 = lam_prev if lam_prev else min(1.0, 1.0 / max(einf, 1e-300))
        Jn = math.inf
        if lam is not None:
            buf.copy_(c)
            cp.step(buf, E, lam)
            Jn = cp.recorded_cost(buf)
        if lam is not None and Jn <= J - 1e-4 * lam * e2 * e2:
            accepted += 1
            c, buf = buf, c
        else:
            fallbacks += 1
            lam, Jn = line_search(cp, c, E, J, lam0)
            cp.step(c, E, lam)
            Jn = cp.recorded_cost(c)
        lam_prev = lam
        J = Jn
        hist.append((_clock(t0), J))
    return _result(cp, hist, c, t0, accepted=accepted, fallbacks=fallbacks)


class SurrogateSteps:
    """Step sizes from the surrogate's curvature: along a direction D from c
    the cost is phi(z) = J(c + z D); its slope phi'(0) = <G, D> is exact
    (the adjoint gradient) and its curvature is taken from the surrogate,
    kappa = (J_s(c + h D) - 2 J_s(c) + J_s(c - h D)) / h^2, three surrogate
    costs in one batched inference.  The step z = -phi'(0) / kappa is the
    minimiser of that quadratic model: the linearised line minimisation
    (LMA) of Section 2.4 with the network's Jacobian in place of the
    tangent-linear solve.  h is the previous step (or a unit RMS move).  The
    MRT solve at the trial decides whether it is accepted."""

    def __init__(self, srg: Surrogate, u_base, u_target, alpha: float):
        self.srg, self.ub, self.ut, self.alpha = srg, u_base, u_target, alpha

    def step(self, c, D, slope: float, h: float):
        J = self.srg.score_steps(c, D, [-h, 0.0, h], self.ub, self.ut, self.alpha)
        kappa = (J[0] - 2.0 * J[1] + J[2]) / (h * h)
        if not (kappa > 0.0 and math.isfinite(kappa)) or not slope < 0.0:
            return None
        return -slope / kappa

    def __call__(self, cg, dg0: float):
        h = cg.last_zeta
        if not h:
            dd = abi.mrt_dot(cg.dp.struct, cg.it.tape.handle, cg.D, cg.D)
            h = 1.0 / math.sqrt(max(dd / cg.it.tape.n_fluid, 1e-300))
        return self.step(cg.c, cg.D, dg0, h)


def optimize_assisted_cg(cp: ControlProblem, srg: Surrogate, u_base, target_J: float,
                         max_iters: int = 40, warm_iters: int = 100, rule: str = "PR",
                         proposals: bool = False) -> dict:
    """Surrogate-assisted conjugate gradients: the warm start minimises the
    surrogate cost (Barzilai-Borwein steps, base field corrected by the
    network's zero-control response), then nonlinear CG on the true cost
    (MRT + AMRT gradients, Wolfe line search from the LMA step); with
    proposals=True the first trial steps come from the surrogate's curvature
    instead (no tangent-linear solve).  Stops once J <= target_J."""
    from .optim import ConjugateGradient
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nx = cp.dp.nx
    ut = cp.dp.u_target[:, :nx]
    alpha = cp.prob.alpha
    u_base = srg.zero_response_base(u_base)
    c0 = srg.warm_start_bb(u_base, ut, alpha, iters=warm_iters)
    steps = SurrogateSteps(srg, u_base, ut, alpha) if proposals else None
    cg = ConjugateGradient(cp.dp, rule=rule, ckpt_every=-1, first_trial=steps)
    cg.c.copy_(c0)
    hist = [(_clock(t0), cg.start())]
    for _ in range(max_iters):
        if hist[-1][1] <= target_J:
            break
        hist.append((_clock(t0), cg.iterate()["J"]))
    cp.n_forward += cg.evals
    cp.n_adjoint += cg.evals
    cp.n_tlm += cg.tlms
    c = cg.control.clone()
    out = _result(cp, hist, c, t0, restarts=cg.restarts)
    cg.close()
    return out


def time_to_reach(res: dict, target: float):
    """Wall time at which a loop first knew a J <= target (None if never)."""
    for t, J in zip(res["times"], res["hist"]):
        if J <= target:
            return t
    return None


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
