"""Device-resident problems, tapes and the gradient-descent loop on top of
the C-ABI (Section 3.2.1, discrete optimisation algorithm: forward N steps,
adjoint N..0, gradient, update, repeat).

Fields live in HBM as [ny, pitch] torch tensors (pitch = nx rounded up to 64
elements); every step of the computation runs in libmrt.so.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

from . import abi

_TORCH_DTYPE = {abi.MRT_F32: torch.float32, abi.MRT_F64: torch.float64}


def padded_pitch(nx: int, align: int = 64) -> int:
    return ((nx + align - 1) // align) * align


def make_problem_struct(prob, dtype_code: int, pitch: int,
                        mask_ptr: Optional[int], nsteps: Optional[int] = None,
                        w0_ptr: Optional[int] = None) -> abi.mrt_problem:
    p = abi.mrt_problem()
    g = p.grid
    g.nx, g.ny, g.pitch, g.q = int(prob.nx), int(prob.ny), int(pitch), 9
    g.periodic = 1 if prob.periodic else 0
    g.dtype = int(dtype_code)
    g.nsteps = int(prob.nsteps if nsteps is None else nsteps)
    g.reserved = 0
    g.mask = mask_ptr
    for dst, D, d, s in ((p.u, prob.Du, prob.du, prob.su),
                         (p.v, prob.Dv, prob.dv, prob.sv)):
        dst.D[:] = [float(x) for x in np.asarray(D, dtype=np.float64).ravel()]
        dst.d = float(d)
        dst.s[:] = [float(x) for x in np.asarray(s, dtype=np.float64).ravel()]
    p.chi = float(prob.chi)
    p.Cchi[:] = [float(x) for x in np.asarray(prob.Cchi, dtype=np.float64).ravel()]
    p.r_u, p.a_uv, p.b_v = float(prob.r_u), float(prob.a_uv), float(prob.b_v)
    p.alpha = float(prob.alpha)
    p.source_term = int(getattr(prob, "source_term", 1))
    p.nspecies = int(getattr(prob, "nspecies", 2))
    if p.nspecies == 3:
        p.w.D[:] = [float(x) for x in np.asarray(prob.Dw, dtype=np.float64).ravel()]
        p.w.d = float(prob.dw)
        p.w.s[:] = [float(x) for x in np.asarray(prob.sw, dtype=np.float64).ravel()]
        p.chi_w = float(prob.chi_w)
        p.Cw[:] = [float(x) for x in np.asarray(prob.Cw, dtype=np.float64).ravel()]
        p.a_w, p.b_w, p.s_w = float(prob.a_w), float(prob.b_w), float(prob.s_w)
        p.w0 = w0_ptr
    return p


class DeviceProblem:
    """A control problem with its fields resident on the GPU."""

    def __init__(self, prob, dtype=torch.float32, device="cuda:0",
                 nsteps: Optional[int] = None):
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be float32 or float64")
        self.prob = prob
        self.dtype = dtype
        self.code = abi.MRT_F64 if dtype == torch.float64 else abi.MRT_F32
        self.device = torch.device(device)
        self.nx, self.ny = int(prob.nx), int(prob.ny)
        self.pitch = padded_pitch(self.nx)
        self.nsteps = int(prob.nsteps if nsteps is None else nsteps)
        self.mask = None
        if prob.solid is not None:
            self.mask = self.field(prob.solid, dtype=torch.uint8)
        self.u0 = self.field(prob.u0)
        self.v0 = self.field(prob.v0)
        self.control = self.field(prob.control)
        self.u_target = self.field(prob.u_target)
        self.nspecies = int(getattr(prob, "nspecies", 2))
        self.w0 = self.field(prob.w0) if self.nspecies == 3 else None
        self.struct = make_problem_struct(
            prob, self.code, self.pitch,
            None if self.mask is None else self.mask.data_ptr(), self.nsteps,
            None if self.w0 is None else self.w0.data_ptr())
        abi.mrt_validate(self.struct)

    # -- host <-> device helpers (set-up and read-back only)
    def field(self, arr, dtype=None) -> torch.Tensor:
        dtype = self.dtype if dtype is None else dtype
        t = torch.zeros((self.ny, self.pitch), dtype=dtype, device=self.device)
        if arr is not None:
            t[:, : self.nx] = torch.as_tensor(np.ascontiguousarray(arr)).to(
                device=self.device, dtype=dtype)
        return t

    def empty_field(self, dtype=None) -> torch.Tensor:
        dtype = self.dtype if dtype is None else dtype
        return torch.zeros((self.ny, self.pitch), dtype=dtype, device=self.device)

    def host(self, t: torch.Tensor) -> np.ndarray:
        return t[:, : self.nx].double().cpu().numpy()

    def state_tensor(self) -> torch.Tensor:
        return torch.zeros((self.nspecies, 9, self.ny, self.pitch), dtype=self.dtype,
                           device=self.device)

    def with_nsteps(self, nsteps: int) -> "DeviceProblem":
        q = object.__new__(DeviceProblem)
        q.__dict__.update(self.__dict__)
        q.nsteps = int(nsteps)
        q.struct = make_problem_struct(
            self.prob, self.code, self.pitch,
            None if self.mask is None else self.mask.data_ptr(), nsteps,
            None if self.w0 is None else self.w0.data_ptr())
        return q


class Tape:
    """Owns an mrt_tape (device workspace + adjoint record)."""

    def __init__(self, dp: DeviceProblem, ckpt_every: int = -1,
                 mem_budget: int = 0):
        """ckpt_every: 0 forward only, -1 store-all, K > 0 checkpoint every
        K steps (K >= nsteps is store-all)."""
        if ckpt_every < 0:
            ckpt_every = dp.nsteps
        self.dp = dp
        with torch.cuda.device(dp.device):
            self.handle = abi.mrt_tape_create(dp.struct, ckpt_every, mem_budget)
        self.info = abi.mrt_tape_query(self.handle)

    @staticmethod
    def bytes_needed(dp: DeviceProblem, ckpt_every: int) -> int:
        return abi.mrt_tape_bytes(dp.struct, ckpt_every)

    @property
    def n_fluid(self) -> int:
        return int(self.info.n_fluid)

    def close(self):
        if getattr(self, "handle", None):
            abi.mrt_tape_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def choose_ckpt_every(dp: DeviceProblem, budget_bytes: int) -> int:
    """Largest record that fits: store-all if possible, else the checkpoint
    interval that minimises memory (about sqrt(N) * the state/record ratio)
    while fitting the budget."""
    if Tape.bytes_needed(dp, dp.nsteps) <= budget_bytes:
        return dp.nsteps
    best = None
    for K in sorted({max(1, int(round(math.sqrt(dp.nsteps * 6 * x)))) for x in
                     (0.25, 0.5, 1, 2, 4)} | {10, 25, 50, 100, 200, 400}):
        if K >= dp.nsteps:
            continue
        b = Tape.bytes_needed(dp, K)
        if b <= budget_bytes and (best is None or b < best[0]):
            best = (b, K)
    if best is None:
        raise MemoryError("no checkpoint interval fits the memory budget")
    return best[1]


class GradientIteration:
    """One discrete gradient of J(c) and the update (Section 3.2.1):
    forward -> cost & seed -> AMRT adjoint -> gradient & norms -> gd_step."""

    def __init__(self, dp: DeviceProblem, ckpt_every: int = -1,
                 mem_budget: int = 0):
        self.dp = dp
        self.tape = Tape(dp, ckpt_every, mem_budget)
        self.uN = dp.empty_field()
        self.vN = dp.empty_field()
        self.seed = dp.empty_field()
        self.gacc = dp.empty_field(torch.float64)
        self.grad = dp.empty_field()

    def forward(self, control=None, stream=None):
        dp = self.dp
        c = dp.control if control is None else control
        abi.mrt_forward(dp.struct, self.tape.handle, dp.u0, dp.v0, c,
                        None, self.uN, self.vN, stream)

    def cost(self, control=None, stream=None) -> dict:
        dp = self.dp
        c = dp.control if control is None else control
        return abi.cost_gradient(dp.struct, self.tape.handle, self.uN,
                                 dp.u_target, c, None, self.seed, None, stream)

    def gradient(self, control=None, stream=None) -> dict:
        """Forward + adjoint; returns J and the gradient norms; the gradient
        is left in self.grad."""
        dp = self.dp
        c = dp.control if control is None else control
        self.forward(c, stream)
        r1 = abi.cost_gradient(dp.struct, self.tape.handle, self.uN,
                               dp.u_target, c, None, self.seed, None, stream)
        abi.amrt_adjoint(dp.struct, self.tape.handle, dp.u0, dp.v0, c,
                         self.seed, None, self.gacc, None, None, stream)
        r2 = abi.cost_gradient(dp.struct, self.tape.handle, self.uN,
                               dp.u_target, c, self.gacc, None, self.grad,
                               stream)
        r2["J"], r2["J_track"], r2["J_reg"] = r1["J"], r1["J_track"], r1["J_reg"]
        return r2

    def gradient_continuous(self, control=None, stream=None) -> dict:
        """As gradient(), with the continuous-adjoint sweep (Section 3.2.2)
        in place of the AMRT: an approximation of the discrete gradient."""
        dp = self.dp
        c = dp.control if control is None else control
        self.forward(c, stream)
        r1 = abi.cost_gradient(dp.struct, self.tape.handle, self.uN,
                               dp.u_target, c, None, self.seed, None, stream)
        abi.mrt_cadjoint(dp.struct, self.tape.handle, dp.u0, dp.v0, c, self.seed,
                         self.gacc, stream)
        r2 = abi.cost_gradient(dp.struct, self.tape.handle, self.uN,
                               dp.u_target, c, self.gacc, None, self.grad,
                               stream)
        r2["J"], r2["J_track"], r2["J_reg"] = r1["J"], r1["J_track"], r1["J_reg"]
        return r2

    def step(self, zeta: float = 0.0, lo: float = -math.inf,
             hi: float = math.inf, stream=None, want_zeta: bool = True) -> dict:
        """One iteration of the gradient algorithm on dp.control (in place)."""
        r = self.gradient(stream=stream)
        r["zeta"] = abi.gd_step(self.dp.struct, self.tape.handle,
                                self.dp.control, self.grad, zeta, lo, hi,
                                want_zeta=want_zeta, stream=stream)
        return r

    def run(self, max_iters: int, gtol: float = 0.0, zeta: float = 0.0,
            lo: float = -math.inf, hi: float = math.inf, stream=None) -> list:
        """The gradient algorithm of Section 3.2.1 for at most max_iters
        iterations, stopping before an update once ||E_k||_2 <= gtol ||E_0||_2
        (the "gradient small enough" test; gtol = 0 runs every iteration).
        Returns the per-iteration scalars; the last entry is the iteration
        that met the test, if any (its gradient was computed, no step taken)."""
        hist = []
        g0 = None
        for _ in range(max_iters):
            r = self.gradient(stream=stream)
            g0 = r["grad_l2"] if g0 is None else g0
            if gtol > 0.0 and r["grad_l2"] <= gtol * g0:
                r["stopped"] = True
                hist.append(r)
                break
            r["zeta"] = abi.gd_step(self.dp.struct, self.tape.handle, self.dp.control,
                                    self.grad, zeta, lo, hi, stream=stream)
            hist.append(r)
        return hist

    def tlm(self, dc=None, du0=None, dv0=None, control=None, stream=None):
        """Tangent-linear response (du^N, dv^N) of the last forward on this
        iteration's tape to the perturbation (dc, du0, dv0)."""
        dp = self.dp
        c = dp.control if control is None else control
        if not hasattr(self, "duN"):
            self.duN = dp.empty_field()
            self.dvN = dp.empty_field()
        abi.mrt_tlm(dp.struct, self.tape.handle, dp.u0, dp.v0, c, dc, du0, dv0,
                    self.duN, self.dvN, stream)
        return self.duN, self.dvN

    def lma_zeta(self, control=None, stream=None) -> float:
        """Step of the linearised line minimisation (LMA, Section 2.4) for the
        quadratic cost, after gradient(): with P = F'(c) E from the
        tangent-linear model,
            zeta = (<u^N - u_t, P> + alpha <c, E>) / (<P, P> + alpha <E, E>)."""
        dp = self.dp
        c = dp.control if control is None else control
        P, _ = self.tlm(dc=self.grad, control=c, stream=stream)
        return abi.mrt_lma_step(dp.struct, self.tape.handle, c, self.grad, self.seed, P, stream)

    def step_lma(self, lo: float = -math.inf, hi: float = math.inf, stream=None) -> dict:
        """One gradient iteration with the LMA step size (one extra
        tangent-linear solve instead of a line search)."""
        r = self.gradient(stream=stream)
        z = self.lma_zeta(stream=stream)
        abi.gd_step(self.dp.struct, self.tape.handle, self.dp.control, self.grad, z, lo, hi,
                    want_zeta=False, stream=stream)
        r["zeta"] = z
        return r

    def close(self):
        self.tape.close()
