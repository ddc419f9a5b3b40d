"""Device-resident D3Q19 problems, tapes and the gradient iteration on top
of the mrt3 C-ABI (Section 3.2.1 on the D3Q19 lattice of the Remark on
DmQq lattices: forward N steps, adjoint N..0, gradient, update).

Fields live in HBM as [nz, ny, pitch] torch tensors (pitch = nx rounded up
to 64 elements); every step of the computation runs in libmrt.so.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

from . import abi
from .solver import padded_pitch


def make_problem3_struct(prob, dtype_code: int, pitch: int, mask_ptr: Optional[int],
                         nsteps: Optional[int] = None) -> abi.mrt3_problem:
    p = abi.mrt3_problem()
    g = p.grid
    g.nx, g.ny, g.nz, g.pitch = int(prob.nx), int(prob.ny), int(prob.nz), int(pitch)
    g.periodic = 1 if prob.periodic else 0
    g.dtype = int(dtype_code)
    g.nsteps = int(prob.nsteps if nsteps is None else nsteps)
    g.reserved = 0
    g.mask = mask_ptr
    for dst, D, d, s in ((p.u, prob.Du, prob.du, prob.su), (p.v, prob.Dv, prob.dv, prob.sv)):
        dst.D[:] = [float(x) for x in np.asarray(D, dtype=np.float64).ravel()]
        dst.d = float(d)
        dst.s[:] = [float(x) for x in np.asarray(s, dtype=np.float64).ravel()]
    p.chi = float(prob.chi)
    p.Cchi[:] = [float(x) for x in np.asarray(prob.Cchi, dtype=np.float64).ravel()]
    p.r_u, p.a_uv, p.b_v = float(prob.r_u), float(prob.a_uv), float(prob.b_v)
    p.alpha = float(prob.alpha)
    return p


class DeviceProblem3:
    """A D3Q19 control problem with its fields resident on the GPU."""

    def __init__(self, prob, dtype=torch.float32, device="cuda:0",
                 nsteps: Optional[int] = None):
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be float32 or float64")
        self.prob = prob
        self.dtype = dtype
        self.code = abi.MRT_F64 if dtype == torch.float64 else abi.MRT_F32
        self.device = torch.device(device)
        self.nx, self.ny, self.nz = int(prob.nx), int(prob.ny), int(prob.nz)
        self.pitch = padded_pitch(self.nx)
        self.nsteps = int(prob.nsteps if nsteps is None else nsteps)
        self.mask = None
        if prob.solid is not None:
            self.mask = self.field(prob.solid, dtype=torch.uint8)
        self.u0 = self.field(prob.u0)
        self.v0 = self.field(prob.v0)
        self.control = self.field(prob.control)
        self.u_target = self.field(prob.u_target)
        self.struct = make_problem3_struct(
            prob, self.code, self.pitch, None if self.mask is None else self.mask.data_ptr(),
            self.nsteps)
        abi.mrt3_validate(self.struct)

    def field(self, arr, dtype=None) -> torch.Tensor:
        dtype = self.dtype if dtype is None else dtype
        t = torch.zeros((self.nz, self.ny, self.pitch), dtype=dtype, device=self.device)
        if arr is not None:
            t[:, :, : self.nx] = torch.as_tensor(np.ascontiguousarray(arr)).to(
                device=self.device, dtype=dtype)
        return t

    def empty_field(self, dtype=None) -> torch.Tensor:
        dtype = self.dtype if dtype is None else dtype
        return torch.zeros((self.nz, self.ny, self.pitch), dtype=dtype, device=self.device)

    def host(self, t: torch.Tensor) -> np.ndarray:
        return t[..., : self.nx].double().cpu().numpy()

    def state_tensor(self) -> torch.Tensor:
        return torch.zeros((2, 19, self.nz, self.ny, self.pitch), dtype=self.dtype,
                           device=self.device)


class Tape3:
    """Owns an mrt3_tape (device workspace + adjoint record)."""

    def __init__(self, dp: DeviceProblem3, ckpt_every: int = -1, mem_budget: int = 0):
        """ckpt_every: 0 forward only, -1 store-all, K > 0 checkpoint every
        K steps (K >= nsteps is store-all)."""
        if ckpt_every < 0:
            ckpt_every = dp.nsteps
        self.dp = dp
        with torch.cuda.device(dp.device):
            self.handle = abi.mrt3_tape_create(dp.struct, ckpt_every, mem_budget)
        self.info = abi.mrt3_tape_query(self.handle)

    @property
    def n_fluid(self) -> int:
        return int(self.info.n_fluid)

    def close(self):
        if getattr(self, "handle", None):
            abi.mrt3_tape_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GradientIteration3:
    """One discrete gradient of J(c) on the D3Q19 lattice and the update:
    forward -> cost & seed -> AMRT adjoint -> gradient & norms -> gd_step."""

    def __init__(self, dp: DeviceProblem3, ckpt_every: int = -1, mem_budget: int = 0):
        self.dp = dp
        self.tape = Tape3(dp, ckpt_every, mem_budget)
        self.uN = dp.empty_field()
        self.vN = dp.empty_field()
        self.seed = dp.empty_field()
        self.gacc = dp.empty_field(torch.float64)
        self.grad = dp.empty_field()

    def forward(self, control=None, state=None, stream=None):
        dp = self.dp
        c = dp.control if control is None else control
        abi.mrt3_forward(dp.struct, self.tape.handle, dp.u0, dp.v0, c, state, self.uN,
                         self.vN, stream)

    def gradient(self, control=None, stream=None) -> dict:
        """Forward + adjoint; returns J and the gradient norms; the gradient
        is left in self.grad."""
        dp = self.dp
        c = dp.control if control is None else control
        self.forward(c, stream=stream)
        r1 = abi.mrt3_cost_gradient(dp.struct, self.tape.handle, self.uN, dp.u_target, c,
                                    None, self.seed, None, stream)
        abi.amrt3_adjoint(dp.struct, self.tape.handle, dp.u0, dp.v0, c, self.seed, None,
                          self.gacc, None, None, stream)
        r2 = abi.mrt3_cost_gradient(dp.struct, self.tape.handle, self.uN, dp.u_target, c,
                                    self.gacc, None, self.grad, stream)
        r2["J"], r2["J_track"], r2["J_reg"] = r1["J"], r1["J_track"], r1["J_reg"]
        return r2

    def step(self, zeta: float = 0.0, lo: float = -math.inf, hi: float = math.inf,
             stream=None, want_zeta: bool = True) -> dict:
        r = self.gradient(stream=stream)
        r["zeta"] = abi.mrt3_gd_step(self.dp.struct, self.tape.handle, self.dp.control,
                                     self.grad, zeta, lo, hi, want_zeta=want_zeta,
                                     stream=stream)
        return r

    def tlm(self, dc=None, du0=None, dv0=None, control=None, stream=None):
        dp = self.dp
        c = dp.control if control is None else control
        if not hasattr(self, "duN"):
            self.duN = dp.empty_field()
            self.dvN = dp.empty_field()
        abi.mrt3_tlm(dp.struct, self.tape.handle, dp.u0, dp.v0, c, dc, du0, dv0, self.duN,
                     self.dvN, stream)
        return self.duN, self.dvN

    def close(self):
        self.tape.close()
