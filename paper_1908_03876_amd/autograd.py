"""The MRT solve as a differentiable torch operation whose backward is the
AMRT sweep (Section 3.2.1: the discrete adjoint gives the exact gradient of
any functional of the final state; Theorem 3, gradientLattice).

    solver = MRTSolve(problem, ckpt_every=100)
    uN, vN = solver(control)                    # forward MRT, N steps
    loss = 0.5 * ((uN - target) ** 2).sum() + 0.5 * alpha * (control ** 2).sum()
    loss.backward()                             # AMRT, seeded by dloss/duN

The forward keeps only checkpoints (one distribution state every
`ckpt_every` steps) plus one segment of the (u, j_v) record, so device memory
is O(N/K * state + K * 12 bytes per node) however long the horizon; the
backward recomputes each segment from its checkpoint.  Every step runs in
libmrt.so; this module only moves tensors in and out of the library's padded
buffers.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import abi
from .solver import DeviceProblem, Tape
from .solver3 import DeviceProblem3, Tape3


class MRTSolve(torch.nn.Module):
    """Differentiable map (control, u0, v0) -> (u^N, v^N) of one problem, on
    D2Q9 (fields [ny, nx]) or, for a problem with a z extent, on D3Q19
    (fields [nz, ny, nx])."""

    def __init__(self, prob, dtype=torch.float32, device="cuda:0",
                 ckpt_every: int = 100, nsteps: Optional[int] = None,
                 mem_budget: int = 0):
        super().__init__()
        self.three_d = hasattr(prob, "nz")
        if self.three_d:
            self.dp = DeviceProblem3(prob, dtype=dtype, device=device, nsteps=nsteps)
            self.tape = Tape3(self.dp, ckpt_every, mem_budget)
            self._fwd, self._adj = abi.mrt3_forward, abi.amrt3_adjoint
        else:
            self.dp = DeviceProblem(prob, dtype=dtype, device=device, nsteps=nsteps)
            self.tape = Tape(self.dp, ckpt_every, mem_budget)
            self._fwd, self._adj = abi.mrt_forward, abi.amrt_adjoint
        dp = self.dp
        # library-side padded buffers ([(nz,) ny, pitch]); the tape's record
        # refers to the contents these held at the last forward
        self._u0, self._v0, self._c = dp.empty_field(), dp.empty_field(), dp.empty_field()
        self._uN, self._vN = dp.empty_field(), dp.empty_field()
        self._su, self._sv = dp.empty_field(), dp.empty_field()
        self._g = dp.empty_field(torch.float64)
        self._au0, self._av0 = dp.empty_field(), dp.empty_field()
        self._generation = 0
        self._recorded = None

    @property
    def shape(self):
        if self.three_d:
            return (self.dp.nz, self.dp.ny, self.dp.nx)
        return (self.dp.ny, self.dp.nx)

    def default_inputs(self):
        nx = self.dp.nx
        return (self.dp.control[..., :nx].clone(), self.dp.u0[..., :nx].clone(),
                self.dp.v0[..., :nx].clone())

    # -- called by the autograd Function
    def _run_forward(self, control, u0, v0):
        nx = self.dp.nx
        self._c[..., :nx].copy_(control)
        self._u0[..., :nx].copy_(u0)
        self._v0[..., :nx].copy_(v0)
        self._fwd(self.dp.struct, self.tape.handle, self._u0, self._v0, self._c, None,
                  self._uN, self._vN)
        self._generation += 1
        self._recorded = self._generation
        return self._uN[..., :nx].clone(), self._vN[..., :nx].clone(), self._generation

    def _run_adjoint(self, generation, control, u0, v0, gu, gv, want_u0, want_v0):
        nx = self.dp.nx
        if self._recorded != generation:
            # another forward ran since: re-record this one first
            self._run_forward(control, u0, v0)
        self._su.zero_()
        self._sv.zero_()
        if gu is not None:
            self._su[..., :nx].copy_(gu)
        sv = None
        if gv is not None:
            self._sv[..., :nx].copy_(gv)
            sv = self._sv
        self._adj(self.dp.struct, self.tape.handle, self._u0, self._v0, self._c, self._su, sv,
                  self._g, self._au0 if want_u0 else None, self._av0 if want_v0 else None)
        # a copy, never a view: in FP64 .to() would return the solver's own
        # buffer, which the next backward overwrites (and which autograd may
        # keep as .grad and accumulate into)
        gc = self._g[..., :nx].to(self.dp.dtype, copy=True)
        gu0 = self._au0[..., :nx].clone() if want_u0 else None
        gv0 = self._av0[..., :nx].clone() if want_v0 else None
        return gc, gu0, gv0

    def forward(self, control, u0=None, v0=None):
        if u0 is None or v0 is None:
            _, du0, dv0 = self.default_inputs()
            u0 = du0 if u0 is None else u0
            v0 = dv0 if v0 is None else v0
        return AMRTFunction.apply(control, u0, v0, self)

    def close(self):
        self.tape.close()


class AMRTFunction(torch.autograd.Function):
    """forward: MRT solve; backward: AMRT sweep seeded with the upstream
    gradients dL/du^N, dL/dv^N (terminal condition psi(T) = dI0/dphi)."""

    @staticmethod
    def forward(ctx, control, u0, v0, solver: MRTSolve):
        uN, vN, gen = solver._run_forward(control, u0, v0)
        ctx.solver = solver
        ctx.generation = gen
        ctx.save_for_backward(control, u0, v0)
        return uN, vN

    @staticmethod
    def backward(ctx, grad_uN, grad_vN):
        control, u0, v0 = ctx.saved_tensors
        s: MRTSolve = ctx.solver
        gc, gu0, gv0 = s._run_adjoint(ctx.generation, control, u0, v0,
                                      grad_uN, grad_vN,
                                      ctx.needs_input_grad[1],
                                      ctx.needs_input_grad[2])
        if not ctx.needs_input_grad[0]:
            gc = None
        return gc, gu0, gv0, None
