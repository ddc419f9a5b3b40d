"""Nonlinear conjugate gradients with a Wolfe-Powell line search for the
control problem (Section 2.4, Remark after Step 6, item 2):

    D_0 = -G_0,   D_k = -G_k + r_{k-1} D_{k-1},   c_{k+1} = c_k + zeta_k D_k,

with r from the Fletcher-Reeves (FR), Polak-Ribiere (PR), Hestenes-Stiefel
(HS) or Dai-Yuan (DY) rule and zeta_k a step satisfying the Wolfe
conditions.  A soft reset (D = -G) is taken when D is not a descent
direction or when consecutive gradients are far from orthogonal (Powell's
test).  The first trial step along D is the linearised line minimisation
(LMA) of the quadratic cost along D, from one tangent-linear solve.

Every field operation (forward MRT, AMRT, gradient, TLM, inner products,
updates) is a libmrt call; this module only takes the scalar decisions.
"""
from __future__ import annotations

import math
from typing import Dict, List

import torch

from . import abi
from .solver import DeviceProblem, GradientIteration

RULES = ("FR", "PR", "HS", "DY")


class ConjugateGradient:
    """Nonlinear CG on dp (the control is kept in the solver's buffers; the
    result is in `control`)."""

    def __init__(self, dp: DeviceProblem, rule: str = "PR", ckpt_every: int = -1,
                 c1: float = 1e-4, c2: float = 0.1, max_ls: int = 12, first_trial=None):
        """first_trial(cg, dg0) -> step or None: the first trial of the line
        search along cg.D from cg.c, given dg0 = <D, G> (default, or on None:
        the LMA step along D)."""
        if rule not in RULES:
            raise ValueError(f"rule must be one of {RULES}")
        self.dp, self.rule, self.c1, self.c2, self.max_ls = dp, rule, c1, c2, max_ls
        self.it = GradientIteration(dp, ckpt_every=ckpt_every)
        self.c = dp.control.clone()       # current control
        self.ct = dp.empty_field()        # trial control
        self.G = dp.empty_field()         # gradient at c
        self.Gt = dp.empty_field()        # gradient at the trial control
        self.D = dp.empty_field()         # search direction
        self.Gprev = dp.empty_field()     # gradient at the previous control
        self.gg_old = 0.0                 # <G_{k-1}, G_{k-1}>
        self.d_gold = 0.0                 # <D_{k-1}, G_{k-1}>
        self.k = 0
        self.evals = 0                    # forward + adjoint solves
        self.tlms = 0
        self.J = None
        self.restarts = 0
        self.first_trial = first_trial
        self.last_zeta = None             # the previous accepted step

    # -- helpers (library calls)
    def _dot(self, x, y) -> float:
        return abi.mrt_dot(self.dp.struct, self.it.tape.handle, x, y)

    def _axpby(self, x, y, a, b) -> None:
        abi.mrt_axpby(self.dp.struct, self.it.tape.handle, x, y, a, b)

    def _eval(self, ctrl, G_out) -> float:
        """J and gradient at ctrl (the tape then holds the forward at ctrl)."""
        r = self.it.gradient(control=ctrl)
        G_out.copy_(self.it.grad)
        self.evals += 1
        return r["J"]

    def _lma_along(self, ctrl) -> float:
        """Minimiser of the quadratic model of J(ctrl + zeta D) (LMA): with
        P = F'(ctrl) D, zeta = -(<u^N - u_t, P> + alpha <ctrl, D>) /
        (<P, P> + alpha <D, D>) (mrt_lma_step along D, negated since the
        step is taken along +D).  Needs the forward at ctrl on the tape."""
        P, _ = self.it.tlm(dc=self.D, control=ctrl)
        self.tlms += 1
        return -abi.mrt_lma_step(self.dp.struct, self.it.tape.handle, ctrl, self.D,
                                 self.it.seed, P)

    def start(self) -> float:
        self.J = self._eval(self.c, self.G)
        return self.J

    def iterate(self) -> Dict:
        """One CG iteration: new direction, Wolfe line search, update."""
        if self.J is None:
            self.start()
        # D <- -G + beta D with the rule's beta, Powell's restart test and
        # the descent check (mrt_cg_direction)
        r = abi.mrt_cg_direction(self.dp.struct, self.it.tape.handle, self.rule, self.k == 0,
                                 self.G, self.Gprev, self.D, self.gg_old, self.d_gold)
        gg, restart, dg0 = r["gg"], r["restart"], r["dg"]   # dg0 = phi'(0) < 0
        self.restarts += int(restart and self.k > 0)
        zeta, Jn = self._line_search(dg0)
        # accept: c <- c + zeta D (the trial buffer already holds it)
        self.Gprev.copy_(self.G)
        self.gg_old = gg
        self.d_gold = dg0
        self.c, self.ct = self.ct, self.c
        self.G, self.Gt = self.Gt, self.G
        self.J = Jn
        self.last_zeta = zeta
        self.k += 1
        return {"J": Jn, "zeta": zeta, "restart": restart}

    def _phi(self, zeta: float):
        """phi(zeta) = J(c + zeta D) and phi'(zeta) = <G(c + zeta D), D>;
        the trial control and its gradient stay in ct, Gt."""
        self.ct.copy_(self.c)
        self._axpby(self.D, self.ct, zeta, 1.0)
        J = self._eval(self.ct, self.Gt)
        return J, self._dot(self.Gt, self.D)

    def _line_search(self, dg0: float):
        """A step z with J(c + z D) <= J + c1 z phi'(0) (sufficient decrease)
        and phi'(z) >= c2 phi'(0) (curvature): bracket by doubling, then
        bisect; the first trial is the LMA step along D.  If the trial budget
        runs out, the best sufficient-decrease step found is taken."""
        J0 = self.J
        z = self.first_trial(self, dg0) if self.first_trial is not None else None
        if z is None:
            z = self._lma_along(self.c)
        if not (z > 0.0 and math.isfinite(z)):
            z = 1.0 / max(self._dot(self.D, self.D) ** 0.5, 1e-300)
        lo, hi = 0.0, math.inf
        best = None
        for _ in range(self.max_ls):
            Jz, dgz = self._phi(z)
            armijo = Jz <= J0 + self.c1 * z * dg0
            if armijo and (best is None or Jz < best[1]):
                best = (z, Jz)
            if not armijo:
                hi = z
            elif dgz < self.c2 * dg0:
                lo = z
            else:
                return z, Jz
            z = 2.0 * z if math.isinf(hi) else 0.5 * (lo + hi)
        if best is None:
            raise RuntimeError("line search found no decrease")
        zb, _ = best
        Jb, _ = self._phi(zb)  # leave the accepted step in ct / Gt
        return zb, Jb

    @property
    def control(self):
        return self.c

    def close(self) -> None:
        self.it.close()


def run(dp: DeviceProblem, rule: str, iters: int, ckpt_every: int = -1) -> Dict:
    """iters CG iterations from dp.control; J history and solve counts."""
    cg = ConjugateGradient(dp, rule=rule, ckpt_every=ckpt_every)
    hist: List[float] = [cg.start()]
    zetas: List[float] = []
    for _ in range(iters):
        r = cg.iterate()
        hist.append(r["J"])
        zetas.append(r["zeta"])
    torch.cuda.synchronize()
    out = {"J": hist, "zeta": zetas, "evals": cg.evals, "tlms": cg.tlms,
           "restarts": cg.restarts, "control": cg.control.clone()}
    cg.close()
    return out
