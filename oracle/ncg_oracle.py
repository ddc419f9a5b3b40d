"""Nonlinear conjugate gradients with a Wolfe-Powell line search on the FP64
oracle (TEST INFRASTRUCTURE ONLY: the reference of the device optimiser;
the product never imports it).

Section 2.4, Remark after Step 6, item 2: D_0 = -G_0, D_k = -G_k +
r_{k-1} D_{k-1}, with r by the Fletcher-Reeves, Polak-Ribiere,
Hestenes-Stiefel or Dai-Yuan rule, and a step along D_k satisfying the Wolfe
conditions.  The printed update z_{k+1} = z_k - zeta_k D_k would step uphill
along D_0 = -G_0; the update taken here is c_{k+1} = c_k + zeta_k D_k.  A
soft reset (D = -G) is taken when D is not a descent direction or when
|<G_k, G_{k-1}>| >= 0.2 <G_k, G_k> (Powell).  The first trial step is the
minimiser of the quadratic model of J along D built from the sensitivity
(tangent-linear) solution P = F'(c) D (the LMA of the same Remark):
zeta = -(<u^N - u_t, P> + alpha <c, D>) / (<P, P> + alpha <D, D>).
Inner products are sums over the fluid nodes.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O


def _beta(rule, G, Gp, D):
    y = G - Gp
    if rule == "FR":
        return (G * G).sum() / (Gp * Gp).sum()
    if rule == "PR":
        return max(0.0, (G * y).sum() / (Gp * Gp).sum())
    if rule == "HS":
        dy = (D * y).sum()
        return max(0.0, (G * y).sum() / dy) if dy != 0.0 else 0.0
    if rule == "DY":
        dy = (D * y).sum()
        return (G * G).sum() / dy if dy != 0.0 else 0.0
    raise ValueError(rule)


def ncg(p, rule="PR", iters=3, c1=1e-4, c2=0.1, max_ls=12, control_on_u=False):
    """Returns the J history, the final control, the gradients and the
    steps.  Fields are float64 [ny, nx]; solids carry 0."""
    f = p.fluid

    def dot(a, b):
        return float((a * b)[f].sum())

    def evaluate(c):
        r = O.cost_gradient(p, control=c, control_on_u=control_on_u)
        return r["J"], r["grad"] * f

    def lma(c, D):
        P, _ = O.tlm(p, dc=D, control=c, control_on_u=control_on_u)
        uN = O.forward(p, control=c, control_on_u=control_on_u)["uN"]
        num = dot(uN - p.u_target, P) + p.alpha * dot(c, D)
        den = dot(P, P) + p.alpha * dot(D, D)
        return -num / den if den > 0 else 0.0

    c = p.control.copy() * f
    J, G = evaluate(c)
    hist, grads, steps = [J], [G.copy()], []
    D = -G
    Gp = None
    for k in range(iters):
        if k > 0:
            gg = dot(G, G)
            restart = abs(dot(G, Gp)) >= 0.2 * gg
            D = -G + (0.0 if restart else _beta(rule, G, Gp, D)) * D
            if not restart and dot(D, G) >= 0.0:
                D = -G
        dg0 = dot(D, G)
        z = lma(c, D)
        if not (z > 0.0 and math.isfinite(z)):
            z = 1.0 / max(math.sqrt(dot(D, D)), 1e-300)
        lo, hi, best, acc = 0.0, math.inf, None, None
        for _ in range(max_ls):
            Jz, Gz = evaluate(c + z * D)
            armijo = Jz <= J + c1 * z * dg0
            if armijo and (best is None or Jz < best[1]):
                best = (z, Jz, Gz)
            if not armijo:
                hi = z
            elif dot(Gz, D) < c2 * dg0:
                lo = z
            else:
                acc = (z, Jz, Gz)
                break
            z = 2.0 * z if math.isinf(hi) else 0.5 * (lo + hi)
        if acc is None:
            if best is None:
                raise RuntimeError("line search found no decrease")
            acc = best
        z, Jn, Gn = acc
        c = (c + z * D) * f
        Gp, G, J = G, Gn, Jn
        hist.append(J)
        grads.append(G.copy())
        steps.append(z)
    return {"J": hist, "control": c, "grads": grads, "steps": steps}
