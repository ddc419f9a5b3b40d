"""Pins of the conjugate-gradient reference (oracle/ncg_oracle.py).

On an exactly quadratic problem (control on u, no reactions, chi = 0: the
state is linear in the control) the first trial step, the minimiser of the
quadratic model built from the sensitivity solution, is the exact line
minimum; conjugate gradients with exact line searches then produce
mutually orthogonal gradients, and the Fletcher-Reeves, Polak-Ribiere,
Hestenes-Stiefel and Dai-Yuan rules generate the same iterates.
"""
import numpy as np

from oracle import ncg_oracle as N
from paper_1908_03876_amd import inputs as I


def _quadratic():
    return I.tiny(L=8, nsteps=10, seed=9).copy(chi=0.0, r_u=0.0, a_uv=0.0, b_v=0.0)


def test_ncg_on_quadratic_is_linear_cg():
    p = _quadratic()
    f = p.fluid
    runs = {r: N.ncg(p, rule=r, iters=4, control_on_u=True) for r in ("FR", "PR", "HS", "DY")}
    ref = runs["FR"]
    for r, out in runs.items():
        np.testing.assert_allclose(out["J"], ref["J"], rtol=1e-10, err_msg=r)
    G = [g[f] for g in ref["grads"]]
    for i in range(len(G)):
        for j in range(i):
            cos = abs(G[i] @ G[j]) / (np.linalg.norm(G[i]) * np.linalg.norm(G[j]))
            assert cos < 1e-8, (i, j, cos)
    assert all(b < a for a, b in zip(ref["J"], ref["J"][1:]))


def test_ncg_beats_steepest_descent_with_exact_steps_on_quadratic():
    """Same number of exact line searches: CG reaches a lower cost than
    steepest descent (whose successive directions are orthogonal)."""
    from oracle import oracle as O
    p = _quadratic()
    f = p.fluid
    cg = N.ncg(p, rule="PR", iters=4, control_on_u=True)
    c = p.control.copy() * f
    for _ in range(4):
        E = O.cost_gradient(p, control=c, control_on_u=True)["grad"] * f
        P, _ = O.tlm(p, dc=E, control=c, control_on_u=True)
        uN = O.forward(p, control=c, control_on_u=True)["uN"]
        z = ((uN - p.u_target) * P)[f].sum() + p.alpha * (c * E)[f].sum()
        z /= (P * P)[f].sum() + p.alpha * (E * E)[f].sum()
        c = (c - z * E) * f
    J_sd = O.cost_gradient(p, control=c, control_on_u=True)["J"]
    assert cg["J"][-1] < J_sd


def test_ncg_decreases_nonlinear_problem():
    p = I.tiny(L=8, nsteps=12, seed=5)
    out = N.ncg(p, rule="PR", iters=3)
    assert all(b < a for a, b in zip(out["J"], out["J"][1:]))
