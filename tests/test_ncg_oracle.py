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


def _triples():
    """(G_k, G_{k-1}, D_{k-1}) triples: random ones, and the gradients of a
    nonlinear run (first direction D_0 = -G_0, then a perturbed one)."""
    rng = np.random.default_rng(17)
    out = []
    for _ in range(4):
        G, Gp, D = (rng.standard_normal(300) for _ in range(3))
        out.append((G, Gp + 0.5 * G, D))
    p = I.tiny(L=8, nsteps=12, seed=5)
    run = N.ncg(p, rule="PR", iters=2)
    f = p.fluid
    G0, G1, G2 = (g[f] for g in run["grads"])
    out.append((G1, G0, -G0))
    out.append((G2, G1, -G1 + 0.3 * G0))
    return out


def test_hestenes_stiefel_direction_is_conjugate():
    """Hestenes-Stiefel picks the multiple of the old direction that makes the
    new one conjugate to the gradient change, <D_k, G_k - G_{k-1}> = 0
    (wherever the rule is not clipped at zero)."""
    n = 0
    for G, Gp, D in _triples():
        y = G - Gp
        b = N._beta("HS", G, Gp, D)
        if b == 0.0:
            continue
        n += 1
        Dn = -G + b * D
        assert abs(Dn @ y) <= 1e-12 * np.linalg.norm(Dn) * np.linalg.norm(y)
    assert n >= 3


def test_dai_yuan_descent_identity():
    """Dai-Yuan: with D_k = -G_k + beta D_{k-1},
    <G_k, D_k> = beta <G_{k-1}, D_{k-1}> (the identity behind its descent
    property)."""
    for G, Gp, D in _triples():
        b = N._beta("DY", G, Gp, D)
        Dn = -G + b * D
        lhs, rhs = G @ Dn, b * (Gp @ D)
        assert abs(lhs - rhs) <= 1e-12 * (abs(G @ G) + abs(b * (G @ D)))


def test_polak_ribiere_differs_from_fletcher_reeves_by_the_overlap():
    """beta_FR - beta_PR = <G_k, G_{k-1}> / |G_{k-1}|^2 where PR is not
    clipped; the two agree only when successive gradients are orthogonal
    (as on a quadratic with exact line searches)."""
    n = 0
    for G, Gp, D in _triples():
        fr, pr = N._beta("FR", G, Gp, D), N._beta("PR", G, Gp, D)
        assert fr > 0.0 and abs(fr * (Gp @ Gp) - G @ G) <= 1e-12 * (G @ G)
        if pr == 0.0:
            continue
        n += 1
        assert abs((fr - pr) - (G @ Gp) / (Gp @ Gp)) <= 1e-12 * fr
        assert abs(G @ Gp) > 1e-6 * np.linalg.norm(G) * np.linalg.norm(Gp)
        assert fr != pr
    assert n >= 3


def test_pr_and_hs_are_clipped_at_zero():
    """PR+ and HS+: a negative overlap with the gradient change gives
    beta = 0 (restart along -G); FR and DY are not clipped."""
    G = np.array([1.0, 0.0, 0.0])
    Gp = np.array([2.0, 0.5, 0.0])     # <G, G - Gp> = -1 < 0
    D = np.array([-1.0, -1.0, 0.0])    # <D, G - Gp> = 1.5 > 0
    assert N._beta("PR", G, Gp, D) == 0.0
    assert N._beta("HS", G, Gp, D) == 0.0
    assert N._beta("FR", G, Gp, D) > 0.0
    assert N._beta("DY", G, Gp, D) > 0.0
