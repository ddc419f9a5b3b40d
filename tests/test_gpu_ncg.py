"""Device nonlinear conjugate gradients (optim.ConjugateGradient: every field
operation in libmrt) against the FP64 oracle's conjugate gradients with the
same decisions (oracle/ncg_oracle.py)."""
import numpy as np
import pytest

from oracle import ncg_oracle as N
from paper_1908_03876_amd import inputs as I
from tests.gpu_util import rel_l2

pytestmark = pytest.mark.gpu


def _problem():
    return I.with_control_bump(I.masked_anisotropic_small(L=64, nsteps=40), amp=3.0,
                               sigma=8.0)


@pytest.mark.parametrize("rule", ["FR", "PR", "HS", "DY"])
def test_device_ncg_matches_oracle_f64(rule):
    """Three iterations in FP64 on the device: the same steps, costs and
    final control as the oracle (the discrete decisions coincide)."""
    import torch
    from paper_1908_03876_amd import optim
    from paper_1908_03876_amd.solver import DeviceProblem
    p = _problem()
    ref = N.ncg(p, rule=rule, iters=3)
    dp = DeviceProblem(p, dtype=torch.float64)
    out = optim.run(dp, rule, 3)
    print(rule, "J", out["J"], "oracle", ref["J"], "steps", out["zeta"], ref["steps"], flush=True)
    np.testing.assert_allclose(out["J"], ref["J"], rtol=1e-10)
    np.testing.assert_allclose(out["zeta"], ref["steps"], rtol=1e-8)
    c = out["control"][:, :dp.nx].double().cpu().numpy()
    assert rel_l2(c, ref["control"], p.fluid) <= 1e-9


def test_device_ncg_f32_reaches_oracle_cost():
    """FP32 on the device: the cost after three PR iterations within 1e-4 of
    the oracle's (single-precision states, same algorithm)."""
    import torch
    from paper_1908_03876_amd import optim
    from paper_1908_03876_amd.solver import DeviceProblem
    p = _problem()
    ref = N.ncg(p, rule="PR", iters=3)
    out = optim.run(DeviceProblem(p, dtype=torch.float32), "PR", 3)
    print("f32 J", out["J"], "oracle", ref["J"], flush=True)
    assert abs(out["J"][-1] - ref["J"][-1]) <= 1e-4 * abs(ref["J"][-1])


def _fields(p, seed, n):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((p.ny, p.nx)) * p.fluid for _ in range(n)]


@pytest.mark.parametrize("case", ["plain", "powell_restart", "not_descent"])
@pytest.mark.parametrize("rule", ["FR", "PR", "HS", "DY"])
def test_cg_direction_matches_reference(rule, case):
    """mrt_cg_direction (FP64): beta by the rule (the oracle's formula on
    the same fields), Powell's restart test, the descent check, the new
    direction and <D, G>, against numpy on the host."""
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.solver import DeviceProblem, Tape
    p = _problem()
    dp = DeviceProblem(p, dtype=torch.float64)
    tape = Tape(dp, 0)
    G, Gp, D = _fields(p, 7, 3)
    if case == "powell_restart":
        Gp = G + 0.3 * Gp              # <G, Gp> far from 0
    elif case == "not_descent":
        D = 40.0 * G + D               # -G + beta D points uphill for FR and PR
    f = p.fluid
    dot = lambda a, b: float((a * b)[f].sum())
    gg_old, dg_old = dot(Gp, Gp), dot(D, Gp)
    Dd = dp.field(D)
    r = abi.mrt_cg_direction(dp.struct, tape.handle, rule, False, dp.field(G), dp.field(Gp), Dd,
                             gg_old, dg_old)
    beta = N._beta(rule, G[f], Gp[f], D[f])
    restart = abs(dot(G, Gp)) >= 0.2 * dot(G, G)
    Dn = -G + (0.0 if restart else beta) * D
    if not restart and dot(Dn, G) >= 0.0:
        Dn, restart = -G, True
    print(rule, case, "beta", r["beta"], beta, "restart", r["restart"], restart, flush=True)
    assert r["restart"] == restart
    assert abs(r["gg"] - dot(G, G)) <= 1e-13 * dot(G, G)
    assert abs(r["beta"] - beta) <= 1e-12 * max(abs(beta), 1e-300)
    assert rel_l2(dp.host(Dd), Dn, f) <= 1e-13
    assert abs(r["dg"] - dot(Dn, G)) <= 1e-12 * abs(dot(Dn, G))
    assert r["dg"] < 0.0
    if case == "not_descent" and rule in ("FR", "PR"):
        assert restart
    if case == "powell_restart":
        assert restart
    # first iteration: D = -G
    r0 = abi.mrt_cg_direction(dp.struct, tape.handle, rule, True, dp.field(G), None, Dd, 0.0, 0.0)
    assert r0["restart"] and rel_l2(dp.host(Dd), -G, f) <= 1e-15
    tape.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_lma_step_matches_formula(prec):
    """mrt_lma_step = (<r, P> + alpha <c, d>) / (<P, P> + alpha <d, d>) over
    the fluid nodes, on random fields (FP64 1e-13, FP32 fields with FP64
    sums 1e-12 against the same sums of the rounded fields)."""
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.solver import DeviceProblem, Tape
    dtype = torch.float64 if prec == "f64" else torch.float32
    p = _problem()
    dp = DeviceProblem(p, dtype=dtype)
    tape = Tape(dp, 0)
    r, P, c, d = _fields(p, 11, 4)
    if prec == "f32":
        r, P, c, d = (x.astype(np.float32).astype(np.float64) for x in (r, P, c, d))
    f = p.fluid
    dot = lambda a, b: float((a * b)[f].sum())
    want = (dot(r, P) + p.alpha * dot(c, d)) / (dot(P, P) + p.alpha * dot(d, d))
    got = abi.mrt_lma_step(dp.struct, tape.handle, dp.field(c), dp.field(d), dp.field(r),
                           dp.field(P))
    assert abs(got - want) <= 1e-12 * abs(want)
    tape.close()
