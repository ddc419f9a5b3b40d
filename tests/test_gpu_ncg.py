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
