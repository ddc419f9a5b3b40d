"""Continuous-adjoint gradient on the device (Section 3.2.2: the continuous
adjoint system solved by the MRT scheme in reversed time) against the FP64
oracle's implementation of the same scheme, and its relation to the exact
discrete (AMRT) gradient at full size."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1908_03876_amd import inputs as I
from tests.gpu_util import rel_l2
from tests.test_gpu_parity import _problem
from tests.test_oracle_pins import _smooth_problem

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-4}


def _cases(name):
    if name == "smooth32":
        return _smooth_problem(32).copy(alpha=1e-3)
    return _problem(name)


def _device_cgrad(p, dtype, ckpt_every=-1):
    import torch
    from paper_1908_03876_amd.solver import DeviceProblem, GradientIteration
    dp = DeviceProblem(p, dtype=dtype)
    it = GradientIteration(dp, ckpt_every=ckpt_every)
    r = it.gradient_continuous()
    torch.cuda.synchronize()
    out = dp.host(it.grad), r
    it.close()
    return out


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", ["smooth32", "masked128", "ragged_masked_periodic",
                                  "walls_only"])
def test_cadjoint_matches_oracle(name, prec):
    import torch
    p = _cases(name)
    print(f"case {name} {prec} {p.nx}x{p.ny} N={p.nsteps}", flush=True)
    ref = O.cost_gradient_continuous(p)
    g, r = _device_cgrad(p, torch.float64 if prec == "f64" else torch.float32)
    assert rel_l2(g, ref["grad"], p.fluid) <= TOL[prec]
    assert abs(r["J"] - ref["J"]) <= max(TOL[prec], 1e-12) * abs(ref["J"])
    if p.solid is not None:
        assert np.all(g[p.solid != 0] == 0)


def test_cadjoint_checkpointed_equals_store_all_bitwise():
    import torch
    p = I.with_control_bump(I.masked_anisotropic_small(L=128, nsteps=70), amp=3.0)
    a, _ = _device_cgrad(p, torch.float32, -1)
    b, _ = _device_cgrad(p, torch.float32, 16)
    assert np.array_equal(a, b)


def test_cadjoint_full_size_tracks_discrete_gradient():
    """2048 x 2048 masked workload, N = 200, FP32: the continuous-adjoint
    gradient is an O(h^2, tau) approximation of the exact discrete one; on
    this rough, wall-dominated problem they stay strongly correlated."""
    import torch
    from paper_1908_03876_amd.solver import DeviceProblem, GradientIteration
    p = I.with_control_bump(I.masked_anisotropic(L=2048, nsteps=200), amp=5.0, sigma=256.0)
    dp = DeviceProblem(p, dtype=torch.float32)
    it = GradientIteration(dp, ckpt_every=-1)
    it.gradient()
    gd = dp.host(it.grad)
    it.gradient_continuous()
    gc = dp.host(it.grad)
    it.close()
    f = p.fluid
    corr = float(np.corrcoef(gd[f], gc[f])[0, 1])
    print(f"rel diff {rel_l2(gc, gd, f):.3e} correlation {corr:.5f}", flush=True)
    assert np.isfinite(gc).all() and corr > 0.9
