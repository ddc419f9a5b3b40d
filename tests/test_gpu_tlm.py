"""Tangent-linear model on the device (sensitivity LBE, LIBEG-V) against
the FP64 oracle's TLM, the discrete adjoint identity between the device TLM
and the device AMRT, the fluid-node dot product and axpby, and the step of
the linearised line minimisation (LMA, Section 2.4)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1908_03876_amd import inputs as I
from tests.gpu_util import rel_l2
from tests.test_gpu_parity import _problem

pytestmark = pytest.mark.gpu

# FP64 device: rounding only; FP32 device: the tolerance of derivatives
TOL = {"f64": 1e-12, "f32": 1e-4}
CASES = ["periodic_control", "masked128", "ragged_masked_periodic", "walls_only",
         "single_site"]


def _dtype(name):
    import torch
    return torch.float64 if name == "f64" else torch.float32


def _directions(p, seed):
    rng = np.random.default_rng(seed)
    f = p.fluid
    return (rng.standard_normal((p.ny, p.nx)) * f, 0.1 * rng.standard_normal((p.ny, p.nx)) * f,
            0.1 * rng.standard_normal((p.ny, p.nx)) * f)


def _device_tlm(p, dtype, ckpt_every, dc, du0, dv0):
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.solver import DeviceProblem, Tape
    dp = DeviceProblem(p, dtype=dtype)
    tape = Tape(dp, ckpt_every)
    uN = dp.empty_field()
    abi.mrt_forward(dp.struct, tape.handle, dp.u0, dp.v0, dp.control, None, uN, None)
    duN, dvN = dp.empty_field(), dp.empty_field()
    abi.mrt_tlm(dp.struct, tape.handle, dp.u0, dp.v0, dp.control, dp.field(dc), dp.field(du0),
                dp.field(dv0), duN, dvN)
    torch.cuda.synchronize()
    out = dp.host(duN), dp.host(dvN)
    tape.close()
    return out


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", CASES)
def test_tlm_matches_oracle(name, prec):
    """du^N, dv^N for a random direction (dc, du0, dv0) against the oracle."""
    p = _problem(name)
    if name == "periodic_control":
        p = p.copy(nsteps=120)
    print(f"case {name} {prec} {p.nx}x{p.ny} N={p.nsteps}", flush=True)
    dc, du0, dv0 = _directions(p, 3)
    ref_u, ref_v = O.tlm(p, dc=dc, du0=du0, dv0=dv0)
    du, dv = _device_tlm(p, _dtype(prec), -1, dc, du0, dv0)
    f = p.fluid
    assert rel_l2(du, ref_u, f) <= TOL[prec]
    assert rel_l2(dv, ref_v, f) <= TOL[prec]
    if p.solid is not None:
        s = p.solid != 0
        assert np.all(du[s] == 0) and np.all(dv[s] == 0)


def test_tlm_checkpointed_equals_store_all_bitwise():
    """Segment-by-segment re-recording reproduces the stored trajectory."""
    import torch
    p = I.with_control_bump(I.masked_anisotropic_small(L=128, nsteps=70), amp=3.0)
    dc, du0, dv0 = _directions(p, 4)
    a = _device_tlm(p, torch.float32, -1, dc, du0, dv0)
    b = _device_tlm(p, torch.float32, 16, dc, du0, dv0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_tlm_then_adjoint_on_one_checkpointed_forward():
    """A TLM sweep re-records every segment; the adjoint sweep that follows
    on the same tape still gives the oracle gradient."""
    import torch
    from paper_1908_03876_amd.solver import DeviceProblem, GradientIteration
    p = I.with_control_bump(I.masked_anisotropic_small(L=128, nsteps=60), amp=3.0)
    ref = O.cost_gradient(p)
    dp = DeviceProblem(p, dtype=torch.float64)
    it = GradientIteration(dp, ckpt_every=16)
    it.forward()
    dc, _, _ = _directions(p, 5)
    it.tlm(dc=dp.field(dc))
    it.gradient()
    torch.cuda.synchronize()
    assert rel_l2(dp.host(it.grad), ref["grad"], p.fluid) <= 1e-12
    it.close()


@pytest.mark.parametrize("L,nsteps", [(128, 200), (2048, 100)])
def test_device_tlm_adjoint_identity(L, nsteps):
    """<a, du^N(dc)> = <g(a), dc> between the device TLM and the device AMRT
    (FP32, store-all), up to the cost of the 2048 x 2048 masked workload:
    the discrete adjoint identity at sizes the oracle cannot run."""
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.solver import DeviceProblem, Tape
    p = I.with_control_bump(I.masked_anisotropic(L=L, nsteps=nsteps) if L > 256 else
                            I.masked_anisotropic_small(L=L, nsteps=nsteps), amp=5.0,
                            sigma=L / 8)
    rng = np.random.default_rng(6)
    f = p.fluid
    a = rng.standard_normal((p.ny, p.nx)) * f
    dc = rng.standard_normal((p.ny, p.nx)) * f
    dp = DeviceProblem(p, dtype=torch.float32)
    tape = Tape(dp, -1)
    at, dct = dp.field(a), dp.field(dc)
    abi.mrt_forward(dp.struct, tape.handle, dp.u0, dp.v0, dp.control, None, None, None)
    duN = dp.empty_field()
    abi.mrt_tlm(dp.struct, tape.handle, dp.u0, dp.v0, dp.control, dct, None, None, duN, None)
    g = dp.empty_field(torch.float64)
    abi.amrt_adjoint(dp.struct, tape.handle, dp.u0, dp.v0, dp.control, at, None, g, None, None)
    torch.cuda.synchronize()
    lhs = float((dp.host(duN) * a).sum())
    rhs = float((dp.host(g) * dc).sum())
    print(f"L={L}: <a, duN> = {lhs:.9e}, <g, dc> = {rhs:.9e}", flush=True)
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)
    tape.close()


def test_dot_and_axpby():
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.solver import DeviceProblem, Tape
    p = I.masked_anisotropic_small(L=128, nsteps=10)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((p.ny, p.nx)) * p.fluid
    y = rng.standard_normal((p.ny, p.nx)) * p.fluid
    for dtype in (torch.float64, torch.float32):
        dp = DeviceProblem(p, dtype=dtype)
        tape = Tape(dp, 0)
        xt, yt = dp.field(x), dp.field(y)
        d = abi.mrt_dot(dp.struct, tape.handle, xt, yt)
        xr, yr = dp.host(xt), dp.host(yt)
        assert abs(d - float((xr * yr)[p.fluid].sum())) <= 1e-12 * abs(d)
        abi.mrt_axpby(dp.struct, tape.handle, xt, yt, 0.5, -2.0)
        torch.cuda.synchronize()
        exp = np.where(p.fluid, 0.5 * xr - 2.0 * yr, 0.0)
        tol = 1e-15 if dtype == torch.float64 else 1e-6
        np.testing.assert_allclose(dp.host(yt), exp, rtol=0, atol=tol * np.abs(exp).max())
        tape.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_lma_step_matches_oracle(prec):
    """The LMA step size from the device gradient, TLM and dot products
    against the same formula on the oracle's gradient and TLM."""
    import torch
    from paper_1908_03876_amd.solver import DeviceProblem, GradientIteration
    p = I.with_control_bump(I.masked_anisotropic_small(L=128, nsteps=80), amp=3.0)
    ref = O.cost_gradient(p)
    E = ref["grad"]
    P, _ = O.tlm(p, dc=E)
    f = p.fluid
    uN = O.forward(p)["uN"]
    num = ((uN - p.u_target) * P)[f].sum() + p.alpha * (p.control * E)[f].sum()
    den = (P * P)[f].sum() + p.alpha * (E * E)[f].sum()
    z_ref = num / den
    dp = DeviceProblem(p, dtype=_dtype(prec))
    it = GradientIteration(dp, ckpt_every=-1)
    it.gradient()
    z = it.lma_zeta()
    print(f"{prec}: zeta {z:.12e} oracle {z_ref:.12e}", flush=True)
    assert abs(z - z_ref) <= (1e-10 if prec == "f64" else 1e-4) * abs(z_ref)
    it.close()
