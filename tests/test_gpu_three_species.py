"""Three species on the device (u, the attractant v and a repulsive signal
w of the attraction-repulsion example (ARC)) against the FP64 oracle:
forward state of all three species, cost and AMRT gradient, general seeds
with the initial sensitivities, the tangent-linear model, the checkpointed
tape, and the TLM/AMRT identity at the 2048 x 2048 masked size."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1908_03876_amd import inputs as I
from tests.gpu_util import device_gradient, rel_l2
from tests.test_gpu_parity import _ragged

pytestmark = pytest.mark.gpu

TOL = {"f64": (1e-12, 1e-12), "f32": (1e-5, 1e-4)}


def _dtype(name):
    import torch
    return torch.float64 if name == "f64" else torch.float32


def _problem(name):
    if name == "periodic_control":
        p = I.with_control_bump(I.periodic_isotropic(), amp=5.0, sigma=8.0).copy(nsteps=120)
    elif name == "masked128":
        p = I.with_control_bump(I.masked_anisotropic_small(L=128, nsteps=80), amp=3.0)
    elif name == "ragged_masked_periodic":
        p = _ragged(32, 257, 19, 25, True, True)
    elif name == "walls_only":
        p = _ragged(33, 70, 45, 30, False, False)
    elif name == "single_site":
        p = _ragged(34, 1, 1, 7, True, False).copy(chi=0.8)
    else:
        raise KeyError(name)
    return I.with_repellent(p)


CASES = ["periodic_control", "masked128", "ragged_masked_periodic", "walls_only",
         "single_site"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", CASES)
def test_three_species_forward_and_gradient_parity(name, prec):
    p = _problem(name)
    print(f"case {name} {prec} {p.nx}x{p.ny} N={p.nsteps} three species", flush=True)
    ref = O.cost_gradient(p)
    fwd = O.forward(p, want_state=True)
    f = p.fluid
    if name != "single_site":
        # the repellent moves u in this case
        assert rel_l2(O.forward(p.copy(chi_w=0.0))["uN"], fwd["uN"], f) > 1e-6
    dev = device_gradient(p, _dtype(prec))
    ftol, gtol = TOL[prec]
    assert dev["state"].shape[0] == 3
    assert rel_l2(dev["uN"], fwd["uN"], f) <= ftol
    assert rel_l2(dev["vN"], fwd["vN"], f) <= ftol
    assert rel_l2(dev["state"], fwd["state"]) <= ftol
    assert rel_l2(dev["state"][2].sum(axis=0), fwd["wN"], f) <= ftol
    assert abs(dev["J"] - ref["J"]) <= max(ftol, 1e-13) * abs(ref["J"]) * 10
    assert rel_l2(dev["grad"], ref["grad"], f) <= gtol
    if p.solid is not None:
        s = p.solid != 0
        assert np.all(dev["state"][:, :, s] == 0) and np.all(dev["grad"][s] == 0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_three_species_adjoint_general_seed_and_initial_sensitivity(prec):
    p = I.with_repellent(_ragged(41, 96, 40, 20, False, True))
    rng = np.random.default_rng(5)
    f = p.fluid
    a = rng.standard_normal((p.ny, p.nx)) * f
    b = rng.standard_normal((p.ny, p.nx)) * f
    g, gu0, gv0 = O.adjoint(p, a, b)
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.solver import DeviceProblem, Tape
    dp = DeviceProblem(p, dtype=_dtype(prec))
    tape = Tape(dp, -1)
    abi.mrt_forward(dp.struct, tape.handle, dp.u0, dp.v0, dp.control, None, None, None)
    gacc = dp.empty_field(torch.float64)
    au0, av0 = dp.empty_field(), dp.empty_field()
    abi.amrt_adjoint(dp.struct, tape.handle, dp.u0, dp.v0, dp.control,
                     dp.field(a), dp.field(b), gacc, au0, av0)
    torch.cuda.synchronize()
    tol = TOL[prec][1]
    assert rel_l2(dp.host(gacc), g, f) <= tol
    assert rel_l2(dp.host(au0), gu0, f) <= tol
    assert rel_l2(dp.host(av0), gv0, f) <= tol
    tape.close()


@pytest.mark.parametrize("ckpt", [16, 7])
def test_three_species_checkpointed_equals_store_all_bitwise(ckpt):
    import torch
    p = _problem("masked128").copy(nsteps=70)
    a = device_gradient(p, torch.float32, ckpt_every=-1)
    b = device_gradient(p, torch.float32, ckpt_every=ckpt)
    assert np.array_equal(a["uN"], b["uN"])
    assert np.array_equal(a["grad"], b["grad"])


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("ckpt", [-1, 16])
def test_three_species_tlm_matches_oracle(prec, ckpt):
    from tests.test_gpu_tlm import _device_tlm, _directions
    p = _problem("masked128").copy(nsteps=70)
    dc, du0, dv0 = _directions(p, 3)
    ref_u, ref_v = O.tlm(p, dc=dc, du0=du0, dv0=dv0)
    du, dv = _device_tlm(p, _dtype(prec), ckpt, dc, du0, dv0)
    tol = {"f64": 1e-12, "f32": 1e-4}[prec]
    assert rel_l2(du, ref_u, p.fluid) <= tol
    assert rel_l2(dv, ref_v, p.fluid) <= tol


def test_three_species_tlm_adjoint_identity_full_size():
    """<a, du^N(dc)> = <g(a), dc> on the 2048 x 2048 masked workload with the
    repellent (FP32, store-all, N = 100)."""
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.solver import DeviceProblem, Tape
    p = I.with_control_bump(I.masked_anisotropic(L=2048, nsteps=100), amp=5.0, sigma=256.0)
    p = I.with_repellent(p)
    rng = np.random.default_rng(6)
    f = p.fluid
    a = rng.standard_normal((p.ny, p.nx)) * f
    dc = rng.standard_normal((p.ny, p.nx)) * f
    dp = DeviceProblem(p, dtype=torch.float32)
    tape = Tape(dp, -1)
    abi.mrt_forward(dp.struct, tape.handle, dp.u0, dp.v0, dp.control, None, None, None)
    duN = dp.empty_field()
    abi.mrt_tlm(dp.struct, tape.handle, dp.u0, dp.v0, dp.control, dp.field(dc), None, None,
                duN, None)
    g = dp.empty_field(torch.float64)
    abi.amrt_adjoint(dp.struct, tape.handle, dp.u0, dp.v0, dp.control, dp.field(a), None, g,
                     None, None)
    torch.cuda.synchronize()
    lhs = float((dp.host(duN) * a).sum())
    rhs = float((dp.host(g) * dc).sum())
    print(f"<a, duN> = {lhs:.9e}, <g, dc> = {rhs:.9e}", flush=True)
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)
    tape.close()


def test_three_species_rejected_where_not_supported():
    """The continuous adjoint and the batched engine take two species."""
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.batched import Batch
    from paper_1908_03876_amd.solver import DeviceProblem, Tape
    p = _problem("periodic_control").copy(nsteps=4)
    dp = DeviceProblem(p, dtype=torch.float32)
    tape = Tape(dp, -1)
    abi.mrt_forward(dp.struct, tape.handle, dp.u0, dp.v0, dp.control, None, None, None)
    with pytest.raises(abi.MrtError) as e:
        abi.mrt_cadjoint(dp.struct, tape.handle, dp.u0, dp.v0, dp.control, dp.empty_field(),
                         dp.empty_field(torch.float64))
    assert e.value.code == abi.MRT_EINVAL
    tape.close()
    with pytest.raises(abi.MrtError) as e:
        Batch([p], dtype=torch.float32, ckpt_every=-1)
    assert e.value.code == abi.MRT_EINVAL
