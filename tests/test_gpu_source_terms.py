"""Second-order source terms of the LBE on the device, against the FP64
oracle: the explicit characteristic difference (eq:LBEG with kappa_t = 1,
kappa_x = 0; source_term 2) and the implicit one (kappa_t = kappa_x = 1;
source_term 3).  Forward, cost and AMRT gradient, the adjoint's initial
sensitivities, the tangent-linear model, and the checkpointed tape (for the
explicit form, the previous step's kinetics saved beside each checkpoint and
restored for every recomputed segment).

Kinetics at rate 0.1 keep the two-step explicit rule stable (tau dPhi/dTheta
near -0.1); starting from u0 near 0.15, far below the logistic equilibrium,
keeps the kinetics changing over the run, so the second-order term moves the
solution well above the tolerances.  Each case checks that it does.  The
implicit form is also run at the workloads' rate 1, where it is stable."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1908_03876_amd import inputs as I
from tests.gpu_util import device_gradient, rel_l2
from tests.test_gpu_parity import _ragged

pytestmark = pytest.mark.gpu

TOL = {"f64": (1e-12, 1e-12), "f32": (1e-5, 1e-4)}
RATE = 0.1


def _dtype(name):
    import torch
    return torch.float64 if name == "f64" else torch.float32


def _problem(name, term=2):
    if name == "periodic_control":
        p = I.with_control_bump(I.periodic_isotropic(), amp=2.0, sigma=8.0).copy(nsteps=60)
    elif name == "masked128":
        p = I.with_control_bump(I.masked_anisotropic_small(L=128, nsteps=50), amp=3.0)
    elif name == "ragged_masked_periodic":
        p = _ragged(32, 257, 19, 25, True, True)
    elif name == "walls_only":
        p = _ragged(33, 70, 45, 30, False, False)
    elif name == "single_site":
        p = _ragged(34, 1, 1, 7, True, False).copy(chi=0.8)
    elif name != "masked128_rate1":
        raise KeyError(name)
    if name == "masked128_rate1":
        return I.with_control_bump(I.masked_anisotropic_small(L=128, nsteps=80),
                                   amp=3.0).copy(source_term=term)
    return I.slow_reaction(p, RATE).copy(source_term=term, u0=0.15 * p.u0)


CASES = ["periodic_control", "masked128", "ragged_masked_periodic", "walls_only",
         "single_site"]


PARITY = [(n, 2) for n in CASES] + [(n, 3) for n in CASES] + [("masked128_rate1", 3)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,term", PARITY)
def test_second_order_forward_and_gradient_parity(name, term, prec):
    p = _problem(name, term)
    print(f"case {name} {prec} {p.nx}x{p.ny} N={p.nsteps} source_term={term}", flush=True)
    ref = O.cost_gradient(p)
    fwd = O.forward(p, want_state=True)
    first = O.forward(p.copy(source_term=1))
    f = p.fluid
    # the second-order term matters in this case
    assert rel_l2(first["uN"], fwd["uN"], f) > (1e-3 if name != "masked128_rate1" else 1e-6)
    dev = device_gradient(p, _dtype(prec))
    ftol, gtol = TOL[prec]
    assert rel_l2(dev["uN"], fwd["uN"], f) <= ftol
    assert rel_l2(dev["vN"], fwd["vN"], f) <= ftol
    assert rel_l2(dev["state"], fwd["state"]) <= ftol
    assert abs(dev["J"] - ref["J"]) <= max(ftol, 1e-13) * abs(ref["J"]) * 10
    assert rel_l2(dev["grad"], ref["grad"], f) <= gtol
    if p.solid is not None:
        s = p.solid != 0
        assert np.all(dev["uN"][s] == 0) and np.all(dev["grad"][s] == 0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("term", [2, 3])
def test_second_order_adjoint_general_seed_and_initial_sensitivity(term, prec):
    """Seeds on both species (for the implicit form, transformed to the last
    state's sums by the node equation) and dJ/du0, dJ/dv0 (the step-0
    adjoint)."""
    q = _ragged(41, 96, 40, 20, False, True)
    p = I.slow_reaction(q, RATE).copy(source_term=term, u0=0.15 * q.u0)
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


@pytest.mark.parametrize("term,ckpt", [(2, 16), (2, 7), (3, 16)])
def test_second_order_checkpointed_equals_store_all_bitwise(term, ckpt):
    """Recomputed segments reproduce the stored trajectory (the explicit form
    restores the kinetics saved with each checkpoint), so the checkpointed
    gradient is the store-all one bit for bit."""
    import torch
    p = _problem("masked128", term)
    a = device_gradient(p, torch.float32, ckpt_every=-1)
    b = device_gradient(p, torch.float32, ckpt_every=ckpt)
    assert np.array_equal(a["uN"], b["uN"])
    assert np.array_equal(a["grad"], b["grad"])


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("term,ckpt", [(2, -1), (2, 16), (3, -1), (3, 16)])
def test_second_order_tlm_matches_oracle(term, ckpt, prec):
    from tests.test_gpu_tlm import _device_tlm, _directions
    p = _problem("masked128", term)
    dc, du0, dv0 = _directions(p, 3)
    ref_u, ref_v = O.tlm(p, dc=dc, du0=du0, dv0=dv0)
    du, dv = _device_tlm(p, _dtype(prec), ckpt, dc, du0, dv0)
    tol = {"f64": 1e-12, "f32": 1e-4}[prec]
    assert rel_l2(du, ref_u, p.fluid) <= tol
    assert rel_l2(dv, ref_v, p.fluid) <= tol


@pytest.mark.parametrize("term", [2, 3])
def test_batched_engine_rejects_second_order(term):
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.batched import Batch
    import torch
    ps = [I.periodic_isotropic().copy(nsteps=4, source_term=term)]
    with pytest.raises(abi.MrtError) as e:
        Batch(ps, dtype=torch.float32, ckpt_every=-1)
    assert e.value.code == abi.MRT_EINVAL


@pytest.mark.parametrize("term", [2, 3])
def test_second_order_tlm_adjoint_identity_full_size(term):
    """<a, du^N(dc)> = <g(a), dc> between the device TLM and the device AMRT
    of the second-order schemes on the 2048 x 2048 masked workload (FP32,
    store-all, N = 100): the discrete adjoint identity at a size the oracle
    cannot run."""
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.solver import DeviceProblem, Tape
    p = I.with_control_bump(I.masked_anisotropic(L=2048, nsteps=100), amp=5.0, sigma=256.0)
    p = I.slow_reaction(p, RATE).copy(source_term=term, u0=0.15 * p.u0)
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
