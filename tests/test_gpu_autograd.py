"""The AMRT sweep as the backward of a torch.autograd.Function with
checkpointed recomputation (differentiation form of the method: the discrete
adjoint gives the exact gradient of a functional of the final state,
Theorem 3)."""

import numpy as np
import pytest

from oracle import oracle as O
from paper_1908_03876_amd import inputs as I
from tests.gpu_util import rel_l2

pytestmark = pytest.mark.gpu


def _loss(uN, ut, c, alpha):
    return 0.5 * ((uN - ut) ** 2).sum() + 0.5 * alpha * (c ** 2).sum()


def _copy128(nsteps):
    """The 128 x 128 copy of the long-horizon masked workload."""
    return I.with_control_bump(I.long_horizon(L=128, nsteps=nsteps), amp=2.0, sigma=16.0)


def _torch_grad(p, dtype, ckpt_every, control=None):
    import torch
    from paper_1908_03876_amd.autograd import MRTSolve
    s = MRTSolve(p, dtype=dtype, ckpt_every=ckpt_every)
    c0 = p.control if control is None else control
    c = torch.tensor(c0, dtype=dtype, device="cuda", requires_grad=True)
    ut = torch.tensor(p.u_target, dtype=dtype, device="cuda")
    fluid = torch.tensor(p.fluid, device="cuda")
    uN, vN = s(c)
    loss = _loss(uN * fluid, ut * fluid, c, p.alpha)
    loss.backward()
    out = {"loss": float(loss), "grad": c.grad.double().cpu().numpy(),
           "uN": uN.detach().double().cpu().numpy(), "solver": s}
    return out


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_autograd_gradient_matches_oracle(dtype_name):
    """dloss/dc from loss.backward() equals the oracle's discrete gradient
    (FP64 device 1e-12, FP32 device 1e-4 relative L2)."""
    import torch
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    p = _copy128(600)
    ref = O.cost_gradient(p)
    out = _torch_grad(p, dtype, ckpt_every=64)
    f = p.fluid
    tol = 1e-12 if dtype_name == "f64" else 1e-4
    assert rel_l2(out["grad"], ref["grad"], f) <= tol
    assert abs(out["loss"] - ref["J"]) <= (1e-12 if dtype_name == "f64" else 1e-5) * ref["J"]
    out["solver"].close()


@pytest.mark.parametrize("variant", ["implicit_source", "three_species"])
def test_autograd_variants_match_oracle(variant):
    """loss.backward() through the implicit second-order source term and
    through the three-species scheme, with checkpointed recomputation,
    against the oracle's discrete gradient (FP64 device)."""
    import torch
    p = _copy128(300)
    p = p.copy(source_term=3) if variant == "implicit_source" else I.with_repellent(p)
    ref = O.cost_gradient(p)
    out = _torch_grad(p, torch.float64, ckpt_every=64)
    assert rel_l2(out["grad"], ref["grad"], p.fluid) <= 1e-12
    assert abs(out["loss"] - ref["J"]) <= 1e-12 * ref["J"]
    out["solver"].close()


def test_autograd_checkpoint_interval_is_exact():
    """Different checkpoint intervals recompute the same trajectory: the
    gradients are bitwise identical (memory bounded by the interval)."""
    import torch
    p = _copy128(700)
    a = _torch_grad(p, torch.float32, ckpt_every=700)   # one segment
    b = _torch_grad(p, torch.float32, ckpt_every=33)
    c = _torch_grad(p, torch.float32, ckpt_every=100)
    assert np.array_equal(a["grad"], b["grad"]) and np.array_equal(a["grad"], c["grad"])
    for o in (a, b, c):
        o["solver"].close()


def test_autograd_second_forward_before_backward():
    """Two forwards then two backwards: the backward of the first re-records
    its trajectory instead of using the second one's."""
    import torch
    from paper_1908_03876_amd.autograd import MRTSolve
    p = _copy128(300)
    s = MRTSolve(p, dtype=torch.float64, ckpt_every=50)
    c1 = torch.tensor(p.control, dtype=torch.float64, device="cuda", requires_grad=True)
    c2 = torch.tensor(p.control * 0.5, dtype=torch.float64, device="cuda", requires_grad=True)
    ut = torch.tensor(p.u_target, dtype=torch.float64, device="cuda")
    fl = torch.tensor(p.fluid, device="cuda")
    l1 = _loss(s(c1)[0] * fl, ut * fl, c1, p.alpha)
    l2 = _loss(s(c2)[0] * fl, ut * fl, c2, p.alpha)
    l1.backward()
    l2.backward()
    r1 = O.cost_gradient(p)
    r2 = O.cost_gradient(p, control=p.control * 0.5)
    f = p.fluid
    assert rel_l2(c1.grad.cpu().numpy(), r1["grad"], f) <= 1e-12
    assert rel_l2(c2.grad.cpu().numpy(), r2["grad"], f) <= 1e-12
    s.close()


def test_autograd_gradient_is_a_copy_not_the_solver_buffer():
    """FP64, a loss in which the control enters only through the solve: the
    gradient autograd stores is a tensor of its own, so a second backward
    after zero_grad(set_to_none=False) gives the same gradient (not twice
    it), and a backward without zeroing accumulates exactly once more."""
    import torch
    from paper_1908_03876_amd.autograd import MRTSolve
    p = _copy128(40)
    s = MRTSolve(p, dtype=torch.float64, ckpt_every=16)
    c = torch.tensor(p.control, dtype=torch.float64, device="cuda", requires_grad=True)
    ut = torch.tensor(p.u_target, dtype=torch.float64, device="cuda")
    fl = torch.tensor(p.fluid, device="cuda")

    def backward_once():
        uN, _ = s(c)
        (0.5 * (((uN - ut) * fl) ** 2).sum()).backward()

    backward_once()
    g1 = c.grad.clone()
    assert c.grad.data_ptr() != s._g.data_ptr()
    assert g1.abs().max() > 0
    c.grad.zero_()
    backward_once()
    assert torch.equal(c.grad, g1)
    backward_once()
    assert torch.equal(c.grad, 2.0 * g1)
    ref = O.cost_gradient(p.copy(alpha=0.0))
    assert rel_l2(g1.cpu().numpy(), ref["grad"], p.fluid) <= 1e-12
    s.close()


def test_autograd_initial_state_gradient():
    """Gradients w.r.t. u0 and v0 through the equilibrium initialisation,
    against the oracle's adjoint."""
    import torch
    from paper_1908_03876_amd.autograd import MRTSolve
    # slow kinetics and a short horizon: with b_v = 1 the chemical forgets v0
    # within a step (dJ/dv0 ~ 1e-50, pure rounding noise on both sides)
    p = _copy128(40).copy(r_u=0.05, a_uv=0.05, b_v=0.05)
    s = MRTSolve(p, dtype=torch.float64, ckpt_every=8)
    c = torch.tensor(p.control, dtype=torch.float64, device="cuda")
    u0 = torch.tensor(p.u0, dtype=torch.float64, device="cuda", requires_grad=True)
    v0 = torch.tensor(p.v0, dtype=torch.float64, device="cuda", requires_grad=True)
    rng = np.random.default_rng(2)
    a = torch.tensor(rng.standard_normal((p.ny, p.nx)) * p.fluid, device="cuda")
    b = torch.tensor(rng.standard_normal((p.ny, p.nx)) * p.fluid, device="cuda")
    uN, vN = s(c, u0, v0)
    ((uN * a).sum() + (vN * b).sum()).backward()
    g, gu0, gv0 = O.adjoint(p, a.cpu().numpy(), b.cpu().numpy())
    f = p.fluid
    assert np.abs(gv0).max() > 1e-3  # a sensitivity that is not noise
    assert rel_l2(u0.grad.cpu().numpy(), gu0, f) <= 1e-12
    assert rel_l2(v0.grad.cpu().numpy(), gv0, f) <= 1e-12
    s.close()


def test_autograd_finite_differences_long_horizon():
    """Central differences (eps = 1e-3, 32 random directions) of the loss
    at the full 10000-step horizon on the 128 x 128 copy, in FP64 on the
    device, agree with the AMRT directional derivatives."""
    import torch
    from paper_1908_03876_amd.autograd import MRTSolve
    p = _copy128(10000)
    s = MRTSolve(p, dtype=torch.float64, ckpt_every=100)
    ut = torch.tensor(p.u_target, dtype=torch.float64, device="cuda")
    fl = torch.tensor(p.fluid, device="cuda")
    c = torch.tensor(p.control, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = _loss(s(c)[0] * fl, ut * fl, c, p.alpha)
    loss.backward()
    g = c.grad.clone()
    eps = 1e-3
    errs = []
    with torch.no_grad():
        for k in range(32):
            h = torch.tensor(I.random_direction(p, 100 + k), device="cuda")
            jp = _loss(s(c + eps * h)[0] * fl, ut * fl, c + eps * h, p.alpha)
            jm = _loss(s(c - eps * h)[0] * fl, ut * fl, c - eps * h, p.alpha)
            fd = float((jp - jm) / (2 * eps))
            ad = float((g * h).sum())
            errs.append(abs(fd - ad) / max(abs(fd), 1e-30))
    # central differences are O(eps^2) accurate; the map is smooth
    assert max(errs) < 1e-5, errs
    s.close()


def test_autograd_full_size_long_horizon_bounded_memory():
    """The 2048 x 2048 masked workload at N = 10000 (the store-all record
    would need ~475 GB): checkpoints every 100 steps keep the tape near
    35 GB, and two checkpoint intervals give bitwise identical gradients."""
    import torch
    from paper_1908_03876_amd.autograd import MRTSolve
    from paper_1908_03876_amd.solver import DeviceProblem, Tape
    p = I.with_control_bump(I.long_horizon(L=2048, nsteps=10000), amp=5.0, sigma=256.0)
    dp = DeviceProblem(p)
    assert Tape.bytes_needed(dp, 10000) > 400e9
    assert Tape.bytes_needed(dp, 100) < 40e9
    del dp
    grads = []
    for K in (100, 250):
        s = MRTSolve(p, dtype=torch.float32, ckpt_every=K)
        c = torch.tensor(p.control, dtype=torch.float32, device="cuda", requires_grad=True)
        ut = torch.tensor(p.u_target, dtype=torch.float32, device="cuda")
        fl = torch.tensor(p.fluid, device="cuda")
        loss = _loss(s(c)[0] * fl, ut * fl, c, p.alpha)
        loss.backward()
        assert torch.isfinite(c.grad).all()
        grads.append(c.grad.cpu().numpy())
        s.close()
        del s
        torch.cuda.empty_cache()
    assert np.array_equal(grads[0], grads[1])


def test_autograd_checkpointed_matches_oracle_2000_steps():
    """The 128 x 128 copy at N = 2000 with checkpoints every 100 steps (20
    recomputed segments): FP32 gradient from loss.backward() against the
    FP64 oracle gradient."""
    import torch
    p = _copy128(2000)
    ref = O.cost_gradient(p)
    out = _torch_grad(p, torch.float32, ckpt_every=100)
    assert out["solver"].tape.info.n_segments == 20
    assert rel_l2(out["grad"], ref["grad"], p.fluid) <= 1e-4
    assert abs(out["loss"] - ref["J"]) <= 1e-5 * ref["J"]
    out["solver"].close()


def _mem_available_gb():
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemAvailable:"):
                    return int(line.split()[1]) / 2 ** 20
    except OSError:
        pass
    return 0.0


@pytest.mark.skipif(_mem_available_gb() < 4.0,
                    reason="the checkpointed FP64 oracle at 10000 steps needs ~0.6 GB of "
                           "host memory; less than 4 GB available")
def test_autograd_long_horizon_matches_oracle():
    """The 128 x 128 copy at the full 10000-step horizon: FP32 device
    gradient (checkpoints every 100) against the FP64 oracle gradient
    (which recomputes its own trajectory from checkpoints every 100 steps:
    about a minute on 16 cores)."""
    import torch
    p = _copy128(10000)
    print("oracle gradient, 128x128, N = 10000", flush=True)
    ref = O.cost_gradient(p)
    out = _torch_grad(p, torch.float32, ckpt_every=100)
    e = rel_l2(out["grad"], ref["grad"], p.fluid)
    eu = rel_l2(out["uN"], ref["uN"], p.fluid)
    print(f"N = 10000: rel L2 uN {eu:.2e} grad {e:.2e}", flush=True)
    assert eu <= 1e-5
    assert e <= 1e-4
    assert abs(out["loss"] - ref["J"]) <= 1e-5 * ref["J"]
    out["solver"].close()


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_autograd_d3q19_matches_oracle(dtype_name):
    """loss.backward() through the D3Q19 solve (checkpointed every 4 steps)
    equals the D3Q19 oracle's discrete gradient, and the initial-state
    gradients its dJ/du0, dJ/dv0.  The box is non-periodic with random
    solids and b_v = 0.2: with b_v = 1 the first collision removes v0 and
    dJ/dv0 is zero."""
    import torch
    from oracle import oracle3d as O3
    from paper_1908_03876_amd.autograd import MRTSolve
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    p = I.ragged_3d(27, 24, 10, 8, 14, False, True)
    ref = O3.cost_gradient(p)
    f = p.fluid
    s = MRTSolve(p, dtype=dtype, ckpt_every=4)
    assert s.shape == (8, 10, 24)
    c = torch.tensor(p.control, dtype=dtype, device="cuda", requires_grad=True)
    u0 = torch.tensor(p.u0, dtype=dtype, device="cuda", requires_grad=True)
    v0 = torch.tensor(p.v0, dtype=dtype, device="cuda", requires_grad=True)
    ut = torch.tensor(p.u_target, dtype=dtype, device="cuda")
    fl = torch.tensor(f, device="cuda")
    uN, _ = s(c, u0, v0)
    loss = _loss(uN * fl, ut * fl, c, p.alpha)
    loss.backward()
    seed = (ref["uN"] - p.u_target) * f
    _, gu0, gv0 = O3.adjoint(p, seed)
    tol = 1e-12 if dtype_name == "f64" else 1e-4
    assert rel_l2(c.grad.double().cpu().numpy(), ref["grad"], f) <= tol
    assert rel_l2(u0.grad.double().cpu().numpy(), gu0, f) <= tol
    assert rel_l2(v0.grad.double().cpu().numpy(), gv0, f) <= tol
    assert abs(float(loss) - ref["J"]) <= (1e-12 if dtype_name == "f64" else 1e-5) * ref["J"]
    s.close()
