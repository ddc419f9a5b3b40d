"""cost_gradient_noalloc, the allocation-free variant of cost_gradient for
callers that cannot allocate device memory: through the C-ABI, its scalars
and fields equal cost_gradient's bit for bit, on two calls in a row (the
second on a smaller lattice, so the shared static scratch is reused), in
both phases (cost and seed; gradient and norms) and both precisions."""
import numpy as np
import pytest

from paper_1908_03876_amd import inputs as I
from tests.test_gpu_parity import _ragged

pytestmark = pytest.mark.gpu

SCALARS = ("J", "J_track", "J_reg", "grad_inf", "grad_l2", "n_fluid")


def _both(prob, dtype):
    """Forward and adjoint once, then the two reductions with and without a
    tape on the same device buffers."""
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.solver import DeviceProblem, Tape

    dp = DeviceProblem(prob, dtype=dtype)
    tape = Tape(dp, -1)
    uN = dp.empty_field()
    gacc = dp.empty_field(torch.float64)
    seed_a, seed_b = dp.empty_field(), dp.empty_field()
    grad_a, grad_b = dp.empty_field(), dp.empty_field()
    # junk in the outputs the calls must overwrite (solid nodes included)
    for t in (seed_a, seed_b, grad_a, grad_b):
        t.fill_(7.0)
    c = dp.control
    abi.mrt_forward(dp.struct, tape.handle, dp.u0, dp.v0, c, None, uN, None)
    r1a = abi.cost_gradient(dp.struct, tape.handle, uN, dp.u_target, c, None, seed_a, None)
    r1b = abi.cost_gradient_noalloc(dp.struct, uN, dp.u_target, c, None, seed_b, None)
    abi.amrt_adjoint(dp.struct, tape.handle, dp.u0, dp.v0, c, seed_a, None, gacc, None, None)
    r2a = abi.cost_gradient(dp.struct, tape.handle, uN, dp.u_target, c, gacc, None, grad_a)
    r2b = abi.cost_gradient_noalloc(dp.struct, uN, dp.u_target, c, gacc, None, grad_b)
    torch.cuda.synchronize()
    out = {"r1": (r1a, r1b), "r2": (r2a, r2b),
           "seed": (dp.host(seed_a), dp.host(seed_b)),
           "grad": (dp.host(grad_a), dp.host(grad_b))}
    tape.close()
    return out


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_noalloc_cost_gradient_equals_tape_version(dtype_name):
    import torch
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    big = I.with_control_bump(I.masked_anisotropic_small(L=160, nsteps=24), amp=3.0)
    small = _ragged(32, 257, 19, 12, True, True)   # ragged, random 8% mask
    for prob in (big, small):
        print(f"noalloc {dtype_name} {prob.nx}x{prob.ny}", flush=True)
        o = _both(prob, dtype)
        for ph in ("r1", "r2"):
            a, b = o[ph]
            for k in SCALARS:
                assert a[k] == b[k], (ph, k, a[k], b[k])
        assert o["r1"][0]["n_fluid"] == int(prob.fluid.sum())
        assert o["r2"][0]["grad_l2"] > 0.0
        for f in ("seed", "grad"):
            a, b = o[f]
            assert np.array_equal(a, b), f
            assert np.all(a[~prob.fluid] == 0.0)


def test_noalloc_rejects_bad_arguments():
    """Missing pointers are MRT_EINVAL before any work is enqueued."""
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.solver import DeviceProblem

    dp = DeviceProblem(I.tiny(), dtype=torch.float32)
    with pytest.raises(abi.MrtError):
        abi.cost_gradient_noalloc(dp.struct, None, dp.u_target, dp.control)
    g = dp.empty_field(torch.float64)
    with pytest.raises(abi.MrtError):
        abi.cost_gradient_noalloc(dp.struct, dp.u0, dp.u_target, dp.control, g, None, None)
