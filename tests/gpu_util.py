"""Helpers shared by the GPU tests: run the HIP path through the C-ABI and
compare it with the CPU oracle."""
import numpy as np


def rel_l2(a, b, mask=None):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if mask is not None:
        a, b = a[mask], b[mask]
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def device_gradient(prob, dtype, ckpt_every=-1, seed_v=None, want_adj0=False,
                    control=None):
    """Forward, cost, adjoint and gradient on the GPU for an inputs.Problem.
    Returns host arrays."""
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.solver import DeviceProblem, Tape

    dp = DeviceProblem(prob, dtype=dtype)
    c = dp.control if control is None else dp.field(control)
    tape = Tape(dp, ckpt_every)
    uN, vN = dp.empty_field(), dp.empty_field()
    state = dp.state_tensor()
    seed = dp.empty_field()
    gacc = dp.empty_field(torch.float64)
    grad = dp.empty_field()
    abi.mrt_forward(dp.struct, tape.handle, dp.u0, dp.v0, c, state, uN, vN)
    r1 = abi.cost_gradient(dp.struct, tape.handle, uN, dp.u_target, c, None,
                           seed, None)
    sv = None if seed_v is None else dp.field(seed_v)
    au0 = dp.empty_field() if want_adj0 else None
    av0 = dp.empty_field() if want_adj0 else None
    abi.amrt_adjoint(dp.struct, tape.handle, dp.u0, dp.v0, c, seed, sv, gacc,
                     au0, av0)
    r2 = abi.cost_gradient(dp.struct, tape.handle, uN, dp.u_target, c, gacc,
                           None, grad)
    torch.cuda.synchronize()
    out = {"uN": dp.host(uN), "vN": dp.host(vN), "seed": dp.host(seed),
           "gacc": dp.host(gacc), "grad": dp.host(grad), "J": r1["J"],
           "J_track": r1["J_track"], "J_reg": r1["J_reg"],
           "grad_inf": r2["grad_inf"], "grad_l2": r2["grad_l2"],
           "n_fluid": r1["n_fluid"],
           "state": state[:, :, :, : dp.nx].double().cpu().numpy()}
    if want_adj0:
        out["adj_u0"], out["adj_v0"] = dp.host(au0), dp.host(av0)
    tape.close()
    return out
