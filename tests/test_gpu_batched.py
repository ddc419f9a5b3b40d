"""Batched form: uneven-size instances advanced by persistent launches,
graph-captured iterations and autotuned launch shapes, each instance checked
against the oracle's gradient iteration (Section 3.2.1)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1908_03876_amd import inputs as I
from tests.gpu_util import rel_l2

pytestmark = pytest.mark.gpu


def _problems(nsteps=30, sizes=(64, 128, 192, 64, 256, 128), n=6, seed=44):
    ps = I.uneven_batch(seed=seed, n=n, nsteps=nsteps, sizes=sizes)
    return [I.with_control_bump(p, seed=100 + k, amp=2.0) for k, p in enumerate(ps)]


def _batch(ps, dtype, **kw):
    from paper_1908_03876_amd.batched import Batch
    return Batch(ps, dtype=dtype, **kw)


def _grads(b):
    return [b.get(k, "grad").double().cpu().numpy() for k in range(b.count)]


def _controls(b):
    return [b.get(k, "control").double().cpu().numpy() for k in range(b.count)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_iteration_matches_oracle(prec, graph):
    """Each instance's cost, gradient and updated control equal the oracle's
    one gradient iteration (FP64 1e-12; FP32 1e-5 fields, 1e-4 gradients)."""
    import torch
    dtype = torch.float64 if prec == "f64" else torch.float32
    ps = _problems()
    b = _batch(ps, dtype)
    b.iterate(use_graph=graph)
    sc = b.scalars()
    grads, ctrls = _grads(b), _controls(b)
    ftol, gtol = (1e-12, 1e-12) if prec == "f64" else (1e-5, 1e-4)
    for k, p in enumerate(ps):
        ref = O.cost_gradient(p)
        assert abs(sc[k]["J"] - ref["J"]) <= 10 * ftol * abs(ref["J"]), k
        assert rel_l2(b.get(k, "uN").double().cpu().numpy(), ref["uN"]) <= ftol, k
        assert rel_l2(grads[k], ref["grad"]) <= gtol, k
        c_ref, z_ref = O.gd_step(p.control, ref["grad"])
        assert abs(sc[k]["zeta"] - z_ref) <= gtol * z_ref, k
        assert rel_l2(ctrls[k], c_ref) <= gtol, k
    b.close()


def test_batch_large_instances_checkpointed_match_oracle():
    """The benchmark's launch configuration on its largest instance sizes:
    1024^2 and 768^2 (with 384^2 and 128^2) in one batch, checkpoints every
    5 of N = 24 steps (a ragged last segment), autotuned tiles, two
    graph-replayed iterations; every instance's cost, u^N, gradient and
    updated control against the oracle's two gradient iterations (FP32)."""
    import torch
    sizes = (1024, 768, 384, 128)
    ps = [I.with_control_bump(I.uneven_batch(seed=45 + k, n=1, nsteps=24, sizes=(L,))[0],
                              seed=100 + k, amp=2.0) for k, L in enumerate(sizes)]
    b = _batch(ps, torch.float32, ckpt_every=5)
    print(f"batch {[p.nx for p in ps]} N=24 K=5 tiles {b.tune(steps=4)}", flush=True)
    refs = [[], []]
    ctrl = [p.control.copy() for p in ps]
    for it in range(2):
        b.iterate(use_graph=True)
        sc = b.scalars()
        grads, ctrls = _grads(b), _controls(b)
        for k, p in enumerate(ps):
            q = p.copy(control=ctrl[k])
            ref = O.cost_gradient(q)
            c_ref, z_ref = O.gd_step(ctrl[k], ref["grad"])
            eg = rel_l2(grads[k], ref["grad"])
            print(f"  iteration {it} L={p.nx}: rel L2 grad {eg:.2e}", flush=True)
            assert abs(sc[k]["J"] - ref["J"]) <= 1e-5 * abs(ref["J"]), (it, k)
            assert rel_l2(b.get(k, "uN").double().cpu().numpy(), ref["uN"]) <= 1e-5, (it, k)
            assert eg <= 1e-4, (it, k)
            assert abs(sc[k]["zeta"] - z_ref) <= 1e-4 * z_ref, (it, k)
            assert rel_l2(ctrls[k], c_ref) <= 1e-4, (it, k)
            ctrl[k] = ctrls[k]  # the next iteration starts from the device's control
    b.close()


def test_batch_graph_replays_equal_eager_iterations():
    """Graph replays, with eager device work and synchronisations between
    them, reproduce eager iterations bit for bit, iteration after iteration."""
    import torch
    ps = _problems(nsteps=24)
    a = _batch(ps, torch.float32)
    g = _batch(ps, torch.float32)
    for it in range(3):
        a.iterate(use_graph=False)
        g.iterate(use_graph=True)
        x = torch.randn(1 << 20, device="cuda")
        _ = float((x * x).sum())  # unrelated eager work between replays
        torch.cuda.synchronize()
        sa, sg = a.scalars(), g.scalars()
        for k in range(len(ps)):
            assert sa[k]["J"] == sg[k]["J"] and sa[k]["grad_l2"] == sg[k]["grad_l2"], (it, k)
        for ca, cg in zip(_controls(a), _controls(g)):
            assert np.array_equal(ca, cg), it
    # J decreases along the gradient iterations for every instance
    a.close()
    g.close()


def test_batch_checkpointed_equals_record_all():
    """Checkpointed recomputation inside the persistent adjoint launch
    reproduces the recorded trajectory exactly."""
    import torch
    ps = _problems(nsteps=40)
    full = _batch(ps, torch.float32, ckpt_every=0)
    ck = _batch(ps, torch.float32, ckpt_every=7)
    full.iterate(use_graph=False)
    ck.iterate(use_graph=True)
    for x, y in zip(_grads(full), _grads(ck)):
        assert np.array_equal(x, y)
    full.close()
    ck.close()


def test_batch_tile_shapes_and_autotuner():
    """Every tile shape and residency computes identical node values; the
    autotuner returns one of them with a positive time per step."""
    import torch
    ps = _problems(nsteps=20)
    ref = None
    b = _batch(ps, torch.float32)
    mx = b.tiles()["max_blocks_per_cu"]
    for tw, bpc in ((64, 1), (128, 2), (256, mx), (64, mx)):
        b2 = _batch(ps, torch.float32)
        b2.set_tiles(tw, bpc)
        b2.iterate(use_graph=True)
        g = _grads(b2)
        if ref is None:
            ref = g
        else:
            for x, y in zip(ref, g):
                assert np.array_equal(x, y), (tw, bpc)
        b2.close()
    best = b.tune(steps=8)
    assert best["tile_w"] in (64, 128, 256) and 1 <= best["blocks_per_cu"] <= mx
    assert best["ms_per_step"] > 0
    assert b.tiles()["tile_w"] == best["tile_w"]
    b.iterate(use_graph=True)
    for x, y in zip(ref, _grads(b)):
        assert np.array_equal(x, y)
    b.close()


def test_batch_descent_over_iterations():
    """Repeated graph-replayed gradient steps lower every instance's cost."""
    import torch
    ps = _problems(nsteps=30)
    b = _batch(ps, torch.float64)
    js = []
    for _ in range(4):
        b.iterate(use_graph=True)
        js.append([s["J"] for s in b.scalars()])
    js = np.array(js)
    assert np.all(js[-1] < js[0])
    b.close()


def test_batch_barrier_timeout_is_reported():
    """Failure path of the persistent launch, forced from the host with a
    zero wait limit: the launch terminates and the error is reported."""
    import torch
    from paper_1908_03876_amd import abi
    ps = _problems(nsteps=10, sizes=(64, 128), n=3)
    b = _batch(ps, torch.float32)
    b.set_timeout(0.0)
    b.iterate(use_graph=False)
    with pytest.raises(abi.MrtError) as e:
        b.scalars()
    assert e.value.code == abi.MRT_EHIP
    b.close()


def _forward_batch(n=160, L=64, nsteps=12, seed=45):
    ps = I.uneven_batch(seed=seed, n=n, nsteps=nsteps, sizes=(L,))
    return [I.with_control_bump(p, seed=300 + k, amp=3.0) for k, p in enumerate(ps)]


def test_batch_forward_only_at_full_occupancy_matches_oracle():
    """The forward-only path launches as many work-groups as the occupancy
    query allows (160 instances of 64^2 give 2560 tiles, more than 256 CUs x
    8 resident work-groups), so every work-group must really be resident for
    the grid barrier to complete; u^N of sampled instances equals the
    oracle's forward (FP32 1e-5) and differs between instances."""
    import torch
    ps = _forward_batch()
    b = _batch(ps, torch.float32, ckpt_every=-1)
    t = b.tiles()
    assert t["tile_w"] * (256 // t["tile_w"]) == 256
    b.forward()
    outs = {k: b.get(k, "uN").double().cpu().numpy() for k in (0, 1, 77, len(ps) - 1)}
    for k, uN in outs.items():
        ref = O.forward(ps[k])["uN"]
        assert rel_l2(uN, ref) <= 1e-5, k
    assert np.abs(outs[0] - outs[1]).max() > 1e-3
    b.close()


def test_batch_forward_timeout_is_reported():
    """The forward-only path reports a grid-barrier time-out (forced from the
    host with a zero wait limit) instead of returning stale outputs."""
    import torch
    from paper_1908_03876_amd import abi
    ps = _forward_batch(n=4, nsteps=6)
    b = _batch(ps, torch.float32, ckpt_every=-1)
    b.set_timeout(0.0)
    with pytest.raises(abi.MrtError) as e:
        b.forward()
    assert e.value.code == abi.MRT_EHIP
    b.close()
