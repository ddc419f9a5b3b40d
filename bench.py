"""Benchmark: gradient iterations of the MRT/AMRT optimal-control hot path on
one MI355X.

Workload (masked anisotropic chemotaxis at scale, FP32): 2048 x 2048 lattice
with a bounce-back mask of 200 random disks (radius 5-30) plus a solid outer
ring, full anisotropic self and chemotactic tensors, N = 4000 time steps per
solve.  One timed step = one gradient iteration of Section 3.2.1: forward MRT
solve recording the adjoint tape, cost and adjoint seed, AMRT reverse sweep,
gradient and norms, gradient step on the control.  Inputs are seeded and
resident in HBM before timing starts.

Prints one JSON line.  value = coupled MRT+AMRT MLUPS
= fluid nodes * N / (seconds per gradient iteration) / 1e6.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# sources the single-lattice step kernels are compiled from: HBM counters
# taken on other sources are stale
KERNEL_SRCS = [os.path.join(ROOT, "paper_1908_03876_amd", "csrc", f)
               for f in ("mrt_kernels.hip", "mrt_device.h", "mrt_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.txt")
# the same for the D3Q19 step kernels
KERNEL3_SRCS = [os.path.join(ROOT, "paper_1908_03876_amd", "csrc", f)
                for f in ("mrt3_kernels.hip", "mrt3_internal.h", "mrt_device.h")]
TRAFFIC3_FILE = os.path.join(ROOT, "profiles", "d3q19_traffic_counters.txt")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash(srcs=None) -> str:
    h = hashlib.sha256()
    for path in (KERNEL_SRCS if srcs is None else srcs):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, L: int, path: str = None, srcs=None):
    """Calibrated HBM bytes per launch of `kernel` from the committed counter
    summary (`key = value` lines), or None when it is absent, taken on
    another workload size, or taken on other kernel sources."""
    path = TRAFFIC_FILE if path is None else path
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if "=" in line:
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_hash(srcs) or kv.get("L") != str(L):
        return None
    v = kv.get(kernel + ".hbm_bytes_per_launch")
    return int(v) if v is not None else None


def bytes_per_site(elem: int, source_term: int = 1, nspecies: int = 2):
    """Algorithmic HBM bytes per fluid node and step (the counts of the
    measurement plan: 148 forward, 160 with the record, 172 adjoint for two
    species in FP32):
    forward with record: 9 NS loads + 9 NS stores + control + record stores
    (u, j_v; and j_w with three species); adjoint: 9 NS + 9 NS + the record
    loads + FP64 gradient read-modify-write.  The explicit second-order
    source term adds a read and a write of two planes (the previous step's
    kinetics, or their adjoint) to both; the implicit one adds no traffic
    (the node solve is arithmetic).  The 2-byte link word every node reads
    is an overhead of the masked layout, reported on its own, not counted."""
    lag = 4 * elem if source_term == 2 else 0
    pops = 18 * nspecies * elem
    rec = (5 if nspecies == 3 else 3) * elem
    fwd = pops + elem + rec + lag
    adj = pops + rec + 16 + lag
    fwd_norec = pops + elem + lag
    return fwd, adj, fwd_norec


def _gomp():
    """The OpenMP runtime the oracle libraries are built against (g++
    -fopenmp links libgomp); its thread count is set here, in process."""
    import ctypes
    return ctypes.CDLL("libgomp.so.1")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_oracle(run, threads: int) -> float:
    """Seconds of run() with the oracle's OpenMP pool at `threads` (0: as
    configured), restoring the previous count afterwards."""
    gomp = _gomp()
    before = gomp.omp_get_max_threads()
    if threads > 0:
        gomp.omp_set_num_threads(threads)
    try:
        t0 = time.perf_counter()
        run()
        return time.perf_counter() - t0
    finally:
        gomp.omp_set_num_threads(before)


def cpu_baseline(L: int, steps: int):
    """Time the FP64 oracle (as it stands) on a bounded sample of the same
    workload: the full L x L masked problem for `steps` forward + adjoint
    steps on all configured threads, and for one step on one thread."""
    from oracle import oracle as O
    from paper_1908_03876_amd import inputs as I

    def problem(n):
        return I.with_control_bump(I.masked_anisotropic(L=L, nsteps=n), amp=5.0, sigma=L / 8)
    p = problem(steps)
    O.lib()
    threads = _gomp().omp_get_max_threads()
    dt = _time_oracle(lambda: O.cost_gradient(p), 0)
    p1 = problem(1)
    dt1 = _time_oracle(lambda: O.cost_gradient(p1), 1)
    return {"value": p.n_fluid * steps / dt / 1e6, "unit": "MLUPS",
            "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle forward+adjoint gradient, {L}x{L} masked "
                      f"anisotropic workload, {steps} steps ({dt:.1f} s)",
            "one_thread": {"value": p1.n_fluid / dt1 / 1e6, "unit": "MLUPS",
                           "sample": f"the same problem, 1 step on 1 thread ({dt1:.1f} s)"},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def bench_batched(args):
    """96 independent periodic problems, L in {128..1024} (seeded), N = 2000
    (or --nsteps if given below 2000), per-instance chi and tensors:
    graph-replayed gradient iterations of the batched persistent engine."""
    import torch
    from paper_1908_03876_amd import inputs as I
    from paper_1908_03876_amd.batched import Batch
    N = min(args.nsteps or 2000, 2000)
    ps = I.uneven_batch(seed=4, n=96, nsteps=N)
    sites = sum(p.nx * p.ny for p in ps)
    K = max(1, int(round((N * 6) ** 0.5)))
    log(f"[bench] batched: 96 instances, {sites} sites, N={N}, ckpt every {K}")
    b = Batch(ps, dtype=torch.float32, ckpt_every=K)
    best = b.tune(steps=30)
    log(f"[bench] autotuner: {best}")
    for w in range(max(args.warmup, 1)):
        b.iterate(use_graph=True)
        b.scalars()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    js = []
    for k in range(args.steps):
        b.iterate(use_graph=True)
        js.append(sum(s["J"] for s in b.scalars()))
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    # per site-step bytes (FP32, periodic, no mask): forward 18+18 planes +
    # control, with the record on the recomputed/last segment, adjoint 18+18
    # planes + 3 record loads + FP64 gradient read-modify-write
    fwd_b, rec_b, adj_b = 36 * 4 + 4, 36 * 4 + 4 + 12, 36 * 4 + 12 + 16
    bytes_it = sites * (N * fwd_b + N * rec_b + N * adj_b)
    out = {"metric": "batched coupled MRT+AMRT MLUPS (96 uneven instances)",
           "value": round(sites * N / (ms / 1e3) / 1e6, 1), "unit": "MLUPS",
           "ms_per_iteration": round(ms, 1), "iterations": args.steps,
           "instances": 96, "sites": sites, "nsteps": N, "ckpt_every": K,
           "tiles": best, "algorithmic_GBps_per_iteration": round(bytes_it / (ms / 1e3) / 1e9, 1),
           "hbm_frac": round(bytes_it / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
           "J_sum_history": [round(x, 4) for x in js]}
    b.close()
    # the streaming probe with each launch's access mix at this size: the
    # iteration's ceiling is its bytes over the sum of each part's bytes at
    # its own ceiling
    dev = torch.device("cuda:0")
    parts = [(19, 18, N * fwd_b), (19, 21, N * rec_b), (23, 20, N * adj_b)]
    t_ideal = 0.0
    ceil = {}
    for r, w, nb in parts:
        c = stream_ceiling(r, w, sites, dev)
        ceil[f"{r}+{w}"] = c["GBps"]
        t_ideal += sites * nb / (c["GBps"] * 1e9)
    out["stream_ceiling_GBps"] = ceil
    out["iteration_stream_ceiling_GBps"] = round(bytes_it / t_ideal / 1e9, 1)
    out["frac_of_stream_ceiling"] = round(t_ideal / (ms / 1e3), 4)
    print(json.dumps(out), flush=True)


def bench_autograd(args):
    """Differentiation form: the 2048^2 masked anisotropic problem at
    N = 10000, FP32, with the AMRT sweep as the backward of a
    torch.autograd.Function and checkpoints every 100 steps.  One step is
    forward, loss, loss.backward() (recomputing each segment from its
    checkpoint) and the gradient-descent update."""
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd import inputs as I
    from paper_1908_03876_amd.autograd import MRTSolve
    N = args.nsteps or 10000
    K = 100 if args.ckpt == "auto" else int(args.ckpt)
    p = I.with_control_bump(I.long_horizon(L=args.L, nsteps=N), amp=5.0, sigma=args.L / 8)
    log(f"[bench] autograd: {args.L}^2 N={N} checkpoints every {K}")
    s = MRTSolve(p, dtype=torch.float32, ckpt_every=K)
    info = s.tape.info
    n_fluid = s.tape.n_fluid
    dev = torch.device("cuda:0")
    c = torch.tensor(p.control, dtype=torch.float32, device=dev, requires_grad=True)
    ut = torch.tensor(p.u_target, dtype=torch.float32, device=dev)
    fl = torch.tensor(p.fluid, dtype=torch.float32, device=dev)

    def one():
        uN, _ = s(c)
        loss = 0.5 * (((uN - ut) * fl) ** 2).sum() + 0.5 * p.alpha * (c * c).sum()
        loss.backward()
        with torch.no_grad():
            g = c.grad
            c.sub_(min(1.0, 1.0 / float(g.abs().max())) * g)
            c.grad = None
        return float(loss)

    hist = [one() for _ in range(max(args.warmup, 1))]
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats(dev)
    abi.mrt_timing_reset()
    abi.mrt_timing_enable(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        hist.append(one())
        log(f"[bench] iter {k}: loss {hist[-1]:.6g}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    abi.mrt_timing_enable(False)
    ms = (t1 - t0) * 1e3 / args.steps
    f_ms, f_n = abi.mrt_timing_read(abi.TIMING_FORWARD)
    a_ms, a_n = abi.mrt_timing_read(abi.TIMING_ADJOINT)
    r_ms, r_n = abi.mrt_timing_read(abi.TIMING_RECOMPUTE)
    b_fwd, b_adj, b_norec = bytes_per_site(4)
    # forward without record, recomputation with record, adjoint
    bytes_it = N * n_fluid * (b_norec + b_fwd + b_adj)
    out = {"metric": "autograd MRT+AMRT MLUPS (forward + checkpointed backward)",
           "value": round(n_fluid * N / (ms / 1e3) / 1e6, 1), "unit": "MLUPS",
           "s_per_iteration": round(ms / 1e3, 3), "iterations": args.steps,
           "config": {"workload": f"masked anisotropic chemotaxis control, {p.nx}x{p.ny}, "
                                  f"N={N} steps, AMRT as autograd backward",
                      "fluid_nodes": n_fluid, "ckpt_every": int(info.ckpt_every),
                      "segments": int(info.n_segments),
                      "tape_gib": round(info.device_bytes / 2**30, 2),
                      "store_all_would_need_gib": round(
                          (N * 12 * p.nx * p.ny) / 2**30, 1)},
           "forward_mlups": round(n_fluid * f_n / (f_ms / 1e3) / 1e6, 1) if f_ms else None,
           "recompute_mlups": round(n_fluid * r_n / (r_ms / 1e3) / 1e6, 1) if r_ms else None,
           "adjoint_mlups": round(n_fluid * a_n / (a_ms / 1e3) / 1e6, 1) if a_ms else None,
           "algorithmic_GBps_per_iteration": round(bytes_it / (ms / 1e3) / 1e9, 1),
           "hbm_frac": round(bytes_it / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
           "torch_peak_gib": round(torch.cuda.max_memory_allocated(dev) / 2**30, 2),
           "loss_history": [round(x, 4) for x in hist]}
    s.close()
    print(json.dumps(out), flush=True)


def bench_lma(args):
    """Gradient iterations on the 2048^2 masked anisotropic problem (N = 4000,
    FP32, store-all) with two step rules from the same start: the heuristic
    zeta = min(1, 1/||E||_inf) and the linearised line minimisation (LMA),
    which costs one tangent-linear solve per iteration."""
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd import inputs as I
    from paper_1908_03876_amd.solver import DeviceProblem, GradientIteration
    N = args.nsteps or 4000
    prob = I.masked_anisotropic(L=args.L, nsteps=N)
    res = {"metric": "J after k iterations: heuristic gradient step, LMA gradient step "
                     "(one tangent-linear solve per iteration) and Polak-Ribiere "
                     "conjugate gradients with a Wolfe line search",
           "config": {"workload": f"masked anisotropic chemotaxis control, {args.L}x{args.L}, "
                                  f"N={N}, FP32, store-all tape"}}
    for rule in ("heuristic", "lma"):
        dp = DeviceProblem(prob, dtype=torch.float32)
        it = GradientIteration(dp, ckpt_every=N)
        hist, zetas = [], []
        it.step() if rule == "heuristic" else it.step_lma()  # warm-up iteration
        dp.control.copy_(dp.field(prob.control))
        torch.cuda.synchronize()
        abi.mrt_timing_reset()
        abi.mrt_timing_enable(True)
        t0 = time.perf_counter()
        for k in range(args.steps):
            r = it.step() if rule == "heuristic" else it.step_lma()
            hist.append(r["J"])
            zetas.append(r["zeta"])
            log(f"[bench] {rule} iter {k}: J={r['J']:.6g} zeta={r['zeta']:.4g}")
        r = it.gradient()
        hist.append(r["J"])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        abi.mrt_timing_enable(False)
        t_ms, t_n = abi.mrt_timing_read(abi.TIMING_TLM)
        res[rule] = {"s_per_iteration": round(dt, 4), "J_history": [round(x, 4) for x in hist],
                     "zeta": [float(f"{z:.5g}") for z in zetas]}
        if rule == "lma" and t_n:
            res[rule]["tlm_mlups"] = round(it.tape.n_fluid * t_n / (t_ms / 1e3) / 1e6, 1)
        it.close()
        del dp
        torch.cuda.empty_cache()
    # nonlinear conjugate gradients (Polak-Ribiere, Wolfe line search whose
    # first trial is the LMA step along the direction)
    from paper_1908_03876_amd import optim
    dp = DeviceProblem(prob, dtype=torch.float32)
    cg = optim.ConjugateGradient(dp, rule="PR", ckpt_every=N)
    hist = [cg.start()]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    zetas = []
    for k in range(args.steps):
        r = cg.iterate()
        hist.append(r["J"])
        zetas.append(r["zeta"])
        log(f"[bench] ncg-PR iter {k}: J={r['J']:.6g} zeta={r['zeta']:.4g}")
    torch.cuda.synchronize()
    res["ncg_pr"] = {"s_per_iteration": round((time.perf_counter() - t0) / args.steps, 4),
                     "J_history": [round(x, 4) for x in hist],
                     "zeta": [float(f"{z:.5g}") for z in zetas],
                     "gradient_solves": cg.evals, "tlm_solves": cg.tlms}
    cg.close()
    j0 = res["heuristic"]["J_history"][0]
    dh = max(j0 - res["heuristic"]["J_history"][-1], 1e-300)
    res["J_decrease_ratio_lma_over_heuristic"] = round((j0 - res["lma"]["J_history"][-1]) / dh, 1)
    res["J_decrease_ratio_ncg_over_heuristic"] = round((j0 - res["ncg_pr"]["J_history"][-1]) / dh, 1)
    print(json.dumps(res), flush=True)


def bench_cadjoint(args):
    """The continuous-adjoint gradient (Section 3.2.2) against the exact
    discrete AMRT gradient on the 2048^2 masked problem (N = 4000, FP32,
    store-all): time per gradient and the relative difference."""
    import torch
    import numpy as np
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd import inputs as I
    from paper_1908_03876_amd.solver import DeviceProblem, GradientIteration
    N = args.nsteps or 4000
    prob = I.with_control_bump(I.masked_anisotropic(L=args.L, nsteps=N), amp=5.0,
                               sigma=args.L / 8)
    dp = DeviceProblem(prob, dtype=torch.float32)
    it = GradientIteration(dp, ckpt_every=N)
    out = {"metric": "continuous-adjoint vs discrete AMRT gradient",
           "config": {"workload": f"masked anisotropic chemotaxis control, {args.L}x{args.L}, "
                                  f"N={N}, FP32, store-all tape"}}
    grads = {}
    for name, fn in (("discrete", it.gradient), ("continuous", it.gradient_continuous)):
        fn()
        torch.cuda.synchronize()
        abi.mrt_timing_reset()
        abi.mrt_timing_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        abi.mrt_timing_enable(False)
        kind = abi.TIMING_ADJOINT if name == "discrete" else abi.TIMING_CADJ
        ms, n = abi.mrt_timing_read(kind)
        grads[name] = dp.host(it.grad)
        out[name] = {"s_per_gradient": round(dt, 4),
                     "sweep_mlups": round(it.tape.n_fluid * n / (ms / 1e3) / 1e6, 1)}
    f = prob.fluid
    d, c = grads["discrete"][f], grads["continuous"][f]
    out["rel_l2_difference"] = float(f"{np.linalg.norm(c - d) / np.linalg.norm(d):.4e}")
    out["correlation"] = round(float(np.corrcoef(d, c)[0, 1]), 6)
    it.close()
    print(json.dumps(out), flush=True)


# FLOP per pixel of the surrogate: the two 32 -> 32 layers (2 * 9 * 32 * 32
# each, on the matrix cores) and the one-channel first and last layers
# (2 * 9 * 32 each, vector ALU)
SRG_C32_FLOP = 2 * 9 * 32 * 32
SRG_THIN_FLOP = 2 * 9 * 32


def bench_srg_kernels(args):
    """Throughput of the surrogate's kernels in its two uses: training steps
    on 64 crops of 64 x 64 (forward, backward with weight gradients, Adam)
    and candidate scoring on 17 fields of 1024 x 1024 (forward only)."""
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd.surrogate import Surrogate
    dev = torch.device("cuda:0")
    srg = Surrogate(17, 1024, 1024, seed=0)
    g = torch.Generator(device=dev).manual_seed(0)
    out = {"metric": "surrogate network throughput (BF16 MFMA, FP32 accumulation)"}
    # scoring: forward of 17 fields of 1024^2
    x = torch.randn((17, 1024, 1024), generator=g, device=dev)
    y = torch.empty_like(x)
    for _ in range(2):
        abi.mrt_srg_forward(srg.handle, x, y, 17, 1024, 1024)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = max(args.steps, 1)
    for _ in range(reps):
        abi.mrt_srg_forward(srg.handle, x, y, 17, 1024, 1024)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    pix = 17 * 1024 * 1024
    flop = pix * (2 * SRG_C32_FLOP + 2 * SRG_THIN_FLOP)
    out["forward_17x1024x1024"] = {"ms": round(ms, 3), "TFLOP_s": round(flop / ms / 1e9, 1)}
    # training steps: 64 crops of 64 x 64
    xb = torch.randn((64, 64, 64), generator=g, device=dev)
    tb = 0.01 * torch.randn((64, 64, 64), generator=g, device=dev)
    for _ in range(3):
        abi.mrt_srg_train_step(srg.handle, xb, tb, 64, 64, 64, 4, 1e-4)
    e0.record()
    reps_t = 50 * reps
    for _ in range(reps_t):
        abi.mrt_srg_train_step(srg.handle, xb, tb, 64, 64, 64, 4, 1e-4)
    e1.record()
    torch.cuda.synchronize()
    ms_t = e0.elapsed_time(e1) / reps_t
    pix_t = 64 * 64 * 64
    # forward + backward data + weight gradients
    flop_t = pix_t * 3 * (2 * SRG_C32_FLOP + 2 * SRG_THIN_FLOP)
    out["train_step_64x64x64"] = {"ms": round(ms_t, 3), "TFLOP_s": round(flop_t / ms_t / 1e9, 1)}
    out["peak_bf16_dense_TFLOP_s"] = 2500.0
    srg.close()
    print(json.dumps(out), flush=True)


def bench_surrogate(args):
    """Surrogate-assisted loop against three plain loops: MRT-generated
    training pairs on 256^2 (N = 1000), crop training, then on 256^2 and
    1024^2 problems with reachable (hidden-control) targets, each plain loop
    (golden-section line search warm-started from the previous step, LMA
    step, Polak-Ribiere CG) for a fixed number of iterations from c = 0, and
    the assisted loop until it reaches the lowest of their costs; the wall
    time each loop takes to reach each plain loop's final cost within 1e-3."""
    import torch
    from paper_1908_03876_amd import surrogate as SG
    N, L = 1000, 256
    n_pairs = int(os.environ.get("MRT_SRG_PAIRS", "20000"))
    iters = args.steps if args.steps < 20 else 10
    t0 = time.perf_counter()
    data = SG.generate_pairs(n_pairs, L, N, seed=5, per_launch=96)
    t_gen = time.perf_counter() - t0
    log(f"[bench] {n_pairs} pairs in {t_gen:.1f} s: render {data['render_s']:.2f} s, "
        f"copies {data['copy_s']:.2f} s, MRT {data['solve_s']:.1f} s "
        f"({data['solve_glups']:.1f} GLUPS)")
    var = float(((data["responses"] - data["u_base"][None]) ** 2).mean())
    srg = SG.Surrogate(32, 1024, 1024, seed=0)
    t0 = time.perf_counter()
    hist = srg.train(data["controls"][:-64], data["responses"][:-64], steps=3000,
                     batch=64, crop=64, border=4, lr=2e-3, seed=1, log_every=500,
                     u_base=data["u_base"])
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    held = srg.loss(data["controls"][-64:-48], data["responses"][-64:-48],
                    sub=data["u_base"])
    log(f"[bench] trained in {t_train:.1f} s: loss {hist} held-out {held:.3e} (var {var:.3e})")
    res = {"metric": "wall time to each plain loop's final cost within 1e-3: "
                     "surrogate-assisted loop vs golden-section, LMA and PR-CG loops",
           "config": {"workload": f"periodic isotropic chemotaxis control, hidden-control "
                                  f"targets, N={N}, FP32; network trained on {n_pairs} "
                                  f"(control, u(T)) pairs of {L}^2"},
           "pairs": n_pairs, "pair_gen_s": round(t_gen, 1),
           "pair_gen": {"render_s": round(data["render_s"], 2), "copy_s": round(data["copy_s"], 2),
                        "mrt_s": round(data["solve_s"], 1),
                        "mrt_glups": round(data["solve_glups"], 1)},
           "train_s": round(t_train, 1), "train_loss": hist, "heldout_mse": held,
           "response_var": var, "plain_iterations": iters, "problems": []}
    loops = (("golden", SG.optimize_plain), ("lma", SG.optimize_lma), ("cg_pr", SG.optimize_cg))
    for size in (256, 1024):
        prob, _ = SG.hidden_target_problem(size, N, seed=9 + size, amax=2.0)
        base = data["u_base"][0, 0].item()
        ub = torch.full((size, size), base, dtype=torch.float32, device="cuda")
        # one untimed pass of every loop first (kernel and graph set-up)
        for _, fn in loops:
            cp = SG.ControlProblem(prob)
            fn(cp, 1)
            cp.close()
        for fn in (lambda cp: SG.optimize_assisted(cp, srg, ub, -math.inf, max_iters=1),
                   lambda cp: SG.optimize_assisted_cg(cp, srg, ub, -math.inf, max_iters=1)):
            cp = SG.ControlProblem(prob)
            fn(cp)
            cp.close()
        row = {"L": size, "plain": {}}
        for name, fn in loops:
            cp = SG.ControlProblem(prob)
            r = fn(cp, iters)
            cp.close()
            tgt = r["J"] * (1 + 1e-3)
            row["plain"][name] = {"J": r["J"], "time_s": round(r["time"], 4),
                                  "time_to_target_s": round(SG.time_to_reach(r, tgt), 4),
                                  "solves": r["solves"], "J_history": r["hist"]}
            log(f"[bench] L={size} {name}: J {r['hist'][0]:.5g} -> {r['J']:.5g} in "
                f"{r['time']:.3f} s, {r['solves']} solves")
        target = min(v["J"] for v in row["plain"].values()) * (1 + 1e-3)
        # the assisted loop (surrogate warm start, then PR-CG), the same with
        # the surrogate's curvature steps as the first line-search trials, and
        # the gradient loop with surrogate steps
        assisted = (("assisted", lambda cp: SG.optimize_assisted_cg(cp, srg, ub, target)),
                    ("assisted_surrogate_steps",
                     lambda cp: SG.optimize_assisted_cg(cp, srg, ub, target, proposals=True)),
                    ("assisted_gd", lambda cp: SG.optimize_assisted(cp, srg, ub, target,
                                                                    max_iters=40)))
        row["assisted_loops"] = {}
        for name, fn in assisted:
            cp = SG.ControlProblem(prob)
            a = fn(cp)
            cp.close()
            rec = {"J": a["J"], "time_s": round(a["time"], 4), "solves": a["solves"],
                   "J_history": a["hist"], "times": [round(t, 4) for t in a["times"]],
                   "vs": {}}
            log(f"[bench] L={size} {name}: J {a['hist'][0]:.5g} -> {a['J']:.5g} in "
                f"{a['time']:.3f} s, {a['solves']} solves")
            for pname, v in row["plain"].items():
                t_a = SG.time_to_reach(a, v["J"] * (1 + 1e-3))
                rec["vs"][pname] = {"reached": t_a is not None,
                                    "time_to_target_s": None if t_a is None else round(t_a, 4),
                                    "speedup": None if t_a is None
                                    else round(v["time_to_target_s"] / t_a, 2)}
                log(f"[bench] L={size} {name} vs {pname}: {rec['vs'][pname]}")
            row["assisted_loops"][name] = rec
        res["problems"].append(row)
    srg.close()
    res["all_reached"] = all(v["reached"] for r in res["problems"]
                             for v in r["assisted_loops"]["assisted"]["vs"].values())
    print(json.dumps(res), flush=True)
    if not res["all_reached"]:
        raise SystemExit("assisted loop did not reach every plain loop's cost")


def traffic_rate(traffic, avg_ms):
    """HBM GB/s from the counter bytes per launch over the measured launch
    time, and its fraction of the peak (empty without counter figures)."""
    if traffic is None:
        return {}
    gbs = traffic / (avg_ms / 1e3) / 1e9
    return {"traffic_GBps": round(gbs, 1), "traffic_frac": round(gbs / HBM_PEAK_GBS, 4)}


def stream_ceiling(reads: int, writes: int, n: int, dev):
    """Bandwidth of the library's streaming probe (mrt_stream_probe) with a
    step kernel's access mix, `reads` + `writes` FP32 planes of n nodes with
    the kernels' non-temporal loads and stores, in both tile orders (launch
    order and XCD-banded), each timed with events on the stream it runs on
    (mean of 20 launches after 3).  The better order's bandwidth is the
    practical ceiling of that mix on this GPU.  Runs after the timed
    region."""
    import torch
    from paper_1908_03876_amd import abi
    inp = torch.ones(reads * n, dtype=torch.float32, device=dev)
    out = torch.empty(writes * n, dtype=torch.float32, device=dev)
    per = {}
    for order in (0, 1):
        for _ in range(3):
            abi.mrt_stream_probe(reads, writes, inp, out, n, order=order)
        k = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            abi.mrt_stream_probe(reads, writes, inp, out, n, order=order)
        e1.record()
        torch.cuda.synchronize()
        per[order] = e0.elapsed_time(e1) / k
    del inp, out
    torch.cuda.empty_cache()
    best = min(per, key=per.get)
    ms = per[best]
    gbs = 4.0 * n * (reads + writes) / (ms / 1e3) / 1e9
    return {"GBps": round(gbs, 1), "avg_ms": round(ms, 5),
            "order": "XCD-banded" if best == 1 else "launch order",
            "GBps_by_order": {"launch": round(4.0 * n * (reads + writes) / per[0] / 1e6, 1),
                              "banded": round(4.0 * n * (reads + writes) / per[1] / 1e6, 1)},
            "mix": f"{reads} read + {writes} write FP32 planes of {n} nodes, non-temporal"}


def add_stream_ceiling(roof: dict, reads: int, writes: int, n: int, dev):
    """The probe's bandwidth beside the roofline, and the dominant kernel's
    algorithmic (and counted) bandwidth as fractions of it."""
    c = stream_ceiling(reads, writes, n, dev)
    roof["stream_ceiling"] = c
    roof["frac_of_stream_ceiling"] = round(roof["achieved"] / c["GBps"], 4)
    if roof.get("traffic_GBps"):
        roof["traffic_frac_of_stream_ceiling"] = round(roof["traffic_GBps"] / c["GBps"], 4)


def copy_calibration(out: dict, dev):
    """A plain 1 GiB device copy: the reference of the byte counters, and the
    bandwidth the runtime's own copy reaches (HIP events, best of 3)."""
    import torch
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    best = None
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    out["copy_calibration_bytes"] = {"read": 4 * n, "write": 4 * n}
    out["copy_GBps"] = round(8 * n / (best / 1e3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()


def bytes_per_site3(elem: int):
    """Algorithmic HBM bytes per fluid node and step on D3Q19 (two species):
    forward with record: 38 loads + 38 stores + control + record stores (u,
    j_v: 4 values); adjoint: 38 + 38 + the record loads + FP64 gradient
    read-modify-write.  The link word (read only by wavefronts next to a
    wall) is not counted."""
    pops = 2 * 2 * 19 * elem
    fwd = pops + elem + 4 * elem
    adj = pops + 4 * elem + 16
    fwd_norec = pops + elem
    return fwd, adj, fwd_norec


def cpu_baseline3(L: int, steps: int, L1: int = 96):
    """Time the FP64 D3Q19 oracle (as it stands) on the full L^3 masked
    problem for `steps` forward + adjoint steps on all configured threads,
    and on the L1^3 problem of the same recipe for one step on one thread."""
    from oracle import oracle3d as O3
    from paper_1908_03876_amd import inputs as I
    p = I.masked_3d(seed=8, L=L, nsteps=steps)
    O3.lib()
    threads = _gomp().omp_get_max_threads()
    dt = _time_oracle(lambda: O3.cost_gradient(p), 0)
    p1 = I.masked_3d(seed=8, L=L1, nsteps=1)
    dt1 = _time_oracle(lambda: O3.cost_gradient(p1), 1)
    return {"value": p.n_fluid * steps / dt / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"FP64 D3Q19 oracle forward+adjoint gradient, {L}^3 masked porous "
                      f"workload, {steps} step(s) ({dt:.1f} s)",
            "one_thread": {"value": p1.n_fluid / dt1 / 1e6, "unit": "MLUPS",
                           "sample": f"{L1}^3 problem of the same recipe, 1 step on 1 thread "
                                     f"({dt1:.1f} s)"},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}


def bench_d3q19(args):
    """D3Q19 two-species MRT+AMRT gradient iterations on the L^3 porous
    workload (seeded solid spheres about 9% of the volume plus a solid
    frame, seeded anisotropic 3x3 tensors), FP32, N steps per solve."""
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd import inputs as I
    from paper_1908_03876_amd.solver3 import DeviceProblem3, GradientIteration3
    L = args.L3
    N = args.nsteps or 200
    dev = torch.device("cuda:0")
    log(f"[bench] d3q19: building workload L={L} N={N}")
    prob = I.masked_3d(seed=8, L=L, nsteps=N)
    dp = DeviceProblem3(prob, dtype=torch.float32, device=dev)
    free, _ = torch.cuda.mem_get_info(dev)
    if args.ckpt == "auto":
        K = N if abi.mrt3_tape_bytes(dp.struct, N) <= int(0.85 * free) else \
            max(1, int(round((N * 10) ** 0.5)))
    elif args.ckpt == "store":
        K = N
    else:
        K = int(args.ckpt)
    it = GradientIteration3(dp, ckpt_every=K)
    info = it.tape.info
    mode = {0: "forward-only", 1: "store-all", 2: "checkpointed"}[info.mode]
    n_fluid = it.tape.n_fluid
    log(f"[bench] tape {mode} K={info.ckpt_every} {info.device_bytes / 2**30:.1f} GiB, "
        f"fluid nodes {n_fluid}")
    hist = []
    for w in range(args.warmup):
        r = it.step()
        hist.append(r["J"])
        log(f"[bench] warmup {w}: J={r['J']:.6g} |E|inf={r['grad_inf']:.3g}")
    torch.cuda.synchronize()
    abi.mrt_timing_reset()
    abi.mrt_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = it.step()
        hist.append(r["J"])
        log(f"[bench] iter {k}: J={r['J']:.6g} |E|inf={r['grad_inf']:.3g} zeta={r['zeta']:.3g}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    abi.mrt_timing_enable(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    f_ms, f_n = abi.mrt_timing_read(abi.TIMING_FORWARD)
    a_ms, a_n = abi.mrt_timing_read(abi.TIMING_ADJOINT)
    r_ms, r_n = abi.mrt_timing_read(abi.TIMING_RECOMPUTE)
    value = n_fluid * N / (ms_step / 1e3) / 1e6
    b_fwd, b_adj, b_norec = bytes_per_site3(4)
    rec_share = 1.0 if info.mode == 1 else 1.0 / info.n_segments
    launch_bytes = {"mrt3_forward_step": n_fluid * (rec_share * b_fwd + (1 - rec_share) * b_norec),
                    "amrt3_adjoint_step": n_fluid * b_adj}
    kern = {"mrt3_forward_step": (f_ms, f_ms / max(f_n, 1)),
            "amrt3_adjoint_step": (a_ms, a_ms / max(a_n, 1))}
    dom = max(kern, key=lambda k: kern[k][0])
    avg_ms = kern[dom][1]
    achieved = launch_bytes[dom] / (avg_ms / 1e3) / 1e9
    traffic = read_traffic(dom, L, TRAFFIC3_FILE, KERNEL3_SRCS) if info.mode == 1 else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": dom, "avg_launch_ms": round(avg_ms, 5),
            "algorithmic_bytes_per_launch": int(launch_bytes[dom]),
            "other_kernel": {k: {"avg_launch_ms": round(kern[k][1], 5),
                                 "GBps": round(launch_bytes[k] / (kern[k][1] / 1e3) / 1e9, 1)}
                             for k in kern if k != dom and kern[k][0] > 0}}
    roof.update(traffic_rate(traffic, avg_ms))
    mix = (44, 40) if dom == "amrt3_adjoint_step" else (39, 42)
    add_stream_ceiling(roof, mix[0], mix[1], L * L * L, dev)
    out = {
        "metric": "coupled MRT+AMRT MLUPS (gradient iteration: forward + adjoint), "
                  "HBM GB/s fraction; s per gradient iteration",
        "value": round(value, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded spheres, tensors, targets)",
        "config": {"workload": f"porous anisotropic chemotaxis control, {L}^3 D3Q19 "
                               f"two-species MRT, solid spheres + frame, N={N} steps per "
                               f"solve, gradient-descent iterations",
                   "L": L, "nsteps": N, "fluid_nodes": n_fluid, "tape": mode,
                   "ckpt_every": int(info.ckpt_every),
                   "tape_gib": round(info.device_bytes / 2**30, 2),
                   "parallelism": "single GPU"},
        "s_per_iteration": round(ms_step / 1e3, 4),
        "forward_mlups": round(n_fluid * f_n / (f_ms / 1e3) / 1e6, 1) if f_ms else None,
        "adjoint_mlups": round(n_fluid * a_n / (a_ms / 1e3) / 1e6, 1) if a_ms else None,
        "recompute_launches": r_n,
        "J_history": [round(x, 6) for x in hist],
        "roofline": roof,
        "other_kernel": side,
    }
    it.close()
    del dp
    torch.cuda.empty_cache()
    if args.copy_calibration:
        copy_calibration(out, dev)
    if args.cpu_steps > 0:
        log(f"[bench] cpu baseline: D3Q19 oracle {L}^3 x 1 step")
        out["cpu_baseline"] = cpu_baseline3(L, 1)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed gradient iterations")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, default=2048)
    ap.add_argument("--L3", type=int, default=256, help="d3q19 workload: cube edge")
    ap.add_argument("--nsteps", type=int, default=None,
                    help="time steps per solve (default: 4000 masked, 10000 "
                         "autograd, 2000 batched)")
    ap.add_argument("--ckpt", default="auto",
                    help="auto | store | K (checkpoint every K steps)")
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="steps of the CPU-oracle sample (0 = skip)")
    ap.add_argument("--workload", default="masked",
                    choices=["masked", "autograd", "batched", "surrogate", "lma",
                             "cadjoint", "srg-kernels", "d3q19"],
                    help="masked: the 2048^2 masked anisotropic workload (the "
                         "reported line); autograd: the same problem at N = 10000 "
                         "through torch.autograd with checkpoints; batched: 96 "
                         "uneven periodic instances; lma: heuristic vs LMA step "
                         "sizes on the masked problem; cadjoint: continuous vs "
                         "discrete adjoint gradient; srg-kernels: surrogate "
                         "network throughput; d3q19: the two-species D3Q19 "
                         "path on a 256^3 porous workload; "
                         "surrogate: CNN-assisted vs plain loop")
    ap.add_argument("--source-term", type=int, default=1, choices=[1, 2, 3],
                    help="masked workload: 1 first-order source term; 2 second "
                         "order by the explicit characteristic difference (a "
                         "two-step rule that needs slower kinetics: the kinetics "
                         "rates are then 0.1); 3 second order by the implicit "
                         "characteristic difference (stable at the workload's "
                         "rates)")
    ap.add_argument("--species", type=int, default=2, choices=[2, 3],
                    help="masked workload: 3 adds the repulsive signal w of the "
                         "attraction-repulsion example (seeded tensors, "
                         "chi_w = -0.4)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy a 1 GiB buffer 3 times with a "
                         "plain device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; "
                          "multi-GPU sharding is a design note (domain "
                          "decomposition), not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "surrogate":
        return bench_surrogate(args)
    if args.workload == "autograd":
        return bench_autograd(args)
    if args.workload == "lma":
        return bench_lma(args)
    if args.workload == "cadjoint":
        return bench_cadjoint(args)
    if args.workload == "srg-kernels":
        return bench_srg_kernels(args)
    if args.workload == "d3q19":
        return bench_d3q19(args)
    if args.nsteps is None:
        args.nsteps = 4000
    import torch
    from paper_1908_03876_amd import abi
    from paper_1908_03876_amd import inputs as I
    from paper_1908_03876_amd.solver import (DeviceProblem, GradientIteration,
                                             choose_ckpt_every)
    dev = torch.device("cuda:0")
    log(f"[bench] building workload L={args.L} N={args.nsteps}")
    prob = I.masked_anisotropic(L=args.L, nsteps=args.nsteps)
    if args.source_term == 2:
        prob = I.slow_reaction(prob, 0.1).copy(source_term=2)
    elif args.source_term == 3:
        prob = prob.copy(source_term=3)
    if args.species == 3:
        prob = I.with_repellent(prob)
    dp = DeviceProblem(prob, dtype=torch.float32, device=dev)
    free, total = torch.cuda.mem_get_info(dev)
    if args.ckpt == "auto":
        K = choose_ckpt_every(dp, int(0.85 * free))
    elif args.ckpt == "store":
        K = dp.nsteps
    else:
        K = int(args.ckpt)
    it = GradientIteration(dp, ckpt_every=K)
    info = it.tape.info
    mode = {0: "forward-only", 1: "store-all", 2: "checkpointed"}[info.mode]
    n_fluid = it.tape.n_fluid
    log(f"[bench] tape {mode} K={info.ckpt_every} {info.device_bytes / 2**30:.1f} GiB, "
        f"fluid nodes {n_fluid}")

    hist = []
    for w in range(args.warmup):
        r = it.step()
        hist.append(r["J"])
        log(f"[bench] warmup {w}: J={r['J']:.6g} |E|inf={r['grad_inf']:.3g}")
    torch.cuda.synchronize()
    abi.mrt_timing_reset()
    abi.mrt_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = it.step()
        hist.append(r["J"])
        log(f"[bench] iter {k}: J={r['J']:.6g} |E|inf={r['grad_inf']:.3g} zeta={r['zeta']:.3g}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    abi.mrt_timing_enable(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    f_ms, f_n = abi.mrt_timing_read(abi.TIMING_FORWARD)
    a_ms, a_n = abi.mrt_timing_read(abi.TIMING_ADJOINT)
    r_ms, r_n = abi.mrt_timing_read(abi.TIMING_RECOMPUTE)
    value = n_fluid * dp.nsteps / (ms_step / 1e3) / 1e6

    elem = 4
    b_fwd, b_adj, b_norec = bytes_per_site(elem, args.source_term, args.species)
    # per-launch algorithmic bytes: fluid nodes only
    launch_bytes_adj = n_fluid * b_adj
    fwd_rec_share = 1.0 if info.mode == 1 else 1.0 / info.n_segments
    launch_bytes_fwd = n_fluid * (fwd_rec_share * b_fwd + (1 - fwd_rec_share) * b_norec)
    avg_adj_ms = a_ms / max(a_n, 1)
    avg_fwd_ms = f_ms / max(f_n, 1)
    kern = {"mrt_forward_step": (f_ms, avg_fwd_ms, launch_bytes_fwd),
            "amrt_adjoint_step": (a_ms, avg_adj_ms, launch_bytes_adj)}
    dom = max(kern, key=lambda k: kern[k][0])
    _, avg_ms, lbytes = kern[dom]
    achieved = lbytes / (avg_ms / 1e3) / 1e9
    traffic = (read_traffic(dom, args.L)
               if args.source_term == 1 and args.species == 2 else None)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic, "kernel": dom,
            "avg_launch_ms": round(avg_ms, 5),
            "algorithmic_bytes_per_launch": int(lbytes),
            "algorithmic_bytes_per_fluid_node": b_adj if dom == "amrt_adjoint_step" else b_fwd,
            "link_word_bytes_per_launch": 2 * dp.nx * dp.ny}
    roof.update(traffic_rate(traffic, avg_ms))
    # the other step kernel beside it, against the ceiling of its own mix
    other = "mrt_forward_step" if dom == "amrt_adjoint_step" else "amrt_adjoint_step"
    _, o_ms, o_bytes = kern[other]
    o_rate = o_bytes / (o_ms / 1e3) / 1e9 if o_ms > 0 else 0.0
    side = {"kernel": other, "avg_launch_ms": round(o_ms, 5),
            "algorithmic_bytes_per_launch": int(o_bytes), "achieved": round(o_rate, 1),
            "unit": "GB/s", "frac": round(o_rate / HBM_PEAK_GBS, 4),
            "traffic": (read_traffic(other, args.L)
                        if args.source_term == 1 and args.species == 2 else None)}
    if o_ms > 0:
        side.update(traffic_rate(side["traffic"], o_ms))
    if args.source_term == 1 and args.species == 2:
        mix = {"amrt_adjoint_step": (23, 20), "mrt_forward_step": (19, 21)}
        add_stream_ceiling(roof, *mix[dom], dp.nx * dp.ny, dev)
        # a recording forward's mix; with a checkpointed tape most forward
        # launches do not record
        if o_rate > 0 and (other == "amrt_adjoint_step" or fwd_rec_share == 1.0):
            add_stream_ceiling(side, *mix[other], dp.nx * dp.ny, dev)
    out = {
        "metric": "coupled MRT+AMRT MLUPS (gradient iteration: forward + adjoint), "
                  "HBM GB/s fraction; s per gradient iteration",
        "value": round(value, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded disks, tensors, targets)",
        "config": {"workload": f"masked anisotropic chemotaxis control, {dp.nx}x{dp.ny} "
                               f"D2Q9 {'three' if args.species == 3 else 'two'}-species MRT, "
                               f"200 disks + wall ring, N={dp.nsteps} "
                               f"steps per solve, gradient-descent iterations"
                               + {1: "", 2: ", second-order source term (explicit "
                                           "characteristic difference), kinetics rates 0.1",
                                  3: ", second-order source term (implicit characteristic "
                                     "difference)"}[args.source_term]
                               + (", three species (repulsive signal w)"
                                  if args.species == 3 else ""),
                   "source_term": args.source_term, "species": args.species,
                   "L": dp.nx, "nsteps": dp.nsteps, "fluid_nodes": n_fluid,
                   "tape": mode, "ckpt_every": int(info.ckpt_every),
                   "tape_gib": round(info.device_bytes / 2**30, 2),
                   "parallelism": "single GPU"},
        "s_per_iteration": round(ms_step / 1e3, 4),
        "forward_mlups": round(n_fluid * f_n / (f_ms / 1e3) / 1e6, 1) if f_ms else None,
        "adjoint_mlups": round(n_fluid * a_n / (a_ms / 1e3) / 1e6, 1) if a_ms else None,
        "recompute_launches": r_n,
        "J_history": [round(x, 6) for x in hist],
        "roofline": roof,
        "other_kernel": side,
    }
    it.close()
    del dp
    torch.cuda.empty_cache()
    if args.copy_calibration:
        copy_calibration(out, dev)
    if args.cpu_steps > 0:
        log(f"[bench] cpu baseline: oracle {args.L}^2 x {args.cpu_steps} steps")
        out["cpu_baseline"] = cpu_baseline(args.L, args.cpu_steps)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
