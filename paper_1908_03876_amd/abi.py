"""ctypes binding of the C-ABI in include/mrt.h and include/mrt3.h (argument marshalling only).

Every function here has the name of the C entry point it calls.  Device
memory comes from torch tensors (``data_ptr()``), streams from
``torch.cuda.current_stream().cuda_stream``.  All computation runs in the
HIP kernels of libmrt.so; if the library is missing this module raises at
import time - there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmrt.so")

MRT_OK, MRT_EINVAL, MRT_ENOMEM, MRT_EHIP, MRT_ENONFINITE, MRT_ESTATE = 0, -1, -2, -3, -4, -5
MRT_F32, MRT_F64 = 0, 1
TIMING_FORWARD, TIMING_ADJOINT, TIMING_RECOMPUTE, TIMING_TLM, TIMING_CADJ = 0, 1, 2, 3, 4


class MrtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class mrt_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("pitch", ctypes.c_int32), ("q", ctypes.c_int32),
                ("periodic", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("nsteps", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("mask", ctypes.c_void_p)]


class mrt_species(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double * 4), ("d", ctypes.c_double),
                ("s", ctypes.c_double * 7)]


class mrt_problem(ctypes.Structure):
    _fields_ = [("grid", mrt_grid), ("u", mrt_species), ("v", mrt_species),
                ("chi", ctypes.c_double), ("Cchi", ctypes.c_double * 4),
                ("r_u", ctypes.c_double), ("a_uv", ctypes.c_double),
                ("b_v", ctypes.c_double), ("alpha", ctypes.c_double),
                ("source_term", ctypes.c_int32), ("nspecies", ctypes.c_int32),
                ("w", mrt_species), ("chi_w", ctypes.c_double),
                ("Cw", ctypes.c_double * 4), ("a_w", ctypes.c_double),
                ("b_w", ctypes.c_double), ("s_w", ctypes.c_double),
                ("w0", ctypes.c_void_p)]


class mrt_scalars(ctypes.Structure):
    _fields_ = [("J", ctypes.c_double), ("J_track", ctypes.c_double),
                ("J_reg", ctypes.c_double), ("grad_inf", ctypes.c_double),
                ("grad_l2", ctypes.c_double), ("n_fluid", ctypes.c_int64)]


class mrt_cg_info(ctypes.Structure):
    _fields_ = [("gg", ctypes.c_double), ("beta", ctypes.c_double), ("dg", ctypes.c_double),
                ("restart", ctypes.c_int32), ("reserved", ctypes.c_int32)]


MRT_CG_RULES = {"FR": 0, "PR": 1, "HS": 2, "DY": 3}


class mrt_tape_info(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("ckpt_every", ctypes.c_int32),
                ("n_segments", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_fluid", ctypes.c_int64), ("device_bytes", ctypes.c_size_t)]


class mrt_batch_tiles(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("max_blocks_per_cu", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ms_per_step", ctypes.c_double)]


class mrt3_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("pitch", ctypes.c_int32), ("periodic", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("nsteps", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("mask", ctypes.c_void_p)]


class mrt3_species(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double * 9), ("d", ctypes.c_double),
                ("s", ctypes.c_double * 16)]


class mrt3_problem(ctypes.Structure):
    _fields_ = [("grid", mrt3_grid), ("u", mrt3_species), ("v", mrt3_species),
                ("chi", ctypes.c_double), ("Cchi", ctypes.c_double * 9),
                ("r_u", ctypes.c_double), ("a_uv", ctypes.c_double),
                ("b_v", ctypes.c_double), ("alpha", ctypes.c_double)]


MRT_FIELD_U0, MRT_FIELD_V0, MRT_FIELD_CONTROL, MRT_FIELD_TARGET = 0, 1, 2, 3
MRT_FIELD_UN, MRT_FIELD_VN, MRT_FIELD_GRAD = 4, 5, 6

EXPORTS = ["mrt_validate", "mrt_tape_bytes", "mrt_tape_create",
           "mrt_tape_destroy", "mrt_tape_query", "mrt_forward", "amrt_adjoint",
           "cost_gradient", "cost_gradient_noalloc", "gd_step", "mrt_last_error",
           "mrt_timing_enable",
           "mrt_timing_reset", "mrt_timing_read", "mrt_stream_probe", "mrt_tlm", "mrt_dot",
           "mrt_axpby",
           "mrt_cadjoint", "mrt_lma_step", "mrt_cg_direction",
           "mrt_batch_create", "mrt_batch_destroy", "mrt_batch_field",
           "mrt_batch_copy", "mrt_batch_set_tiles", "mrt_batch_get_tiles",
           "mrt_batch_tune", "mrt_batch_set_timeout", "mrt_batch_iteration",
           "mrt_batch_scalars", "mrt_batch_forward",
           "mrt_srg_create", "mrt_srg_destroy", "mrt_srg_param", "mrt_srg_copy_param",
           "mrt_srg_sync",
           "mrt_srg_forward", "mrt_srg_backward", "mrt_srg_loss",
           "mrt_srg_train_step", "mrt_srg_gather", "mrt_srg_objective",
           "mrt_srg_score_steps", "mrt_srg_warm_start", "mrt_srg_warm_start_bb",
           "mrt3_validate", "mrt3_tape_bytes", "mrt3_tape_create", "mrt3_tape_destroy",
           "mrt3_tape_query", "mrt3_forward", "amrt3_adjoint", "mrt3_tlm",
           "mrt3_cost_gradient", "mrt3_gd_step"]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1908_03876_amd.build`")
    # torch first, so that libmrt.so binds to the HIP runtime torch loaded
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(mrt_problem)
    vp = ctypes.c_void_p
    L.mrt_validate.argtypes = [P]
    L.mrt_tape_bytes.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    L.mrt_tape_create.argtypes = [P, ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.mrt_tape_destroy.argtypes = [vp]
    L.mrt_tape_destroy.restype = None
    L.mrt_tape_query.argtypes = [vp, ctypes.POINTER(mrt_tape_info)]
    L.mrt_forward.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp]
    L.amrt_adjoint.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.cost_gradient.argtypes = [P, vp, vp, vp, vp, vp, vp, vp,
                                ctypes.POINTER(mrt_scalars), vp]
    L.cost_gradient_noalloc.argtypes = [P, vp, vp, vp, vp, vp, vp,
                                        ctypes.POINTER(mrt_scalars), vp]
    L.gd_step.argtypes = [P, vp, vp, vp, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double, ctypes.POINTER(ctypes.c_double), vp]
    L.mrt_tlm.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.mrt_dot.argtypes = [P, vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    L.mrt_cadjoint.argtypes = [P, vp, vp, vp, vp, vp, vp, vp]
    L.mrt_axpby.argtypes = [P, vp, vp, vp, ctypes.c_double, ctypes.c_double, vp]
    L.mrt_lma_step.argtypes = [P, vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    L.mrt_cg_direction.argtypes = [P, vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp,
                                   ctypes.c_double, ctypes.c_double,
                                   ctypes.POINTER(mrt_cg_info), vp]
    L.mrt_last_error.restype = ctypes.c_char_p
    L.mrt_timing_enable.argtypes = [ctypes.c_int32]
    L.mrt_timing_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int64)]
    L.mrt_stream_probe.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_void_p]
    T = ctypes.POINTER(mrt_batch_tiles)
    L.mrt_batch_create.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_size_t,
                                   ctypes.POINTER(vp)]
    L.mrt_batch_destroy.argtypes = [vp]
    L.mrt_batch_destroy.restype = None
    L.mrt_batch_field.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(vp)]
    L.mrt_batch_copy.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp]
    L.mrt_batch_set_tiles.argtypes = [vp, T]
    L.mrt_batch_get_tiles.argtypes = [vp, T]
    L.mrt_batch_tune.argtypes = [vp, ctypes.c_int32, T, vp]
    L.mrt_batch_set_timeout.argtypes = [vp, ctypes.c_double]
    L.mrt_batch_iteration.argtypes = [vp, ctypes.c_double, ctypes.c_int32, vp]
    L.mrt_batch_scalars.argtypes = [vp, ctypes.POINTER(mrt_scalars),
                                    ctypes.POINTER(ctypes.c_double), vp]
    L.mrt_batch_forward.argtypes = [vp, vp]
    i32, f32 = ctypes.c_int32, ctypes.c_float
    L.mrt_srg_create.argtypes = [i32, i32, i32, i32, f32, f32, ctypes.POINTER(vp)]
    L.mrt_srg_destroy.argtypes = [vp]
    L.mrt_srg_destroy.restype = None
    L.mrt_srg_param.argtypes = [vp, i32, i32, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int64)]
    L.mrt_srg_copy_param.argtypes = [vp, i32, i32, i32, vp, vp]
    L.mrt_srg_sync.argtypes = [vp, vp]
    L.mrt_srg_forward.argtypes = [vp, vp, vp, i32, i32, i32, vp]
    L.mrt_srg_backward.argtypes = [vp, vp, vp, vp, i32, i32, i32, i32, vp]
    L.mrt_srg_loss.argtypes = [vp, vp, vp, i32, i32, i32, i32, ctypes.POINTER(ctypes.c_double), vp]
    L.mrt_srg_train_step.argtypes = [vp, vp, vp, i32, i32, i32, i32, f32,
                                     ctypes.POINTER(ctypes.c_double), vp]
    L.mrt_srg_gather.argtypes = [vp, i32, vp, vp, vp, vp, vp, i32, i32, i32, vp]
    dbl = ctypes.c_double
    L.mrt_srg_objective.argtypes = [vp, vp, vp, vp, dbl, i32, i32, i32,
                                    ctypes.POINTER(dbl), vp, vp]
    L.mrt_srg_score_steps.argtypes = [vp, vp, vp, ctypes.POINTER(dbl), i32, vp, vp, dbl,
                                      i32, i32, ctypes.POINTER(dbl), vp]
    L.mrt_srg_warm_start.argtypes = [vp, vp, vp, dbl, i32, i32, i32, f32, vp, vp]
    L.mrt_srg_warm_start_bb.argtypes = [vp, vp, vp, dbl, i32, i32, i32, f32, vp, vp]
    P3 = ctypes.POINTER(mrt3_problem)
    L.mrt3_validate.argtypes = [P3]
    L.mrt3_tape_bytes.argtypes = [P3, i32, ctypes.POINTER(ctypes.c_size_t)]
    L.mrt3_tape_create.argtypes = [P3, i32, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.mrt3_tape_destroy.argtypes = [vp]
    L.mrt3_tape_destroy.restype = None
    L.mrt3_tape_query.argtypes = [vp, ctypes.POINTER(mrt_tape_info)]
    L.mrt3_forward.argtypes = [P3, vp, vp, vp, vp, vp, vp, vp, vp]
    L.amrt3_adjoint.argtypes = [P3, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.mrt3_tlm.argtypes = [P3, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.mrt3_cost_gradient.argtypes = [P3, vp, vp, vp, vp, vp, vp, vp,
                                     ctypes.POINTER(mrt_scalars), vp]
    L.mrt3_gd_step.argtypes = [P3, vp, vp, vp, dbl, dbl, dbl, ctypes.POINTER(dbl), vp]
    return L


lib = _load()


def _check(rc: int):
    if rc != MRT_OK:
        raise MrtError(rc, lib.mrt_last_error().decode())


def _ptr(t):
    """Device pointer of a tensor (or None)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ----------------------------------------------------------- entry points

def mrt_validate(p: mrt_problem) -> None:
    _check(lib.mrt_validate(ctypes.byref(p)))


def mrt_tape_bytes(p: mrt_problem, ckpt_every: int) -> int:
    n = ctypes.c_size_t()
    _check(lib.mrt_tape_bytes(ctypes.byref(p), int(ckpt_every), ctypes.byref(n)))
    return n.value


def mrt_tape_create(p: mrt_problem, ckpt_every: int, mem_budget: int = 0):
    h = ctypes.c_void_p()
    _check(lib.mrt_tape_create(ctypes.byref(p), int(ckpt_every), int(mem_budget),
                               ctypes.byref(h)))
    return h


def mrt_tape_destroy(tape) -> None:
    lib.mrt_tape_destroy(tape)


def mrt_tape_query(tape) -> mrt_tape_info:
    info = mrt_tape_info()
    _check(lib.mrt_tape_query(tape, ctypes.byref(info)))
    return info


def mrt_forward(p, tape, u0, v0, control, state=None, uN=None, vN=None,
                stream=None) -> None:
    _check(lib.mrt_forward(ctypes.byref(p), tape, _ptr(u0), _ptr(v0),
                           _ptr(control), _ptr(state), _ptr(uN), _ptr(vN),
                           _stream(stream)))


def amrt_adjoint(p, tape, u0, v0, control, seed_u, seed_v, grad_accum,
                 adj_u0=None, adj_v0=None, stream=None) -> None:
    _check(lib.amrt_adjoint(ctypes.byref(p), tape, _ptr(u0), _ptr(v0),
                            _ptr(control), _ptr(seed_u), _ptr(seed_v),
                            _ptr(grad_accum), _ptr(adj_u0), _ptr(adj_v0),
                            _stream(stream)))


def cost_gradient(p, tape, uN, u_target, control, grad_accum=None,
                  seed_out=None, grad_out=None, stream=None) -> dict:
    s = mrt_scalars()
    _check(lib.cost_gradient(ctypes.byref(p), tape, _ptr(uN), _ptr(u_target),
                             _ptr(control), _ptr(grad_accum), _ptr(seed_out),
                             _ptr(grad_out), ctypes.byref(s), _stream(stream)))
    return {"J": s.J, "J_track": s.J_track, "J_reg": s.J_reg,
            "grad_inf": s.grad_inf, "grad_l2": s.grad_l2, "n_fluid": s.n_fluid}


def cost_gradient_noalloc(p, uN, u_target, control, grad_accum=None,
                          seed_out=None, grad_out=None, stream=None) -> dict:
    s = mrt_scalars()
    _check(lib.cost_gradient_noalloc(ctypes.byref(p), _ptr(uN), _ptr(u_target),
                                     _ptr(control), _ptr(grad_accum), _ptr(seed_out),
                                     _ptr(grad_out), ctypes.byref(s), _stream(stream)))
    return {"J": s.J, "J_track": s.J_track, "J_reg": s.J_reg,
            "grad_inf": s.grad_inf, "grad_l2": s.grad_l2, "n_fluid": s.n_fluid}


def gd_step(p, tape, control, grad, zeta=0.0, lo=-math.inf, hi=math.inf,
            want_zeta=True, stream=None):
    z = ctypes.c_double(0.0)
    _check(lib.gd_step(ctypes.byref(p), tape, _ptr(control), _ptr(grad),
                       float(zeta), float(lo), float(hi),
                       ctypes.byref(z) if want_zeta else None, _stream(stream)))
    return z.value if want_zeta else None


def mrt_tlm(p, tape, u0, v0, control, dc=None, du0=None, dv0=None, duN=None, dvN=None,
            stream=None) -> None:
    _check(lib.mrt_tlm(ctypes.byref(p), tape, _ptr(u0), _ptr(v0), _ptr(control), _ptr(dc),
                       _ptr(du0), _ptr(dv0), _ptr(duN), _ptr(dvN), _stream(stream)))


def mrt_cadjoint(p, tape, u0, v0, control, seed_u, grad_accum, stream=None) -> None:
    _check(lib.mrt_cadjoint(ctypes.byref(p), tape, _ptr(u0), _ptr(v0), _ptr(control),
                            _ptr(seed_u), _ptr(grad_accum), _stream(stream)))


def mrt_dot(p, tape, x, y, stream=None) -> float:
    v = ctypes.c_double()
    _check(lib.mrt_dot(ctypes.byref(p), tape, _ptr(x), _ptr(y), ctypes.byref(v),
                       _stream(stream)))
    return v.value


def mrt_lma_step(p, tape, control, direction, resid, P, stream=None) -> float:
    z = ctypes.c_double()
    _check(lib.mrt_lma_step(ctypes.byref(p), tape, _ptr(control), _ptr(direction), _ptr(resid),
                            _ptr(P), ctypes.byref(z), _stream(stream)))
    return z.value


def mrt_cg_direction(p, tape, rule: str, first: bool, G, Gprev, D, gg_old: float,
                     dg_old: float, stream=None) -> dict:
    r = mrt_cg_info()
    _check(lib.mrt_cg_direction(ctypes.byref(p), tape, MRT_CG_RULES[rule], 1 if first else 0,
                                _ptr(G), _ptr(Gprev), _ptr(D), float(gg_old), float(dg_old),
                                ctypes.byref(r), _stream(stream)))
    return {"gg": r.gg, "beta": r.beta, "dg": r.dg, "restart": bool(r.restart)}


def mrt_axpby(p, tape, x, y, a: float, b: float, stream=None) -> None:
    _check(lib.mrt_axpby(ctypes.byref(p), tape, _ptr(x), _ptr(y), float(a), float(b),
                         _stream(stream)))


def mrt_timing_enable(on: bool) -> None:
    _check(lib.mrt_timing_enable(1 if on else 0))


def mrt_timing_reset() -> None:
    _check(lib.mrt_timing_reset())


def mrt_timing_read(kind: int):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib.mrt_timing_read(int(kind), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def mrt_stream_probe(reads: int, writes: int, inp, out, n: int, order: int = 1,
                     stream=None) -> None:
    _check(lib.mrt_stream_probe(int(reads), int(writes), int(order), _ptr(inp), _ptr(out),
                                int(n), _stream(stream)))


# ------------------------------------------------------------- batched form

def mrt_batch_create(problems, ckpt_every: int = 0, mem_budget: int = 0):
    arr = (mrt_problem * len(problems))(*problems)
    h = ctypes.c_void_p()
    _check(lib.mrt_batch_create(arr, len(problems), int(ckpt_every), int(mem_budget),
                                ctypes.byref(h)))
    return h


def mrt_batch_destroy(batch) -> None:
    lib.mrt_batch_destroy(batch)


def mrt_batch_field(batch, k: int, which: int) -> int:
    p = ctypes.c_void_p()
    _check(lib.mrt_batch_field(batch, int(k), int(which), ctypes.byref(p)))
    return p.value


def mrt_batch_copy(batch, k: int, which: int, to_batch: bool, data, stream=None) -> None:
    _check(lib.mrt_batch_copy(batch, int(k), int(which), 1 if to_batch else 0,
                              _ptr(data), _stream(stream)))


def mrt_batch_set_tiles(batch, tile_w: int, blocks_per_cu: int) -> None:
    t = mrt_batch_tiles(tile_w=int(tile_w), blocks_per_cu=int(blocks_per_cu))
    _check(lib.mrt_batch_set_tiles(batch, ctypes.byref(t)))


def mrt_batch_get_tiles(batch) -> dict:
    t = mrt_batch_tiles()
    _check(lib.mrt_batch_get_tiles(batch, ctypes.byref(t)))
    return {"tile_w": t.tile_w, "blocks_per_cu": t.blocks_per_cu,
            "max_blocks_per_cu": t.max_blocks_per_cu}


def mrt_batch_tune(batch, steps: int = 20, stream=None) -> dict:
    t = mrt_batch_tiles()
    _check(lib.mrt_batch_tune(batch, int(steps), ctypes.byref(t), _stream(stream)))
    return {"tile_w": t.tile_w, "blocks_per_cu": t.blocks_per_cu,
            "max_blocks_per_cu": t.max_blocks_per_cu, "ms_per_step": t.ms_per_step}


def mrt_batch_set_timeout(batch, seconds: float) -> None:
    _check(lib.mrt_batch_set_timeout(batch, float(seconds)))


def mrt_batch_iteration(batch, zeta: float = 0.0, use_graph: bool = True,
                        stream=None) -> None:
    _check(lib.mrt_batch_iteration(batch, float(zeta), 1 if use_graph else 0,
                                   _stream(stream)))


def mrt_batch_scalars(batch, count: int, stream=None):
    out = (mrt_scalars * count)()
    z = (ctypes.c_double * count)()
    _check(lib.mrt_batch_scalars(batch, out, z, _stream(stream)))
    return [{"J": s.J, "J_track": s.J_track, "J_reg": s.J_reg,
             "grad_inf": s.grad_inf, "grad_l2": s.grad_l2, "n_fluid": s.n_fluid,
             "zeta": z[i]} for i, s in enumerate(out)]


def mrt_batch_forward(batch, stream=None) -> None:
    _check(lib.mrt_batch_forward(batch, _stream(stream)))


# --------------------------------------------------------------- surrogate

def mrt_srg_create(channels: int, max_batch: int, max_h: int, max_w: int,
                   in_scale: float, out_scale: float):
    h = ctypes.c_void_p()
    _check(lib.mrt_srg_create(int(channels), int(max_batch), int(max_h), int(max_w),
                              float(in_scale), float(out_scale), ctypes.byref(h)))
    return h


def mrt_srg_destroy(s) -> None:
    lib.mrt_srg_destroy(s)


def mrt_srg_param(s, layer: int, kind: int):
    p = ctypes.c_void_p()
    n = ctypes.c_int64()
    _check(lib.mrt_srg_param(s, int(layer), int(kind), ctypes.byref(p), ctypes.byref(n)))
    return p.value, n.value


def mrt_srg_copy_param(s, layer: int, kind: int, to_srg: bool, data, stream=None) -> None:
    _check(lib.mrt_srg_copy_param(s, int(layer), int(kind), 1 if to_srg else 0, _ptr(data),
                                  _stream(stream)))


def mrt_srg_sync(s, stream=None) -> None:
    _check(lib.mrt_srg_sync(s, _stream(stream)))


def mrt_srg_forward(s, x, y, B, H, W, stream=None) -> None:
    _check(lib.mrt_srg_forward(s, _ptr(x), _ptr(y), int(B), int(H), int(W), _stream(stream)))


def mrt_srg_backward(s, x, dy, dx, weight_grads, B, H, W, stream=None) -> None:
    _check(lib.mrt_srg_backward(s, _ptr(x), _ptr(dy), _ptr(dx), 1 if weight_grads else 0,
                                int(B), int(H), int(W), _stream(stream)))


def mrt_srg_loss(s, x, target, B, H, W, border, stream=None) -> float:
    v = ctypes.c_double()
    _check(lib.mrt_srg_loss(s, _ptr(x), _ptr(target), int(B), int(H), int(W), int(border),
                            ctypes.byref(v), _stream(stream)))
    return v.value


def mrt_srg_train_step(s, x, target, B, H, W, border, lr, want_loss=False, stream=None):
    v = ctypes.c_double()
    _check(lib.mrt_srg_train_step(s, _ptr(x), _ptr(target), int(B), int(H), int(W),
                                  int(border), float(lr),
                                  ctypes.byref(v) if want_loss else None, _stream(stream)))
    return v.value if want_loss else None


def mrt_srg_gather(src, L, idx, oy, ox, out, n, h, w, sub=None, stream=None) -> None:
    _check(lib.mrt_srg_gather(_ptr(src), int(L), _ptr(idx), _ptr(oy), _ptr(ox), _ptr(sub),
                              _ptr(out), int(n), int(h), int(w), _stream(stream)))


def mrt_srg_objective(s, x, u_base, u_target, alpha, B, H, W, want_J=True, dx=None,
                      stream=None):
    """Per-field surrogate costs (list of B floats, or None) and, into dx,
    their input gradients."""
    J = (ctypes.c_double * int(B))()
    _check(lib.mrt_srg_objective(s, _ptr(x), _ptr(u_base), _ptr(u_target), float(alpha),
                                 int(B), int(H), int(W), J if want_J else None, _ptr(dx),
                                 _stream(stream)))
    return list(J) if want_J else None


def mrt_srg_score_steps(s, c, E, lambdas, u_base, u_target, alpha, H, W, stream=None):
    n = len(lambdas)
    lam = (ctypes.c_double * n)(*[float(v) for v in lambdas])
    J = (ctypes.c_double * n)()
    _check(lib.mrt_srg_score_steps(s, _ptr(c), _ptr(E), lam, int(n), _ptr(u_base),
                                   _ptr(u_target), float(alpha), int(H), int(W), J,
                                   _stream(stream)))
    return list(J)


def mrt_srg_warm_start(s, u_base, u_target, alpha, H, W, iters, lr, c, stream=None) -> None:
    _check(lib.mrt_srg_warm_start(s, _ptr(u_base), _ptr(u_target), float(alpha), int(H),
                                  int(W), int(iters), float(lr), _ptr(c), _stream(stream)))


def mrt_srg_warm_start_bb(s, u_base, u_target, alpha, H, W, iters, step0, c,
                          stream=None) -> None:
    _check(lib.mrt_srg_warm_start_bb(s, _ptr(u_base), _ptr(u_target), float(alpha), int(H),
                                     int(W), int(iters), float(step0), _ptr(c),
                                     _stream(stream)))


# ----------------------------------------------------------- D3Q19 (mrt3.h)

def mrt3_validate(p: mrt3_problem) -> None:
    _check(lib.mrt3_validate(ctypes.byref(p)))


def mrt3_tape_bytes(p: mrt3_problem, ckpt_every: int) -> int:
    n = ctypes.c_size_t()
    _check(lib.mrt3_tape_bytes(ctypes.byref(p), int(ckpt_every), ctypes.byref(n)))
    return n.value


def mrt3_tape_create(p: mrt3_problem, ckpt_every: int, mem_budget: int = 0):
    h = ctypes.c_void_p()
    _check(lib.mrt3_tape_create(ctypes.byref(p), int(ckpt_every), int(mem_budget),
                                ctypes.byref(h)))
    return h


def mrt3_tape_destroy(tape) -> None:
    lib.mrt3_tape_destroy(tape)


def mrt3_tape_query(tape) -> mrt_tape_info:
    info = mrt_tape_info()
    _check(lib.mrt3_tape_query(tape, ctypes.byref(info)))
    return info


def mrt3_forward(p, tape, u0, v0, control, state=None, uN=None, vN=None, stream=None) -> None:
    _check(lib.mrt3_forward(ctypes.byref(p), tape, _ptr(u0), _ptr(v0), _ptr(control),
                            _ptr(state), _ptr(uN), _ptr(vN), _stream(stream)))


def amrt3_adjoint(p, tape, u0, v0, control, seed_u, seed_v, grad_accum, adj_u0=None,
                  adj_v0=None, stream=None) -> None:
    _check(lib.amrt3_adjoint(ctypes.byref(p), tape, _ptr(u0), _ptr(v0), _ptr(control),
                             _ptr(seed_u), _ptr(seed_v), _ptr(grad_accum), _ptr(adj_u0),
                             _ptr(adj_v0), _stream(stream)))


def mrt3_tlm(p, tape, u0, v0, control, dc=None, du0=None, dv0=None, duN=None, dvN=None,
             stream=None) -> None:
    _check(lib.mrt3_tlm(ctypes.byref(p), tape, _ptr(u0), _ptr(v0), _ptr(control), _ptr(dc),
                        _ptr(du0), _ptr(dv0), _ptr(duN), _ptr(dvN), _stream(stream)))


def mrt3_cost_gradient(p, tape, uN, u_target, control, grad_accum=None, seed_out=None,
                       grad_out=None, stream=None) -> dict:
    s = mrt_scalars()
    _check(lib.mrt3_cost_gradient(ctypes.byref(p), tape, _ptr(uN), _ptr(u_target),
                                  _ptr(control), _ptr(grad_accum), _ptr(seed_out),
                                  _ptr(grad_out), ctypes.byref(s), _stream(stream)))
    return {"J": s.J, "J_track": s.J_track, "J_reg": s.J_reg,
            "grad_inf": s.grad_inf, "grad_l2": s.grad_l2, "n_fluid": s.n_fluid}


def mrt3_gd_step(p, tape, control, grad, zeta=0.0, lo=-math.inf, hi=math.inf,
                 want_zeta=True, stream=None):
    z = ctypes.c_double(0.0)
    _check(lib.mrt3_gd_step(ctypes.byref(p), tape, _ptr(control), _ptr(grad), float(zeta),
                            float(lo), float(hi), ctypes.byref(z) if want_zeta else None,
                            _stream(stream)))
    return z.value if want_zeta else None
