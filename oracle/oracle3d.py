"""ctypes wrapper of the FP64 CPU oracle of the D3Q19 scheme
(``mrt3d_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product path never imports it.

Fields are float64 numpy arrays [nz, ny, nx] in C order; the problem is any
object with the attributes of ``paper_1908_03876_amd.inputs.Problem3``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrt3d_oracle.so")
SRC_PATH = os.path.join(HERE, "mrt3d_oracle.cpp")


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c++17", "-Wall", SRC_PATH, "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Orc3Species(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double * 9), ("d", ctypes.c_double),
                ("s", ctypes.c_double * 16)]


class Orc3Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("periodic", ctypes.c_int), ("solid", ctypes.POINTER(ctypes.c_ubyte)),
                ("u", Orc3Species), ("v", Orc3Species),
                ("chi", ctypes.c_double), ("Cchi", ctypes.c_double * 9),
                ("r_u", ctypes.c_double), ("a_uv", ctypes.c_double),
                ("b_v", ctypes.c_double), ("alpha", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(Orc3Problem)
        L.orc3_tables.argtypes = [dp, dp, dp, dp]
        L.orc3_species_ops.argtypes = [ctypes.POINTER(Orc3Species), dp, dp, dp]
        L.orc3_collide.argtypes = [P, dp, ctypes.c_double, dp]
        L.orc3_local_jacobian.argtypes = [P, dp, dp]
        L.orc3_forward.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp, dp]
        L.orc3_adjoint.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc3_tlm.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc3_cost_complex_step.argtypes = [P, ctypes.c_int, dp, dp, dp, dp,
                                             ctypes.c_double, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _species(D, d, s) -> Orc3Species:
    sp = Orc3Species()
    sp.D[:] = [float(x) for x in np.asarray(D, dtype=np.float64).ravel()]
    sp.d = float(d)
    sp.s[:] = [float(x) for x in np.asarray(s, dtype=np.float64).ravel()]
    return sp


class _Prob:
    def __init__(self, p):
        self.solid = None if p.solid is None else np.ascontiguousarray(p.solid, dtype=np.uint8)
        s = Orc3Problem()
        s.nx, s.ny, s.nz = int(p.nx), int(p.ny), int(p.nz)
        s.periodic = 1 if p.periodic else 0
        s.solid = (self.solid.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))
                   if self.solid is not None else None)
        s.u = _species(p.Du, p.du, p.su)
        s.v = _species(p.Dv, p.dv, p.sv)
        s.chi = float(p.chi)
        s.Cchi[:] = [float(x) for x in np.asarray(p.Cchi).ravel()]
        s.r_u, s.a_uv, s.b_v = float(p.r_u), float(p.a_uv), float(p.b_v)
        s.alpha = float(p.alpha)
        self.s = s

    @property
    def ptr(self):
        return ctypes.byref(self.s)


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"oracle call failed ({rc})")


def tables():
    E = np.zeros((19, 3)); w = np.zeros(19); M = np.zeros((19, 19)); Minv = np.zeros((19, 19))
    _check(lib().orc3_tables(_dp(E), _dp(w), _dp(M), _dp(Minv)))
    return E, w, M, Minv


def species_ops(D, d=1.0, s=None):
    s = np.ones(16) if s is None else s
    sp = _species(D, d, s)
    K = np.zeros(9); C = np.zeros((19, 19)); weq = np.zeros(19)
    _check(lib().orc3_species_ops(ctypes.byref(sp), _dp(K), _dp(C), _dp(weq)))
    return K.reshape(3, 3), C, weq


def collide(p, phi, c=0.0):
    pr = _Prob(p)
    phi = _f64(phi).ravel().copy()
    out = np.zeros(38)
    _check(lib().orc3_collide(pr.ptr, _dp(phi), float(c), _dp(out)))
    return out


def local_jacobian(p, phi):
    pr = _Prob(p)
    phi = _f64(phi).ravel().copy()
    J = np.zeros((38, 38))
    _check(lib().orc3_local_jacobian(pr.ptr, _dp(phi), _dp(J)))
    return J


def forward(p, nsteps=None, control=None, u0=None, v0=None, want_state=False):
    n = p.nsteps if nsteps is None else nsteps
    pr = _Prob(p)
    shp = (p.nz, p.ny, p.nx)
    uN = np.zeros(shp); vN = np.zeros(shp)
    state = np.zeros((2, 19) + shp) if want_state else None
    _check(lib().orc3_forward(pr.ptr, n, _dp(_f64(p.u0 if u0 is None else u0)),
                              _dp(_f64(p.v0 if v0 is None else v0)),
                              _dp(_f64(p.control if control is None else control)),
                              _dp(uN), _dp(vN), _dp(state)))
    out = {"uN": uN, "vN": vN}
    if want_state:
        out["state"] = state
    return out


def cost(p, uN, control=None):
    c = p.control if control is None else control
    f = p.fluid
    jt = 0.5 * ((uN - p.u_target)[f] ** 2).sum()
    jr = 0.5 * p.alpha * (c[f] ** 2).sum()
    return jt + jr, jt, jr


def adjoint(p, seed_u, seed_v=None, nsteps=None, control=None):
    n = p.nsteps if nsteps is None else nsteps
    pr = _Prob(p)
    shp = (p.nz, p.ny, p.nx)
    g = np.zeros(shp); du0 = np.zeros(shp); dv0 = np.zeros(shp)
    _check(lib().orc3_adjoint(pr.ptr, n, _dp(_f64(p.u0)), _dp(_f64(p.v0)),
                              _dp(_f64(p.control if control is None else control)),
                              _dp(_f64(seed_u)), _dp(_f64(seed_v)), _dp(g), _dp(du0), _dp(dv0)))
    return g, du0, dv0


def tlm(p, dc=None, du0=None, dv0=None, nsteps=None):
    n = p.nsteps if nsteps is None else nsteps
    pr = _Prob(p)
    shp = (p.nz, p.ny, p.nx)
    duN = np.zeros(shp); dvN = np.zeros(shp)
    _check(lib().orc3_tlm(pr.ptr, n, _dp(_f64(p.u0)), _dp(_f64(p.v0)), _dp(_f64(p.control)),
                          _dp(_f64(dc)), _dp(_f64(du0)), _dp(_f64(dv0)), _dp(duN), _dp(dvN)))
    return duN, dvN


def cost_complex_step(p, dc, h=1e-20, nsteps=None):
    n = p.nsteps if nsteps is None else nsteps
    pr = _Prob(p)
    jr = ctypes.c_double(); ji = ctypes.c_double()
    _check(lib().orc3_cost_complex_step(pr.ptr, n, _dp(_f64(p.u0)), _dp(_f64(p.v0)),
                                        _dp(_f64(p.control)), _dp(_f64(dc)), float(h),
                                        _dp(_f64(p.u_target)), ctypes.byref(jr),
                                        ctypes.byref(ji)))
    return jr.value, ji.value / h


def cost_gradient(p, nsteps=None, control=None):
    """J and the discrete gradient g + alpha c (0 on solid cells)."""
    c = p.control if control is None else control
    fwd = forward(p, nsteps=nsteps, control=c)
    f = p.fluid
    J, jt, jr = cost(p, fwd["uN"], control=c)
    seed = (fwd["uN"] - p.u_target) * f
    g, _, _ = adjoint(p, seed, nsteps=nsteps, control=c)
    return {"J": J, "J_track": jt, "J_reg": jr, "grad": (g + p.alpha * c) * f, "uN": fwd["uN"]}
