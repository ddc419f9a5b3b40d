"""ctypes wrapper of the FP64 CPU oracle (``mrt_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product path never imports it.

All arrays are float64 numpy arrays of shape [ny, nx] (fields) in C order.
The problem argument is any object with the attributes of
``paper_1908_03876_amd.inputs.Problem``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrt_oracle.so")
SRC_PATH = os.path.join(HERE, "mrt_oracle.cpp")


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c++17", "-Wall", SRC_PATH, "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class OrcSpecies(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double * 4), ("d", ctypes.c_double),
                ("s", ctypes.c_double * 7)]


class OrcProblem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("periodic", ctypes.c_int),
                ("solid", ctypes.POINTER(ctypes.c_ubyte)),
                ("u", OrcSpecies), ("v", OrcSpecies),
                ("chi", ctypes.c_double), ("Cchi", ctypes.c_double * 4),
                ("r_u", ctypes.c_double), ("a_uv", ctypes.c_double),
                ("b_v", ctypes.c_double), ("alpha", ctypes.c_double),
                ("control_on_u", ctypes.c_int), ("source_term", ctypes.c_int),
                ("nspecies", ctypes.c_int), ("w", OrcSpecies),
                ("chi_w", ctypes.c_double), ("Cw", ctypes.c_double * 4),
                ("a_w", ctypes.c_double), ("b_w", ctypes.c_double),
                ("s_w", ctypes.c_double), ("w0", ctypes.POINTER(ctypes.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(OrcProblem)
        L.orc_tables.argtypes = [dp, dp, dp, dp]
        L.orc_species_ops.argtypes = [ctypes.POINTER(OrcSpecies), dp, dp, dp, dp]
        L.orc_collide.argtypes = [P, dp, ctypes.c_double, dp]
        L.orc_local_jacobian.argtypes = [P, dp, dp]
        L.orc_local_adjoint.argtypes = [P, dp, dp, dp]
        L.orc_forward.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_cost.argtypes = [P, dp, dp, dp, dp, dp]
        L.orc_cost.restype = ctypes.c_double
        L.orc_adjoint.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_adjoint_theta.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp, dp]
        L.orc_tlm.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_cost_complex_step.argtypes = [P, ctypes.c_int, dp, dp, dp, dp,
                                            ctypes.c_double, dp, dp, dp]
        L.orc_cost_gradient.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp,
                                        dp, dp, dp, dp]
        L.orc_cadjoint.argtypes = [P, ctypes.c_int, dp, dp, dp, dp, dp]
        L.orc_gd_step.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double]
        L.orc_gd_step.restype = ctypes.c_double
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _species(D, d, s) -> OrcSpecies:
    sp = OrcSpecies()
    sp.D[:] = [float(x) for x in np.asarray(D, dtype=np.float64).ravel()]
    sp.d = float(d)
    sp.s[:] = [float(x) for x in np.asarray(s, dtype=np.float64).ravel()]
    return sp


class _Prob:
    """Keeps the ctypes struct and the mask buffer alive together."""

    def __init__(self, p, control_on_u: bool = False):
        self.solid = None if p.solid is None else np.ascontiguousarray(p.solid, dtype=np.uint8)
        s = OrcProblem()
        s.nx, s.ny = int(p.nx), int(p.ny)
        s.periodic = 1 if p.periodic else 0
        s.solid = (self.solid.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))
                   if self.solid is not None else None)
        s.u = _species(p.Du, p.du, p.su)
        s.v = _species(p.Dv, p.dv, p.sv)
        s.chi = float(p.chi)
        s.Cchi[:] = [float(x) for x in np.asarray(p.Cchi).ravel()]
        s.r_u, s.a_uv, s.b_v = float(p.r_u), float(p.a_uv), float(p.b_v)
        s.alpha = float(p.alpha)
        s.control_on_u = 1 if control_on_u else 0
        s.source_term = int(getattr(p, "source_term", 1))
        s.nspecies = int(getattr(p, "nspecies", 2))
        self.w0 = None
        if s.nspecies == 3:
            s.w = _species(p.Dw, p.dw, p.sw)
            s.chi_w = float(p.chi_w)
            s.Cw[:] = [float(x) for x in np.asarray(p.Cw).ravel()]
            s.a_w, s.b_w, s.s_w = float(p.a_w), float(p.b_w), float(p.s_w)
            if p.w0 is not None:
                self.w0 = np.ascontiguousarray(p.w0, dtype=np.float64)
                s.w0 = self.w0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.s = s

    @property
    def ptr(self):
        return ctypes.byref(self.s)


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"oracle call failed ({rc})")


def tables():
    E = np.zeros((9, 2)); w = np.zeros(9); M = np.zeros((9, 9)); Minv = np.zeros((9, 9))
    _check(lib().orc_tables(_dp(E), _dp(w), _dp(M), _dp(Minv)))
    return E, w, M, Minv


def species_ops(D, d=1.0, s=None):
    s = np.ones(7) if s is None else s
    sp = _species(D, d, s)
    K = np.zeros(4); Pi = np.zeros((9, 9)); C = np.zeros((9, 9)); weq = np.zeros(9)
    _check(lib().orc_species_ops(ctypes.byref(sp), _dp(K), _dp(Pi), _dp(C), _dp(weq)))
    return K.reshape(2, 2), Pi, C, weq


def collide(p, phi, c=0.0, control_on_u=False):
    pr = _Prob(p, control_on_u)
    phi = _f64(phi).ravel().copy()
    out = np.zeros(18)
    _check(lib().orc_collide(pr.ptr, _dp(phi), float(c), _dp(out)))
    return out


def local_jacobian(p, phi):
    pr = _Prob(p)
    phi = _f64(phi).ravel().copy()
    J = np.zeros((18, 18))
    _check(lib().orc_local_jacobian(pr.ptr, _dp(phi), _dp(J)))
    return J


def local_adjoint(p, phi, nu):
    pr = _Prob(p)
    phi = _f64(phi).ravel().copy(); nu = _f64(nu).ravel().copy()
    lam = np.zeros(18)
    _check(lib().orc_local_adjoint(pr.ptr, _dp(phi), _dp(nu), _dp(lam)))
    return lam


def forward(p, nsteps=None, control=None, u0=None, v0=None, want_state=False,
            want_traj=False, control_on_u=False):
    """Returns dict with uN, vN and optionally state [2,9,ny,nx] and the
    trajectory traj_u [N,ny,nx], traj_j [N,2,ny,nx]."""
    n = p.nsteps if nsteps is None else nsteps
    pr = _Prob(p, control_on_u)
    u0 = _f64(p.u0 if u0 is None else u0)
    v0 = _f64(p.v0 if v0 is None else v0)
    c = _f64(p.control if control is None else control)
    shp = (p.ny, p.nx)
    ns = int(getattr(p, "nspecies", 2))
    want_state = want_state or ns == 3
    uN = np.zeros(shp); vN = np.zeros(shp)
    state = np.zeros((ns, 9) + shp) if want_state else None
    tu = np.zeros((n,) + shp) if want_traj else None
    tj = np.zeros((n, 2) + shp) if want_traj else None
    _check(lib().orc_forward(pr.ptr, n, _dp(u0), _dp(v0), _dp(c), _dp(uN), _dp(vN),
                             _dp(state), _dp(tu), _dp(tj)))
    out = {"uN": uN, "vN": vN}
    if want_state:
        out["state"] = state
    if ns == 3:
        out["wN"] = state[2].sum(axis=0)
    if want_traj:
        out["traj_u"], out["traj_j"] = tu, tj
    return out


def cost(p, uN, control=None):
    pr = _Prob(p)
    c = _f64(p.control if control is None else control)
    jt = ctypes.c_double(); jr = ctypes.c_double()
    J = lib().orc_cost(pr.ptr, _dp(_f64(uN)), _dp(_f64(p.u_target)), _dp(c),
                       ctypes.byref(jt), ctypes.byref(jr))
    return J, jt.value, jr.value


def adjoint(p, seed_u, seed_v=None, nsteps=None, control=None, u0=None, v0=None,
            control_on_u=False):
    """Returns (g, dJ/du0, dJ/dv0): g = sum_n tau sum_i w_i psi_v,i."""
    n = p.nsteps if nsteps is None else nsteps
    pr = _Prob(p, control_on_u)
    u0 = _f64(p.u0 if u0 is None else u0)
    v0 = _f64(p.v0 if v0 is None else v0)
    c = _f64(p.control if control is None else control)
    shp = (p.ny, p.nx)
    g = np.zeros(shp); du0 = np.zeros(shp); dv0 = np.zeros(shp)
    _check(lib().orc_adjoint(pr.ptr, n, _dp(u0), _dp(v0), _dp(c), _dp(_f64(seed_u)),
                             _dp(_f64(seed_v)), _dp(g), _dp(du0), _dp(dv0)))
    return g, du0, dv0


def theta_gradient(p, seed_u, seed_v=None, nsteps=None, control=None, u0=None, v0=None,
                   control_on_u=False):
    """The paper's trapezoid-in-time form of the gradient (JD-H-B), a
    diagnostic beside the exact transpose that adjoint() returns: the
    integrand at t_n is step n's term of the exact gradient, h_n, and at t_N
    the terminal adjoint's tau sum_i w_i psi_c,i^N; theta_0 = theta_N = 1/2,
    so g_theta = g - h_0/2 + h_N/2 (first source form, nsteps >= 1)."""
    n = p.nsteps if nsteps is None else nsteps
    pr = _Prob(p, control_on_u)
    u0 = _f64(p.u0 if u0 is None else u0)
    v0 = _f64(p.v0 if v0 is None else v0)
    c = _f64(p.control if control is None else control)
    gt = np.zeros((p.ny, p.nx))
    _check(lib().orc_adjoint_theta(pr.ptr, n, _dp(u0), _dp(v0), _dp(c), _dp(_f64(seed_u)),
                                   _dp(_f64(seed_v)), _dp(gt)))
    return gt


def tlm(p, dc=None, du0=None, dv0=None, nsteps=None, control=None,
        control_on_u=False):
    n = p.nsteps if nsteps is None else nsteps
    pr = _Prob(p, control_on_u)
    c = _f64(p.control if control is None else control)
    shp = (p.ny, p.nx)
    duN = np.zeros(shp); dvN = np.zeros(shp)
    _check(lib().orc_tlm(pr.ptr, n, _dp(_f64(p.u0)), _dp(_f64(p.v0)), _dp(c),
                         _dp(_f64(dc)), _dp(_f64(du0)), _dp(_f64(dv0)),
                         _dp(duN), _dp(dvN)))
    return duN, dvN


def cost_complex_step(p, dc, h=1e-20, nsteps=None, control=None,
                      control_on_u=False):
    n = p.nsteps if nsteps is None else nsteps
    pr = _Prob(p, control_on_u)
    c = _f64(p.control if control is None else control)
    jr = ctypes.c_double(); ji = ctypes.c_double()
    _check(lib().orc_cost_complex_step(pr.ptr, n, _dp(_f64(p.u0)), _dp(_f64(p.v0)),
                                       _dp(c), _dp(_f64(dc)), float(h),
                                       _dp(_f64(p.u_target)), ctypes.byref(jr),
                                       ctypes.byref(ji)))
    return jr.value, ji.value / h


def set_traj_budget(nbytes: int) -> None:
    """Bytes of forward states the adjoint keeps whole before it switches to
    checkpoints every ceil(sqrt(N)) steps with segment recomputation
    (default 16 GiB)."""
    f = lib().orc_set_traj_budget
    f.argtypes = [ctypes.c_size_t]
    f.restype = None
    f(int(nbytes))


def cost_gradient(p, nsteps=None, control=None, control_on_u=False):
    """Returns dict(J, J_track, J_reg, grad, uN) of the full discrete gradient."""
    n = p.nsteps if nsteps is None else nsteps
    pr = _Prob(p, control_on_u)
    c = _f64(p.control if control is None else control)
    shp = (p.ny, p.nx)
    grad = np.zeros(shp); uN = np.zeros(shp)
    J = ctypes.c_double(); jt = ctypes.c_double(); jr = ctypes.c_double()
    _check(lib().orc_cost_gradient(pr.ptr, n, _dp(_f64(p.u0)), _dp(_f64(p.v0)),
                                   _dp(c), _dp(_f64(p.u_target)), _dp(grad),
                                   ctypes.byref(J), ctypes.byref(jt),
                                   ctypes.byref(jr), _dp(uN)))
    return {"J": J.value, "J_track": jt.value, "J_reg": jr.value,
            "grad": grad, "uN": uN}


def cadjoint(p, seed_u, nsteps=None, control=None):
    """Continuous-adjoint part of the gradient: tau * sum over the reversed
    steps of q (the adjoint of v), [ny, nx]."""
    n = p.nsteps if nsteps is None else nsteps
    pr = _Prob(p, False)
    c = _f64(p.control if control is None else control)
    g = np.zeros((p.ny, p.nx))
    _check(lib().orc_cadjoint(pr.ptr, n, _dp(_f64(p.u0)), _dp(_f64(p.v0)), _dp(c),
                              _dp(_f64(seed_u)), _dp(g)))
    return g


def cost_gradient_continuous(p, nsteps=None, control=None):
    """J and the continuous-adjoint gradient tau sum q + alpha c (0 on solids)."""
    c = p.control if control is None else control
    fwd = forward(p, nsteps=nsteps, control=c)
    f = p.fluid
    seed = (fwd["uN"] - p.u_target) * f
    g = cadjoint(p, seed, nsteps=nsteps, control=c)
    return {"J": cost(p, fwd["uN"], control=c)[0], "grad": (g + p.alpha * c) * f}


def gd_step(control, grad, zeta=0.0, lo=-np.inf, hi=np.inf):
    c = _f64(control).copy()
    E = _f64(grad)
    z = lib().orc_gd_step(c.size, _dp(c), _dp(E), float(zeta), float(lo), float(hi))
    return c, z
