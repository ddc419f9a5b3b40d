"""Seeded synthetic inputs for the chemotaxis optimal-control workloads.

This module is shared by the CPU oracle tests, the GPU parity tests and the
benchmark.  It only draws random fields and parameters (initial states,
obstacle masks, diffusion tensors, targets, controls); it contains none of the
lattice Boltzmann arithmetic.  Everything is generated in float64 with
``numpy.random.default_rng(seed)`` and cast by the caller.

Problem statement followed (Section 1, eq. (ReacDiff) and (classicJ)):
two species, cell density u and chemical v, on a 2-D lattice,

    du/dt - div(D_u grad u) = r_u u (1 - u) - div(chi u C_chi grad v)
    dv/dt - div(D_v grad v) = a_uv u - b_v v + c(x)

with a static distributed control c on the v equation and the terminal
tracking cost 1/2 ||u(T) - u_target||^2 + alpha/2 ||c||^2 (Section 2.1,
(classicJ) with a_1 = 1 and a quadratic control penalty).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class Problem:
    """One control problem instance (lattice units: h = tau = 1)."""

    nx: int
    ny: int
    nsteps: int
    periodic: bool
    solid: Optional[np.ndarray]  # uint8 [ny, nx], 1 = solid, or None
    Du: np.ndarray               # 2x2 self-diffusion tensor of u
    Dv: np.ndarray               # 2x2 self-diffusion tensor of v
    chi: float                   # chemotactic sensitivity
    Cchi: np.ndarray             # 2x2 shape of the chemotactic tensor
    r_u: float = 1.0             # logistic rate of u
    a_uv: float = 1.0            # production of v by u
    b_v: float = 1.0             # decay of v
    alpha: float = 1e-3          # control penalty weight
    du: float = 1.0              # equilibrium parameter d_u
    dv: float = 1.0              # equilibrium parameter d_v
    su: np.ndarray = dataclasses.field(default_factory=lambda: np.ones(7))
    sv: np.ndarray = dataclasses.field(default_factory=lambda: np.ones(7))
    u0: np.ndarray = None        # [ny, nx]
    v0: np.ndarray = None        # [ny, nx]
    control: np.ndarray = None   # [ny, nx], initial guess of c
    u_target: np.ndarray = None  # [ny, nx]
    # third species (attraction-repulsion example): a repulsive signal w,
    # Phi_w = a_w u - b_w w + s_w, cross-diffusion of u D_u2 = chi_w u C_w
    nspecies: int = 2
    Dw: np.ndarray = None
    dw: float = 1.0
    sw: np.ndarray = dataclasses.field(default_factory=lambda: np.ones(7))
    chi_w: float = 0.0
    Cw: np.ndarray = None
    a_w: float = 0.0
    b_w: float = 0.0
    s_w: float = 0.0
    w0: np.ndarray = None        # [ny, nx]
    source_term: int = 1        # 1: tau w_i Phi; 2: plus (tau^2/2) dF/dt by the
                                 # explicit characteristic difference (kappa_x = 0);
                                 # 3: plus (tau^2/2)(d/dt + e.grad) F by the
                                 # implicit one (kappa_x = 1)
    name: str = ""

    @property
    def fluid(self) -> np.ndarray:
        if self.solid is None:
            return np.ones((self.ny, self.nx), dtype=bool)
        return self.solid == 0

    @property
    def n_fluid(self) -> int:
        return int(self.fluid.sum())

    def copy(self, **changes) -> "Problem":
        p = dataclasses.replace(self, **changes)
        for f in ("solid", "Du", "Dv", "Cchi", "su", "sv", "u0", "v0",
                  "control", "u_target", "Dw", "sw", "Cw", "w0"):
            val = getattr(p, f)
            if isinstance(val, np.ndarray) and f not in changes:
                setattr(p, f, val.copy())
        return p


# ---------------------------------------------------------------- helpers

def random_spd(rng: np.random.Generator, lo: float = 0.05, hi: float = 1.0,
               rmax: float = 0.3) -> np.ndarray:
    """Symmetric tensor with diagonal ~ U[lo, hi] and off-diagonal
    r*sqrt(D11*D22), r ~ U(-rmax, rmax): positive definite for rmax < 1."""
    d1, d2 = rng.uniform(lo, hi, size=2)
    r = rng.uniform(-rmax, rmax)
    off = r * np.sqrt(d1 * d2)
    return np.array([[d1, off], [off, d2]], dtype=np.float64)


def periodic_sqdist(nx: int, ny: int, x0: float, y0: float) -> np.ndarray:
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    dx = np.abs(x[None, :] - x0)
    dy = np.abs(y[:, None] - y0)
    dx = np.minimum(dx, nx - dx)
    dy = np.minimum(dy, ny - dy)
    return dx * dx + dy * dy


def plain_sqdist(nx: int, ny: int, x0: float, y0: float) -> np.ndarray:
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    return (x[None, :] - x0) ** 2 + (y[:, None] - y0) ** 2


def gaussian_bumps(nx: int, ny: int, centres, sigmas, amps,
                   periodic: bool) -> np.ndarray:
    out = np.zeros((ny, nx), dtype=np.float64)
    dist = periodic_sqdist if periodic else plain_sqdist
    for (cx, cy), s, a in zip(centres, sigmas, amps):
        out += a * np.exp(-dist(nx, ny, cx, cy) / (2.0 * s * s))
    return out


def disk_mask(nx: int, ny: int, rng: np.random.Generator, n_disks: int,
              rmin: int, rmax: int, ring: bool = True) -> np.ndarray:
    """uint8 mask, 1 = solid: union of disks (x-cx)^2+(y-cy)^2 <= r^2 on
    integer cell coordinates (no wrap), plus a one-cell solid outer ring."""
    solid = np.zeros((ny, nx), dtype=np.uint8)
    cx = rng.uniform(0, nx, size=n_disks)
    cy = rng.uniform(0, ny, size=n_disks)
    rr = rng.integers(rmin, rmax + 1, size=n_disks)
    for x0, y0, r in zip(cx, cy, rr):
        xl, xh = max(int(np.floor(x0 - r)), 0), min(int(np.ceil(x0 + r)) + 1, nx)
        yl, yh = max(int(np.floor(y0 - r)), 0), min(int(np.ceil(y0 + r)) + 1, ny)
        if xl >= xh or yl >= yh:
            continue
        xs = np.arange(xl, xh, dtype=np.float64)
        ys = np.arange(yl, yh, dtype=np.float64)
        inside = (xs[None, :] - x0) ** 2 + (ys[:, None] - y0) ** 2 <= float(r) ** 2
        solid[yl:yh, xl:xh] |= inside.astype(np.uint8)
    if ring:
        solid[0, :] = 1
        solid[-1, :] = 1
        solid[:, 0] = 1
        solid[:, -1] = 1
    return solid


def noisy_initial_u(nx: int, ny: int, rng: np.random.Generator,
                    amp: float = 0.1) -> np.ndarray:
    return 1.0 + amp * rng.uniform(-1.0, 1.0, size=(ny, nx))


def random_bump_control(nx: int, ny: int, rng: np.random.Generator,
                        kmin: int = 1, kmax: int = 8, smin: float = 4.0,
                        smax: float = 32.0, amax: float = 5.0,
                        periodic: bool = True) -> np.ndarray:
    """Sum of K ~ U{kmin..kmax} Gaussian bumps with uniform centres,
    sigma ~ U[smin, smax] and amplitude ~ U[-amax, amax]."""
    k = int(rng.integers(kmin, kmax + 1))
    centres = list(zip(rng.uniform(0, nx, size=k), rng.uniform(0, ny, size=k)))
    sig = rng.uniform(smin, smax, size=k)
    amp = rng.uniform(-amax, amax, size=k)
    return gaussian_bumps(nx, ny, centres, sig, amp, periodic)


def _zero_solids(p: Problem) -> Problem:
    if p.solid is not None:
        f = p.solid != 0
        for name in ("u0", "v0", "control", "u_target"):
            arr = getattr(p, name)
            arr[f] = 0.0
    return p


# ---------------------------------------------------------------- workloads

def periodic_isotropic(seed: int = 1, L: int = 64, nsteps: int = 200) -> Problem:
    """Plain method, FP64: L x L periodic, isotropic D_u = 0.1, D_v = 1.0,
    chi = 0.5, logistic u, v driven by u, zero initial control, Gaussian
    target bump of sigma = 8 cells."""
    rng = np.random.default_rng(seed)
    u0 = noisy_initial_u(L, L, rng)
    x0, y0 = rng.uniform(0, L, size=2)
    ut = 1.0 + 0.5 * np.exp(-periodic_sqdist(L, L, x0, y0) / (2.0 * 8.0 ** 2))
    return Problem(nx=L, ny=L, nsteps=nsteps, periodic=True, solid=None,
                   Du=0.1 * np.eye(2), Dv=1.0 * np.eye(2), chi=0.5,
                   Cchi=np.eye(2), u0=u0, v0=np.zeros((L, L)),
                   control=np.zeros((L, L)), u_target=ut, name=f"periodic_L{L}")


def masked_anisotropic(seed: int = 2, L: int = 2048, nsteps: int = 4000,
                       n_disks: int = 200, rmin: int = 5, rmax: int = 30,
                       n_target_bumps: int = 8, target_sigma: float = 64.0) -> Problem:
    """Plain method at scale, FP32: L x L with a bounce-back mask of random
    disks plus a solid outer ring, full anisotropic self and chemotactic
    tensors (diagonal in [0.05, 1], off-diagonal U(-0.3, 0.3) of the
    geometric mean of the diagonal)."""
    rng = np.random.default_rng(seed)
    solid = disk_mask(L, L, rng, n_disks, rmin, rmax, ring=True)
    Du = random_spd(rng)
    Dv = random_spd(rng)
    Cchi = random_spd(rng)
    u0 = noisy_initial_u(L, L, rng)
    cen = list(zip(rng.uniform(0, L, n_target_bumps), rng.uniform(0, L, n_target_bumps)))
    ut = 1.0 + gaussian_bumps(L, L, cen, [target_sigma] * n_target_bumps,
                              [0.5] * n_target_bumps, periodic=False)
    p = Problem(nx=L, ny=L, nsteps=nsteps, periodic=False, solid=solid,
                Du=Du, Dv=Dv, chi=0.5, Cchi=Cchi, u0=u0,
                v0=np.zeros((L, L)), control=np.zeros((L, L)),
                u_target=ut, name=f"masked_L{L}_N{nsteps}")
    return _zero_solids(p)


def masked_anisotropic_small(seed: int = 2, L: int = 128, nsteps: int = 200) -> Problem:
    """The small copy of the masked anisotropic workload: same tensor
    recipe, 4 disks of radius 3..8 cells plus the outer ring."""
    return masked_anisotropic(seed=seed, L=L, nsteps=nsteps, n_disks=4, rmin=3, rmax=8,
                              n_target_bumps=2, target_sigma=L / 8.0)


def long_horizon(seed: int = 3, L: int = 2048, nsteps: int = 10000) -> Problem:
    """Differentiation form: the masked anisotropic workload at a longer
    horizon."""
    if L <= 256:
        return masked_anisotropic(seed=seed, L=L, nsteps=nsteps, n_disks=4, rmin=3,
                                  rmax=8, n_target_bumps=2, target_sigma=L / 8.0)
    return masked_anisotropic(seed=seed, L=L, nsteps=nsteps)


def uneven_batch(seed: int = 4, n: int = 96, nsteps: int = 2000,
                 sizes=(128, 256, 384, 512, 768, 1024)) -> List[Problem]:
    """Batched form: n independent periodic problems of uneven square size,
    per-instance chi ~ U[0.1, 1], seeded tensors and one target bump of
    sigma = L/8."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        L = int(rng.choice(sizes))
        Du, Dv, Cchi = random_spd(rng), random_spd(rng), random_spd(rng)
        chi = float(rng.uniform(0.1, 1.0))
        u0 = noisy_initial_u(L, L, rng)
        x0, y0 = rng.uniform(0, L, size=2)
        ut = 1.0 + 0.5 * np.exp(-periodic_sqdist(L, L, x0, y0) / (2.0 * (L / 8.0) ** 2))
        out.append(Problem(nx=L, ny=L, nsteps=nsteps, periodic=True, solid=None,
                           Du=Du, Dv=Dv, chi=chi, Cchi=Cchi, u0=u0,
                           v0=np.zeros((L, L)), control=np.zeros((L, L)),
                           u_target=ut, name=f"uneven_{k}_L{L}"))
    return out


def with_control_bump(p: Problem, seed: int = 11, amp: float = 5.0,
                      sigma: float = None) -> Problem:
    """Copy of p with a non-zero control (one Gaussian bump), so that the
    state is not driven to the trivial fixed point u = v = 1."""
    rng = np.random.default_rng(seed)
    sigma = sigma if sigma is not None else max(p.nx, p.ny) / 8.0
    cx, cy = rng.uniform(0, p.nx), rng.uniform(0, p.ny)
    c = gaussian_bumps(p.nx, p.ny, [(cx, cy)], [sigma], [amp], p.periodic)
    q = p.copy(control=c)
    return _zero_solids(q)


def slow_reaction(p: Problem, rate: float = 0.01) -> Problem:
    """Copy of p with slow kinetics r_u = a_uv = b_v = rate."""
    return p.copy(r_u=rate, a_uv=rate, b_v=rate)


def with_repellent(p: Problem, seed: int = 21, chi_w: float = -0.4) -> Problem:
    """Copy of p with a third species w, a repulsive chemical signal
    (attraction-repulsion example): seeded SPD D_w and C_w (recipe of the
    other tensors), chi_w < 0, Phi_w = 0.5 u - 0.8 w + 0.05, non-unit
    relaxation rates, w0 ~ 0.2 U(0, 1) on fluid nodes."""
    rng = np.random.default_rng(seed)
    w0 = 0.2 * rng.uniform(0, 1, size=(p.ny, p.nx)) * p.fluid
    return p.copy(nspecies=3, Dw=random_spd(rng), dw=1.0, sw=rng.uniform(0.8, 1.6, size=7),
                  chi_w=chi_w, Cw=random_spd(rng), a_w=0.5, b_w=0.8, s_w=0.05, w0=w0)


def random_direction(p: Problem, seed: int) -> np.ndarray:
    """Random perturbation h ~ N(0,1) on fluid cells, scaled to max |h| = 1."""
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((p.ny, p.nx))
    h[~p.fluid] = 0.0
    return h / np.abs(h).max()


def tiny(seed: int = 5, L: int = 8, nsteps: int = 10, masked: bool = False,
         anisotropic: bool = True) -> Problem:
    """Small randomised instance for brute-force checks (finite differences,
    complex step, transposition identities)."""
    rng = np.random.default_rng(seed)
    if anisotropic:
        Du, Dv, Cchi = random_spd(rng), random_spd(rng), random_spd(rng)
    else:
        Du, Dv, Cchi = 0.1 * np.eye(2), 1.0 * np.eye(2), np.eye(2)
    solid = None
    if masked:
        solid = np.zeros((L, L), dtype=np.uint8)
        solid[0, :] = solid[-1, :] = solid[:, 0] = solid[:, -1] = 1
        solid[L // 2, L // 2] = 1
    u0 = 1.0 + 0.3 * rng.uniform(-1, 1, size=(L, L))
    v0 = 0.5 * rng.uniform(0, 1, size=(L, L))
    c = rng.uniform(-1, 1, size=(L, L))
    ut = 1.0 + 0.5 * rng.uniform(0, 1, size=(L, L))
    su = rng.uniform(0.8, 1.6, size=7)
    sv = rng.uniform(0.8, 1.6, size=7)
    p = Problem(nx=L, ny=L, nsteps=nsteps, periodic=not masked, solid=solid,
                Du=Du, Dv=Dv, chi=0.7, Cchi=Cchi, r_u=0.3, a_uv=0.4, b_v=0.2,
                alpha=1e-2, su=su, sv=sv, u0=u0, v0=v0, control=c,
                u_target=ut, name=f"tiny_L{L}")
    return _zero_solids(p)


# ------------------------------------------------------------ D3Q19 problems


@dataclasses.dataclass
class Problem3:
    """A control problem on a D3Q19 lattice (two species, lattice units)."""

    nx: int
    ny: int
    nz: int
    nsteps: int
    periodic: bool
    solid: Optional[np.ndarray]  # uint8 [nz, ny, nx], 1 = solid, or None
    Du: np.ndarray               # 3x3 self-diffusion tensors
    Dv: np.ndarray
    chi: float
    Cchi: np.ndarray             # 3x3 shape of the chemotactic tensor
    r_u: float = 1.0
    a_uv: float = 1.0
    b_v: float = 1.0
    alpha: float = 1e-3
    du: float = 1.0
    dv: float = 1.0
    su: np.ndarray = dataclasses.field(default_factory=lambda: np.ones(16))
    sv: np.ndarray = dataclasses.field(default_factory=lambda: np.ones(16))
    u0: np.ndarray = None        # [nz, ny, nx]
    v0: np.ndarray = None
    control: np.ndarray = None
    u_target: np.ndarray = None
    name: str = ""

    @property
    def fluid(self) -> np.ndarray:
        if self.solid is None:
            return np.ones((self.nz, self.ny, self.nx), dtype=bool)
        return self.solid == 0

    @property
    def n_fluid(self) -> int:
        return int(self.fluid.sum())

    def copy(self, **changes) -> "Problem3":
        p = dataclasses.replace(self, **changes)
        for f in ("solid", "Du", "Dv", "Cchi", "su", "sv", "u0", "v0", "control", "u_target"):
            val = getattr(p, f)
            if isinstance(val, np.ndarray) and f not in changes:
                setattr(p, f, val.copy())
        return p


def random_spd3(rng: np.random.Generator, lo: float = 0.05, hi: float = 1.0) -> np.ndarray:
    """3x3 SPD tensor: diagonal ~ U[lo, hi], off-diagonals r sqrt(D_ii D_jj)
    with r ~ U(-0.3, 0.3) (unit-diagonal part diagonally dominant, so SPD)."""
    d = rng.uniform(lo, hi, size=3)
    r = rng.uniform(-0.3, 0.3, size=3)
    R = np.array([[1.0, r[0], r[1]], [r[0], 1.0, r[2]], [r[1], r[2], 1.0]])
    s = np.sqrt(d)
    return R * np.outer(s, s)


def _bump3(shape, rng, n, sigma, periodic=True):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros(shape)
    for _ in range(n):
        c = rng.uniform(0, 1, size=3) * np.array([nz, ny, nx])
        dz, dy, dx = z - c[0], y - c[1], x - c[2]
        if periodic:
            dz = np.minimum(np.abs(dz), nz - np.abs(dz))
            dy = np.minimum(np.abs(dy), ny - np.abs(dy))
            dx = np.minimum(np.abs(dx), nx - np.abs(dx))
        out += np.exp(-(dx * dx + dy * dy + dz * dz) / (2 * sigma * sigma))
    return out


def _zero_solids3(p: Problem3) -> Problem3:
    if p.solid is not None:
        s = p.solid != 0
        for f in ("u0", "v0", "control", "u_target"):
            getattr(p, f)[s] = 0.0
    return p


def periodic_3d(seed: int = 7, L: int = 16, nsteps: int = 30) -> Problem3:
    """Periodic cube with seeded anisotropic tensors, a control bump and a
    target bump; kinetics r_u = a_uv = b_v = 1."""
    rng = np.random.default_rng(seed)
    shp = (L, L, L)
    u0 = 1.0 + 0.1 * rng.uniform(-1, 1, size=shp)
    return Problem3(nx=L, ny=L, nz=L, nsteps=nsteps, periodic=True, solid=None,
                    Du=random_spd3(rng), Dv=random_spd3(rng), chi=0.5, Cchi=random_spd3(rng),
                    u0=u0, v0=np.zeros(shp), control=2.0 * _bump3(shp, rng, 1, L / 6),
                    u_target=1.0 + 0.5 * _bump3(shp, rng, 1, L / 6), name=f"periodic3d_L{L}")


def masked_3d(seed: int = 8, L: int = 24, nsteps: int = 30, n_spheres: int = None,
              rmin: int = None, rmax: int = None) -> Problem3:
    """Cube with a one-cell solid frame and seeded solid spheres (a porous
    medium: centres uniform, integer radii U{rmin..rmax}, by default
    max(2, L/64)..max(4, L/24) and max(3, L^3/16000) spheres, about 9% of
    the volume at L = 256); tensors, bumps and kinetics as in periodic_3d."""
    rng = np.random.default_rng(seed)
    shp = (L, L, L)
    rmin = max(2, L // 64) if rmin is None else rmin
    rmax = max(4, L // 24) if rmax is None else rmax
    solid = np.zeros(shp, dtype=np.uint8)
    solid[0], solid[-1] = 1, 1
    solid[:, 0], solid[:, -1] = 1, 1
    solid[:, :, 0], solid[:, :, -1] = 1, 1
    n = n_spheres if n_spheres is not None else max(3, (L * L * L) // 16000)
    for _ in range(n):
        c = rng.uniform(0, L, size=3)
        r = int(rng.integers(rmin, rmax + 1))
        lo = [max(0, int(np.floor(c[k] - r))) for k in range(3)]
        hi = [min(L, int(np.ceil(c[k] + r)) + 1) for k in range(3)]
        z, y, x = np.ogrid[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        ball = (z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2 <= r * r
        solid[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] |= ball.astype(np.uint8)
    u0 = 1.0 + 0.1 * rng.uniform(-1, 1, size=shp)
    p = Problem3(nx=L, ny=L, nz=L, nsteps=nsteps, periodic=False, solid=solid,
                 Du=random_spd3(rng), Dv=random_spd3(rng), chi=0.5, Cchi=random_spd3(rng),
                 u0=u0, v0=np.zeros(shp), control=2.0 * _bump3(shp, rng, 2, L / 8, False),
                 u_target=1.0 + 0.5 * _bump3(shp, rng, 2, L / 8, False), name=f"masked3d_L{L}")
    return _zero_solids3(p)


def tiny3d(seed: int = 9, nx: int = 5, ny: int = 4, nz: int = 3, nsteps: int = 6,
           masked: bool = False) -> Problem3:
    """Small randomised D3Q19 instance for brute-force checks."""
    rng = np.random.default_rng(seed)
    shp = (nz, ny, nx)
    solid = None
    if masked:
        solid = np.zeros(shp, dtype=np.uint8)
        solid[nz // 2, ny // 2, nx // 2] = 1
        solid[0, 0, :] = 1
    p = Problem3(nx=nx, ny=ny, nz=nz, nsteps=nsteps, periodic=not masked, solid=solid,
                 Du=random_spd3(rng), Dv=random_spd3(rng), chi=0.7, Cchi=random_spd3(rng),
                 r_u=0.3, a_uv=0.4, b_v=0.2, alpha=1e-2,
                 su=rng.uniform(0.8, 1.6, size=16), sv=rng.uniform(0.8, 1.6, size=16),
                 u0=1.0 + 0.3 * rng.uniform(-1, 1, size=shp), v0=0.5 * rng.uniform(0, 1, size=shp),
                 control=rng.uniform(-1, 1, size=shp), u_target=1.0 + 0.5 * rng.uniform(0, 1, size=shp),
                 name="tiny3d")
    return _zero_solids3(p)


def random_direction3(p: Problem3, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((p.nz, p.ny, p.nx)) * p.fluid
    return h / np.abs(h).max()


def ragged_3d(seed: int, nx: int, ny: int, nz: int, nsteps: int, periodic: bool,
              masked: bool, solid_frac: float = 0.06) -> Problem3:
    """Box of any shape with seeded tensors, rates, kinetics and fields;
    masked: each node solid with probability solid_frac (seeded)."""
    rng = np.random.default_rng(seed)
    shp = (nz, ny, nx)
    solid = (rng.uniform(size=shp) < solid_frac).astype(np.uint8) if masked else None
    p = Problem3(nx=nx, ny=ny, nz=nz, nsteps=nsteps, periodic=periodic, solid=solid,
                 Du=random_spd3(rng), Dv=random_spd3(rng), chi=0.3, Cchi=random_spd3(rng),
                 r_u=0.3, a_uv=0.4, b_v=0.2, alpha=1e-2,
                 su=rng.uniform(0.8, 1.6, size=16), sv=rng.uniform(0.8, 1.6, size=16),
                 u0=1.0 + 0.3 * rng.uniform(-1, 1, size=shp), v0=0.5 * rng.uniform(0, 1, size=shp),
                 control=0.2 * rng.uniform(-1, 1, size=shp),
                 u_target=1.0 + 0.5 * rng.uniform(0, 1, size=shp),
                 name=f"ragged3d_{nx}x{ny}x{nz}")
    return _zero_solids3(p)
