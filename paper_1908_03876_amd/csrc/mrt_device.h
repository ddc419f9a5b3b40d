// Per-node device code of the two- and three-species D2Q9 MRT step and of
// its exact discrete adjoint (AMRT), shared by the single-lattice kernels
// and the batched persistent kernels.
//
// Method: arXiv:1908.03876, Section 3.1 (eq:LBE, S, PhiS, MF, MC, phieq,
// BC11, the relaxation matrix Pi and D = d Cs^2 tau (K^-1 - I/2)) and
// Section 3.2.1 (LIBEG, CAE, AEDs, RFS1, CAEL, gradientLattice).
#pragma once

#include <hip/hip_runtime.h>

#include "mrt_internal.h"

namespace mrt {
namespace dev {

constexpr int kBlock = 256;
constexpr int kXcds = 8;

// D2Q9 opposite directions: e3 = -e1, e4 = -e2, e7 = -e5, e8 = -e6.
__device__ __forceinline__ constexpr int opp(int i) {
  return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5);
}

// Linear work-group id -> tile id such that XCD k (ids = k mod 8) owns the
// contiguous tile range [k*n/8, (k+1)*n/8).
__device__ __forceinline__ int xcd_tile(int id, int n) {
  const int per = n / kXcds, rem = n % kXcds;
  const int xcd = id % kXcds, k = id / kXcds;
  // the first `rem` XCDs own per+1 tiles
  const int base = xcd * per + (xcd < rem ? xcd : rem);
  return base + k;
}

struct NodeIdx {
  int x, y;
  int xm, xp;        // x - 1, x + 1 with periodic wrap
  size_t r0, rm, rp; // row offsets of y, y - 1, y + 1 with wrap
  bool ex0, ex1;     // x == 0, x == nx - 1
  bool ey0, ey1;     // y == 0, y == ny - 1
};

// Neighbour bookkeeping of node (x, y) of a lattice.
__device__ __forceinline__ void make_node(const Geometry& g, int x, int y,
                                          NodeIdx& n) {
  n.x = x;
  n.y = y;
  n.ex0 = n.x == 0;
  n.ex1 = n.x + 1 == g.nx;
  n.ey0 = n.y == 0;
  n.ey1 = n.y + 1 == g.ny;
  n.xm = n.ex0 ? g.nx - 1 : n.x - 1;
  n.xp = n.ex1 ? 0 : n.x + 1;
  const int ym = n.ey0 ? g.ny - 1 : n.y - 1;
  const int yp = n.ey1 ? 0 : n.y + 1;
  n.r0 = size_t(n.y) * g.pitch;
  n.rm = size_t(ym) * g.pitch;
  n.rp = size_t(yp) * g.pitch;
}

// Node of this thread in the single-lattice kernels: 256-node row tiles,
// XCD-banded (each of the 8 XCDs owns a contiguous range of tiles).
__device__ __forceinline__ bool node_of_block(const Geometry& g, NodeIdx& n) {
  const int nbx = (g.nx + kBlock - 1) / kBlock;
  const int ntiles = nbx * g.ny;
  const int id = blockIdx.x;
  if (id >= ntiles) return false;
  // the id -> tile map is a bijection on [0, ntiles) because ids are dealt
  // round-robin to XCDs
  const int t = xcd_tile(id, ntiles);
  const int x = (t % nbx) * kBlock + threadIdx.x;
  if (x >= g.nx) return false;
  make_node(g, x, t / nbx, n);
  return true;
}

// Per-wavefront wall flag (64 consecutive nodes of a row, one scalar load):
// 0 = the nodes and their neighbours are all fluid, 1 = mixed, 2 = all
// nodes solid.  Flag-0 wavefronts never read the link mask; in mixed ones
// the link load is independent of the population loads, so it adds no
// latency to them.
__device__ __forceinline__ unsigned wave_flag(const Geometry& g,
                                              const NodeIdx& n) {
  const int seg = __builtin_amdgcn_readfirstlane(n.y * g.nsx + (n.x >> 6));
  return g.wflag[seg];
}

__device__ __forceinline__ unsigned link_of(const Geometry& g, unsigned flag,
                                            size_t idx) {
  return flag ? unsigned(g.link[idx]) : 0u;
}

// Offset (within a plane) of node x - e_i for i = 0..8 (periodic wrap).
__device__ __forceinline__ size_t pull_off(const NodeIdx& n, int i) {
  switch (i) {
    case 0: return n.r0 + n.x;
    case 1: return n.r0 + n.xm;   // e1 = (1,0)
    case 2: return n.rm + n.x;    // e2 = (0,1)
    case 3: return n.r0 + n.xp;   // e3 = (-1,0)
    case 4: return n.rp + n.x;    // e4 = (0,-1)
    case 5: return n.rm + n.xm;   // e5 = (1,1)
    case 6: return n.rm + n.xp;   // e6 = (-1,1)
    case 7: return n.rp + n.xp;   // e7 = (-1,-1)
    default: return n.rp + n.xm;  // e8 = (1,-1)
  }
}

// Offset of node x + e_i = x - e_opp(i).
__device__ __forceinline__ size_t push_off(const NodeIdx& n, int i) {
  return pull_off(n, opp(i));
}

// Is x - e_i outside the lattice (meaningful for non-periodic lattices)?
__device__ __forceinline__ bool pull_outside(const NodeIdx& n, int i) {
  switch (i) {
    case 0: return false;
    case 1: return n.ex0;
    case 2: return n.ey0;
    case 3: return n.ex1;
    case 4: return n.ey1;
    case 5: return n.ex0 || n.ey0;
    case 6: return n.ex1 || n.ey0;
    case 7: return n.ex1 || n.ey1;
    default: return n.ex0 || n.ey1;
  }
}

// Is x + e_i outside the lattice?
__device__ __forceinline__ bool push_outside(const NodeIdx& n, int i) {
  return pull_outside(n, opp(i));
}

// Source of the population that node x pulls in direction i: plane i at
// x - e_i.  A solid in-domain neighbour needs no test: its slot holds the
// reflected population written by the previous step's wall stores.  Only
// at the edge of a non-periodic lattice does the node take its own
// opposite population (halfway bounce-back).
template <bool PERIODIC>
__device__ __forceinline__ size_t pull_src(const NodeIdx& n, int i,
                                           size_t plane) {
  if (!PERIODIC && pull_outside(n, i))
    return size_t(opp(i)) * plane + n.r0 + n.x;
  return size_t(i) * plane + pull_off(n, i);
}

// Adjoint gather source: plane i at x + e_i (transpose of the pull), or the
// node's own opposite value at the edge of a non-periodic lattice.
template <bool PERIODIC>
__device__ __forceinline__ size_t gather_src(const NodeIdx& n, int i,
                                             size_t plane) {
  if (!PERIODIC && push_outside(n, i))
    return size_t(opp(i)) * plane + n.r0 + n.x;
  return size_t(i) * plane + push_off(n, i);
}

// Relaxation in moment space: f <- f - M0^-1 Pi (M0 f - m_eq(theta)).
// With theta = 0 and the K block transposed this is f <- f - C^T f
// (C^T = M0^-1 Pi^T M0 since Pi only couples moments of equal row norm),
// without the conserved zeroth-moment part.  Returns the scaled amounts
// (a1, a2) of the e and epsilon moments for the adjoint equilibrium term.
template <typename T>
__device__ __forceinline__ void relax(T f[9], T theta,
                                      const SpeciesCoef<T>& c, T& a1o,
                                      T& a2o) {
  const T sa = f[1] + f[2] + f[3] + f[4];
  const T sd = f[5] + f[6] + f[7] + f[8];
  const T m1 = T(-4) * f[0] - sa + T(2) * sd;       // e
  const T m2 = T(4) * f[0] - T(2) * sa + sd;        // epsilon
  const T dx = f[5] - f[6] - f[7] + f[8];
  const T dy = f[5] + f[6] - f[7] - f[8];
  const T m3 = f[1] - f[3] + dx;                    // j_x
  const T m4 = T(-2) * (f[1] - f[3]) + dx;          // q_x
  const T m5 = f[2] - f[4] + dy;                    // j_y
  const T m6 = T(-2) * (f[2] - f[4]) + dy;          // q_y
  const T m7 = f[1] - f[2] + f[3] - f[4];           // p_xx
  const T m8 = f[5] - f[6] + f[7] - f[8];           // p_xy
  const T a1 = c.s1 * (m1 - c.e_eq * theta);
  const T a2 = c.s2 * (m2 - c.eps_eq * theta);
  const T a3 = c.k00 * m3 + c.k01 * m5;
  const T a5 = c.k10 * m3 + c.k11 * m5;
  const T a4 = c.s3 * m4;
  const T a6 = c.s4 * m6;
  const T a7 = c.s5 * m7;
  const T a8 = c.s6 * m8;
  const T b = T(2) * a1 + a2;
  const T h = -a1 - T(2) * a2;
  f[0] -= T(4) * (a2 - a1);
  f[1] -= h + a3 - T(2) * a4 + a7;
  f[2] -= h + a5 - T(2) * a6 - a7;
  f[3] -= h - a3 + T(2) * a4 + a7;
  f[4] -= h - a5 + T(2) * a6 - a7;
  f[5] -= b + a3 + a4 + a5 + a6 + a8;
  f[6] -= b - a3 - a4 + a5 + a6 - a8;
  f[7] -= b - a3 - a4 - a5 - a6 + a8;
  f[8] -= b + a3 + a4 - a5 - a6 - a8;
  a1o = a1;
  a2o = a2;
}

// --------------------------------------------------------------- forward

// Pre-collision populations of node n: the pull from src (with wall slots),
// or the equilibrium initialisation phi_i = w_i Theta_0 (phieq, zero flux)
// on the first step.  Also returns the node's control value, so that every
// load of a node update can be issued before any of its stores.
template <typename T, bool PERIODIC, bool FIRST>
__device__ __forceinline__ void forward_gather(const Geometry& g, const NodeIdx& n,
                                               const ModelCoef<T>& m, const T* __restrict__ src,
                                               const T* __restrict__ u0, const T* __restrict__ v0,
                                               const T* __restrict__ ctrl, T fu[9], T fv[9],
                                               T& c) {
  const size_t idx = n.r0 + n.x;
  if (FIRST) {
    const T a = u0[idx], b = v0[idx];
    fu[0] = m.u.w_rest * a;
    fv[0] = m.v.w_rest * b;
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      fu[i] = m.u.w_axis * a;
      fv[i] = m.v.w_axis * b;
    }
#pragma unroll
    for (int i = 5; i < 9; ++i) {
      fu[i] = m.u.w_diag * a;
      fv[i] = m.v.w_diag * b;
    }
  } else {
    const T* sv = src + 9 * g.plane;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const size_t o = pull_src<PERIODIC>(n, i, g.plane);
      fu[i] = src[o];
      fv[i] = sv[o];
    }
  }
  c = ctrl[idx];
}

// Sources tau S_i + tau w_i Phi (S, PhiS) with tau = 1, 1/Cs^2 = 3: the
// chemotactic flux (ax, ay) and the kinetics phu on the u populations, phv
// on the v populations.
template <typename T>
__device__ __forceinline__ void add_sources(T fu[9], T fv[9], T phu, T ax, T ay, T phv) {
  const T p9 = phu * T(1.0 / 9.0), p36 = phu * T(1.0 / 36.0);
  const T x3 = ax * T(1.0 / 3.0), y3 = ay * T(1.0 / 3.0);
  const T x12 = ax * T(1.0 / 12.0), y12 = ay * T(1.0 / 12.0);
  fu[0] += phu * T(4.0 / 9.0);
  fu[1] += p9 + x3;
  fu[2] += p9 + y3;
  fu[3] += p9 - x3;
  fu[4] += p9 - y3;
  fu[5] += p36 + x12 + y12;
  fu[6] += p36 - x12 + y12;
  fu[7] += p36 - x12 - y12;
  fu[8] += p36 + x12 - y12;
  const T q9 = phv * T(1.0 / 9.0), q36 = phv * T(1.0 / 36.0);
  fv[0] += phv * T(4.0 / 9.0);
#pragma unroll
  for (int i = 1; i < 5; ++i) fv[i] += q9;
#pragma unroll
  for (int i = 5; i < 9; ++i) fv[i] += q36;
}

// Post-collision state of a fluid node: non-temporal stores (the state does
// not fit the caches and is next read one whole sweep later) and the wall
// slots: a population phi*_i streaming into the solid node x + e_i is
// reflected; it is parked in that node's slot of plane opp(i), where the
// next step's pull in direction opp(i) at x reads it.
template <typename T, bool MASKED>
__device__ __forceinline__ void store_state(const Geometry& g, const NodeIdx& n,
                                            const T fu[9], const T fv[9],
                                            T* __restrict__ dst, unsigned lm) {
  const size_t idx = n.r0 + n.x;
  T* dv = dst + 9 * g.plane;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    __builtin_nontemporal_store(fu[i], &dst[size_t(i) * g.plane + idx]);
    __builtin_nontemporal_store(fv[i], &dv[size_t(i) * g.plane + idx]);
  }
  if (MASKED && (lm & 0x1FEu)) {
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      if ((lm >> opp(i)) & 1u) {
        const size_t o = size_t(opp(i)) * g.plane + push_off(n, i);
        dst[o] = fu[i];
        dv[o] = fv[i];
      }
    }
  }
}

__device__ __forceinline__ float dsqrt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double dsqrt(double x) { return __builtin_sqrt(x); }

// Implicit characteristic difference of the second-order source (eq:LBEG
// with kappa_t = kappa_x = 1): the scheme carries g = phi - (tau/2) w Phi,
// and Theta solves Theta - (tau/2) Phi(Theta) = G = sum_i g_i at each node:
// u from (tau r_u / 2) u^2 + (1 - tau r_u / 2) u - G_u = 0 (the root that
// tends to G_u as r_u -> 0, written without cancellation; tau r_u < 2),
// then v from the linear equation (a_uv u - b_v v + c enters at weight 1/2).
template <typename T>
__device__ __forceinline__ void implicit_solve(const ModelCoef<T>& m, T Gu, T Gv, T c, T& u,
                                               T& v) {
  const T hr = T(0.5) * m.r_u;
  const T bq = T(1) - hr;
  u = T(2) * Gu / (bq + dsqrt(bq * bq + T(4) * hr * Gu));
  v = (Gv + T(0.5) * (m.a_uv * u + c)) / (T(1) + T(0.5) * m.b_v);
}

// Scheme variants: the source term of (eq:LBEG) for two species, 1 first
// order (tau F_i), 2 explicit characteristic difference (kappa_t = 1,
// kappa_x = 0), 3 implicit characteristic difference (kappa_t = kappa_x =
// 1); 4 three species (u, v and a repulsive signal w, first-order source).
constexpr int kVarFirst = 1, kVarExplicit = 2, kVarImplicit = 3, kVarThree = 4;

// Third species of a node: its pull from planes 18..26 of src (with wall
// slots), or w_i w0 at the first step.
template <typename T, bool PERIODIC, bool FIRST>
__device__ __forceinline__ void gather_w(const Geometry& g, const NodeIdx& n,
                                         const ModelCoef<T>& m, const T* __restrict__ src,
                                         const T* __restrict__ w0, T fw[9]) {
  if (FIRST) {
    const T a = w0 ? w0[n.r0 + n.x] : T(0);
    fw[0] = m.w.w_rest * a;
#pragma unroll
    for (int i = 1; i < 5; ++i) fw[i] = m.w.w_axis * a;
#pragma unroll
    for (int i = 5; i < 9; ++i) fw[i] = m.w.w_diag * a;
  } else {
    const T* sw = src + 18 * g.plane;
#pragma unroll
    for (int i = 0; i < 9; ++i) fw[i] = sw[pull_src<PERIODIC>(n, i, g.plane)];
  }
}

// Stores of the third species' post-collision values (planes 18..26 of
// dst) with their wall slots, as store_state does for u and v.
template <typename T, bool MASKED>
__device__ __forceinline__ void store_w(const Geometry& g, const NodeIdx& n, const T fw[9],
                                        T* __restrict__ dst, unsigned lm) {
  const size_t idx = n.r0 + n.x;
  T* dw = dst + 18 * g.plane;
#pragma unroll
  for (int i = 0; i < 9; ++i) __builtin_nontemporal_store(fw[i], &dw[size_t(i) * g.plane + idx]);
  if (MASKED && (lm & 0x1FEu)) {
#pragma unroll
    for (int i = 1; i < 9; ++i)
      if ((lm >> opp(i)) & 1u) dw[size_t(opp(i)) * g.plane + push_off(n, i)] = fw[i];
  }
}

// Kinetics source tau w_i Phi on one species' populations.
template <typename T>
__device__ __forceinline__ void add_kinetics(T f[9], T ph) {
  f[0] += ph * T(4.0 / 9.0);
#pragma unroll
  for (int i = 1; i < 5; ++i) f[i] += ph * T(1.0 / 9.0);
#pragma unroll
  for (int i = 5; i < 9; ++i) f[i] += ph * T(1.0 / 36.0);
}

// Collision of the gathered node values and the stores: record (u, j_v),
// post-collision state, wall slots.  `lm` is the node's link word (0
// without a mask).
//
// LAG: second-order source term of (eq:LBEG) with kappa_t = 1, kappa_x = 0
// by the explicit characteristic difference: tau F + (tau/2)(F - F_prev)
// = tau (3/2 F - 1/2 F_prev) per population.  lag [2][plane] holds the
// kinetics r_u u (1-u), a_uv u - b_v v of the previous step at this node
// (the static control cancels in the difference) and is overwritten with
// this step's; at the first step there is no previous value and the
// difference is zero.
//
// kVarImplicit: the gathered values are g (phi at the first step, which
// starts from phi^0 = w~ Theta_0); Theta comes from implicit_solve, phi =
// g + (tau/2) w Phi, and the stored post-collision value is
// g* = relax(phi) + tau S + (tau/2) w Phi: the departure half of the
// difference, -(tau/2) F_i(x, t), plus the arrival half, which the next
// step's node solve takes at x + e_i.  The first moment of g equals that of
// phi (sum_i w_i e_i = 0).
//
// kVarThree: fw holds the third species; the record gains j_w (planes 3
// and 4), the chemotactic flux of u gains u Bw j_w (the repulsion
// A_u2 grad w with grad w = -K_w j_w / (tau d_w Cs^2)), and w relaxes with
// its own rates and receives Phi_w = a_w u - b_w w + s_w.
template <typename T, bool MASKED, int VAR = kVarFirst>
__device__ __forceinline__ void forward_collide_store(const Geometry& g, const NodeIdx& n,
                                                      const ModelCoef<T>& m, T fu[9], T fv[9],
                                                      T c, T* __restrict__ dst,
                                                      T* __restrict__ rec, unsigned lm,
                                                      T* __restrict__ lag = nullptr,
                                                      bool first = false,
                                                      T* __restrict__ fw = nullptr) {
  constexpr bool W3 = VAR == kVarThree;
  constexpr bool LAG = VAR == kVarExplicit;
  const size_t idx = n.r0 + n.x;
  // macroscopic values (UGS) and the first moment of v
  T u = T(0), v = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    u += fu[i];
    v += fv[i];
  }
  const T jx = fv[1] - fv[3] + fv[5] - fv[6] - fv[7] + fv[8];
  const T jy = fv[2] - fv[4] + fv[5] + fv[6] - fv[7] - fv[8];
  if (VAR == kVarImplicit && !first) {
    const T Gu = u, Gv = v;
    implicit_solve(m, Gu, Gv, c, u, v);
    const T hu = T(0.5) * m.r_u * u * (T(1) - u);
    const T hv = T(0.5) * (m.a_uv * u - m.b_v * v + c);
    add_sources(fu, fv, hu, T(0), T(0), hv);  // phi = g + (tau/2) w Phi
  }
  T wv = T(0), kx = T(0), ky = T(0);
  if (W3) {
#pragma unroll
    for (int i = 0; i < 9; ++i) wv += fw[i];
    kx = fw[1] - fw[3] + fw[5] - fw[6] - fw[7] + fw[8];
    ky = fw[2] - fw[4] + fw[5] + fw[6] - fw[7] - fw[8];
  }
  if (rec != nullptr) {
    // the record is read back only by the adjoint sweep, much later.  The
    // solid lanes of a mixed wavefront store it too (zeros, read by nobody)
    // so that the stores fill whole 64-byte chunks: a store instruction
    // that leaves part of a chunk unwritten costs a read-modify-write
    __builtin_nontemporal_store(u, &rec[idx]);
    __builtin_nontemporal_store(jx, &rec[g.plane + idx]);
    __builtin_nontemporal_store(jy, &rec[2 * g.plane + idx]);
    if (W3) {
      __builtin_nontemporal_store(kx, &rec[3 * g.plane + idx]);
      __builtin_nontemporal_store(ky, &rec[4 * g.plane + idx]);
    }
  }
  // chemotactic source: A_u1 grad v = u * B * j_v with the local gradient
  // grad v = -K_v j_v / (tau d_v Cs^2)
  T ax = u * (m.b00 * jx + m.b01 * jy);
  T ay = u * (m.b10 * jx + m.b11 * jy);
  if (W3) {
    ax += u * (m.bw00 * kx + m.bw01 * ky);
    ay += u * (m.bw10 * kx + m.bw11 * ky);
  }
  const T ru = m.r_u * u * (T(1) - u);
  const T rv = m.a_uv * u - m.b_v * v;
  T phu, phv;
  if (LAG) {
    const T lu = first ? ru : lag[idx];
    const T lv = first ? rv : lag[g.plane + idx];
    phu = T(1.5) * ru - T(0.5) * lu;
    phv = T(1.5) * rv - T(0.5) * lv + c;
    lag[idx] = ru;  // every lane, as the record
    lag[g.plane + idx] = rv;
  } else if (VAR == kVarImplicit) {
    phu = T(0.5) * ru;
    phv = T(0.5) * (rv + c);
  } else {
    phu = ru;
    phv = rv + c;
  }
  T t1, t2;
  relax(fu, u, m.u, t1, t2);
  relax(fv, v, m.v, t1, t2);
  add_sources(fu, fv, phu, ax, ay, phv);
  if (W3) {
    relax(fw, wv, m.w, t1, t2);
    add_kinetics(fw, m.a_w * u - m.b_w * wv + m.s_w);
  }
  // solid nodes of mixed wavefronts computed on zeros; they store no state
  // (their slots hold the neighbours' wall stores)
  if (MASKED && (lm & 1u)) return;
  store_state<T, MASKED>(g, n, fu, fv, dst, lm);
  if (W3) store_w<T, MASKED>(g, n, fw, dst, lm);
}

// Tangent-linear step (sensitivity LBE, LIBEG-V) at a node: the derivative
// of the collision of forward step n applied to the gathered perturbation
// (fu, fv), with the recorded pre-collision u and j_v of that step and the
// control perturbation dc.  The relaxation is linear (relax with theta =
// the perturbed density); the sources give
//   d(u B j_v) = du B j_v + u B dj_v,   dPhi_u = r_u (1 - 2u) du,
//   dPhi_v = a_uv du - b_v dv + dc.
// LAG: the second-order source as in the forward, on the perturbed
// kinetics; dlag [2][plane] carries their previous-step values.
// kVarImplicit: the perturbation of g; the node equation linearised at the
// recorded u gives du = dG_u / (1 - (tau/2) r_u (1 - 2u)) and
// dv = (dG_v + (tau/2)(a_uv du + dc)) / (1 + (tau/2) b_v) (none at the first
// step, whose input is dphi^0).
// kVarThree: fw holds the perturbation of the third species;
// d(u Bw j_w) = du Bw j_w + u Bw dj_w with j_w recorded, and
// dPhi_w = a_w du - b_w dw.
template <typename T, bool MASKED, int VAR = kVarFirst>
__device__ __forceinline__ void tlm_collide_store(const Geometry& g, const NodeIdx& n,
                                                  const ModelCoef<T>& m, T fu[9], T fv[9],
                                                  T dc, const T* __restrict__ rec,
                                                  T* __restrict__ dst, unsigned lm,
                                                  T* __restrict__ dlag = nullptr,
                                                  bool first = false,
                                                  T* __restrict__ fw = nullptr) {
  constexpr bool LAG = VAR == kVarExplicit;
  constexpr bool W3 = VAR == kVarThree;
  const size_t idx = n.r0 + n.x;
  const T u = __builtin_nontemporal_load(&rec[idx]);
  const T jx = __builtin_nontemporal_load(&rec[g.plane + idx]);
  const T jy = __builtin_nontemporal_load(&rec[2 * g.plane + idx]);
  T du = T(0), dv = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    du += fu[i];
    dv += fv[i];
  }
  if (VAR == kVarImplicit && !first) {
    du = du / (T(1) - T(0.5) * m.r_u * (T(1) - T(2) * u));
    dv = (dv + T(0.5) * (m.a_uv * du + dc)) / (T(1) + T(0.5) * m.b_v);
    const T hu = T(0.5) * m.r_u * (T(1) - T(2) * u) * du;
    const T hv = T(0.5) * (m.a_uv * du - m.b_v * dv + dc);
    add_sources(fu, fv, hu, T(0), T(0), hv);  // dphi = dg + (tau/2) w dPhi
  }
  const T djx = fv[1] - fv[3] + fv[5] - fv[6] - fv[7] + fv[8];
  const T djy = fv[2] - fv[4] + fv[5] + fv[6] - fv[7] - fv[8];
  T dax = du * (m.b00 * jx + m.b01 * jy) + u * (m.b00 * djx + m.b01 * djy);
  T day = du * (m.b10 * jx + m.b11 * jy) + u * (m.b10 * djx + m.b11 * djy);
  T dw = T(0);
  if (W3) {
    const T kx = __builtin_nontemporal_load(&rec[3 * g.plane + idx]);
    const T ky = __builtin_nontemporal_load(&rec[4 * g.plane + idx]);
#pragma unroll
    for (int i = 0; i < 9; ++i) dw += fw[i];
    const T dkx = fw[1] - fw[3] + fw[5] - fw[6] - fw[7] + fw[8];
    const T dky = fw[2] - fw[4] + fw[5] + fw[6] - fw[7] - fw[8];
    dax += du * (m.bw00 * kx + m.bw01 * ky) + u * (m.bw00 * dkx + m.bw01 * dky);
    day += du * (m.bw10 * kx + m.bw11 * ky) + u * (m.bw10 * dkx + m.bw11 * dky);
  }
  const T dru = m.r_u * (T(1) - T(2) * u) * du;
  const T drv = m.a_uv * du - m.b_v * dv;
  T dphu, dphv;
  if (LAG) {
    const T lu = first ? dru : dlag[idx];
    const T lv = first ? drv : dlag[g.plane + idx];
    dphu = T(1.5) * dru - T(0.5) * lu;
    dphv = T(1.5) * drv - T(0.5) * lv + dc;
    if (!(MASKED && (lm & 1u))) {
      dlag[idx] = dru;
      dlag[g.plane + idx] = drv;
    }
  } else if (VAR == kVarImplicit) {
    dphu = T(0.5) * dru;
    dphv = T(0.5) * (drv + dc);
  } else {
    dphu = dru;
    dphv = drv + dc;
  }
  T t1, t2;
  relax(fu, du, m.u, t1, t2);
  relax(fv, dv, m.v, t1, t2);
  add_sources(fu, fv, dphu, dax, day, dphv);
  if (W3) {
    relax(fw, dw, m.w, t1, t2);
    add_kinetics(fw, m.a_w * du - m.b_w * dw);
  }
  if (MASKED && (lm & 1u)) return;
  store_state<T, MASKED>(g, n, fu, fv, dst, lm);
  if (W3) store_w<T, MASKED>(g, n, fw, dst, lm);
}

// Continuous-adjoint step (Section 3.2.2: the continuous adjoint system of
// the two-species instance solved by the MRT scheme in reversed time) at a
// node, from the gathered adjoint populations (fp of p, fq of q) and the
// recorded forward u, j_v at this time:
//   p_s = div(D_u grad p) + chi (C grad v).grad p + r_u (1 - 2u) p + a_uv q
//   q_s = div(D_v grad q) - b_v q - div(chi u C^T grad p)
// p relaxes like u and q like v; the advection and the couplings are
// scalar sources, the cross-diffusion of q a flux source, as the
// chemotaxis of u in the forward.  Accumulates g += tau q (pre-collision).
template <typename T, bool MASKED, bool FIRST>
__device__ __forceinline__ void cadj_collide_store(const Geometry& g, const NodeIdx& n,
                                                   const ModelCoef<T>& m, const CadjCoef<T>& cc,
                                                   T fp[9], T fq[9], const T* __restrict__ rec,
                                                   T* __restrict__ dst, double* __restrict__ gacc,
                                                   unsigned lm) {
  const size_t idx = n.r0 + n.x;
  const T u = __builtin_nontemporal_load(&rec[idx]);
  const T jvx = __builtin_nontemporal_load(&rec[g.plane + idx]);
  const T jvy = __builtin_nontemporal_load(&rec[2 * g.plane + idx]);
  T P = T(0), Qv = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    P += fp[i];
    Qv += fq[i];
  }
  const T jpx = fp[1] - fp[3] + fp[5] - fp[6] - fp[7] + fp[8];
  const T jpy = fp[2] - fp[4] + fp[5] + fp[6] - fp[7] - fp[8];
  const bool solid = MASKED && (lm & 1u);
  if (!solid) {
    if (FIRST)
      gacc[idx] = double(Qv);
    else
      gacc[idx] += double(Qv);
  }
  const T adv = jpx * (cc.m00 * jvx + cc.m01 * jvy) + jpy * (cc.m10 * jvx + cc.m11 * jvy);
  const T php = m.r_u * (T(1) - T(2) * u) * P + m.a_uv * Qv + adv;
  const T phq = -m.b_v * Qv;
  const T aqx = u * (cc.q00 * jpx + cc.q01 * jpy);
  const T aqy = u * (cc.q10 * jpx + cc.q11 * jpy);
  T t1, t2;
  relax(fp, P, m.u, t1, t2);
  relax(fq, Qv, m.v, t1, t2);
  add_sources(fp, fq, php, T(0), T(0), phq);
  // flux source of q: 3 w_i e_i . a_q
  const T x3 = aqx * T(1.0 / 3.0), y3 = aqy * T(1.0 / 3.0);
  const T x12 = aqx * T(1.0 / 12.0), y12 = aqy * T(1.0 / 12.0);
  fq[1] += x3;
  fq[2] += y3;
  fq[3] -= x3;
  fq[4] -= y3;
  fq[5] += x12 + y12;
  fq[6] += y12 - x12;
  fq[7] -= x12 + y12;
  fq[8] += x12 - y12;
  if (solid) return;
  store_state<T, MASKED>(g, n, fp, fq, dst, lm);
}

// One forward step (eq:LBE with S, PhiS, MF, MC) at node n.  Recording is a
// run-time flag (rec != null), not a template parameter: the recorded and
// the plain steps then run the same machine code, so a checkpointed
// recomputation reproduces the recorded trajectory bit for bit.
template <typename T, bool PERIODIC, bool MASKED, bool FIRST, int VAR = kVarFirst>
__device__ __forceinline__ void forward_node(
    const Geometry& g, const NodeIdx& n, const ModelCoef<T>& m, const T* __restrict__ src, T* __restrict__ dst,
    const T* __restrict__ u0, const T* __restrict__ v0,
    const T* __restrict__ ctrl, T* __restrict__ rec, T* __restrict__ lag = nullptr,
    const T* __restrict__ w0 = nullptr) {
  unsigned lm = 0;
  if (MASKED) {
    const unsigned flag = wave_flag(g, n);
    if (flag == 2u) return;  // wavefront inside a solid region
    lm = link_of(g, flag, n.r0 + n.x);
  }
  // a solid node of a mixed wavefront loads nothing and collides zeros: it
  // stores no state (its slots hold the neighbours' wall stores) but takes
  // part in the record stores
  const bool solid = MASKED && (lm & 1u);
  T fu[9], fv[9], c = T(0);
  if (solid) {
#pragma unroll
    for (int i = 0; i < 9; ++i) fu[i] = fv[i] = T(0);
  } else {
    forward_gather<T, PERIODIC, FIRST>(g, n, m, src, u0, v0, ctrl, fu, fv, c);
  }
  if (VAR == kVarThree) {
    T fw[9];
    if (solid) {
#pragma unroll
      for (int i = 0; i < 9; ++i) fw[i] = T(0);
    } else {
      gather_w<T, PERIODIC, FIRST>(g, n, m, src, w0, fw);
    }
    forward_collide_store<T, MASKED, VAR>(g, n, m, fu, fv, c, dst, rec, lm, lag, FIRST, fw);
  } else {
    forward_collide_store<T, MASKED, VAR>(g, n, m, fu, fv, c, dst, rec, lm, lag, FIRST);
  }
}

// Terminal streaming: the state after the last step and its sums.  IMPL
// (implicit characteristic difference): the streamed values are g; Theta^N
// comes from the node solve and the state is phi^N = g + (tau/2) w Phi.
// W3: the third species' populations are also streamed into the state.
template <typename T, bool PERIODIC, bool MASKED, bool IMPL = false, bool W3 = false>
__device__ __forceinline__ void finalize_node(
    const Geometry& g, const NodeIdx& n, const T* __restrict__ src, T* __restrict__ state,
    T* __restrict__ uN, T* __restrict__ vN, const ModelCoef<T>* m = nullptr,
    const T* __restrict__ ctrl = nullptr) {
  const size_t idx = n.r0 + n.x;
  const bool solid = MASKED && (link_of(g, wave_flag(g, n), idx) & 1u);
  T fu[9], fv[9];
  if (solid) {
#pragma unroll
    for (int i = 0; i < 9; ++i) fu[i] = fv[i] = T(0);
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const size_t o = pull_src<PERIODIC>(n, i, g.plane);
      fu[i] = src[o];
      fv[i] = src[9 * g.plane + o];
    }
  }
  T u = T(0), v = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    u += fu[i];
    v += fv[i];
  }
  if (IMPL && !solid) {
    const T c = ctrl[idx];
    const T Gu = u, Gv = v;
    implicit_solve(*m, Gu, Gv, c, u, v);
    add_sources(fu, fv, T(0.5) * m->r_u * u * (T(1) - u), T(0), T(0),
                T(0.5) * (m->a_uv * u - m->b_v * v + c));
  }
  if (uN) uN[idx] = u;
  if (vN) vN[idx] = v;
  if (state) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      state[size_t(i) * g.plane + idx] = fu[i];
      state[size_t(9 + i) * g.plane + idx] = fv[i];
    }
    if (W3) {
#pragma unroll
      for (int i = 0; i < 9; ++i)
        state[size_t(18 + i) * g.plane + idx] =
            solid ? T(0) : src[18 * g.plane + pull_src<PERIODIC>(n, i, g.plane)];
    }
  }
}

// --------------------------------------------------------------- adjoint

// LAG: adjoint of the second-order source.  The scheme's state then also
// holds the previous step's kinetics F_prev; mu [2][plane] is the adjoint
// of the kinetics this step stores for the next one.  With sigma = w . nu
// per species, the adjoint of this step's kinetics is rho = 3/2 sigma + mu
// (sigma + mu at step 0, where F_prev = F), and the new mu = -1/2 sigma.
// FIRST (step N-1) reads no mu: nothing reads the last stored kinetics.
// step0 marks step 0 (a run-time flag: LAST is set only when dJ/du0,
// dJ/dv0 are requested).
//
// kVarImplicit: the adjoint of g.  With A the relaxation (phi -> phi -
// C (phi - w~ Theta)), a step maps g to g* = A g + (tau/2)(A w + w) Phi +
// tau S with Theta from the node equation, so the sensitivity to Phi_s is
// kappa_s = (tau/2)(w . A^T nu_s + sigma_s); through the linearised node
// solve (alpha = 1 / (1 - (tau/2) r_u (1 - 2u)), beta = 1 / (1 +
// (tau/2) b_v)) the sums G_s receive Gbar_v = beta vbar and Gbar_u =
// alpha (ubar + (tau/2) a_uv beta vbar), and the control kappa_v beta.  At
// step 0 the input is phi^0 itself: kappa_s = (tau/2) sigma_s, no solve.
//
// kVarThree: the adjoint of w as well (planes 18..26; zero at the terminal
// step, the cost not depending on w): sigma_w enters u's source through
// a_w, w's own through -b_w; the repulsive flux u Bw j_w adds
// p . (Bw j_w) to u's and e_i . (u Bw^T p) to w's.
//
// adjoint_node = adjoint_gather + adjoint_update.
//
// Adjoint gather of node n (FIRST: the terminal seeds), the half of the
// node update that loads; adjoint_update finishes it.
template <typename T, bool PERIODIC, bool MASKED, bool FIRST, int VAR = kVarFirst>
__device__ __forceinline__ void adjoint_gather(const Geometry& g, const NodeIdx& n,
                                               const T* __restrict__ src,
                                               const T* __restrict__ seed_u,
                                               const T* __restrict__ seed_v, unsigned lm,
                                               T nu[9], T nv[9], T nw[9]) {
  const size_t idx = n.r0 + n.x;
  // reverse streaming: nu_i(x) = lambda_i(x + e_i), or lambda_opp(i)(x)
  // when x + e_i is a wall (exact transpose of the pull with bounce-back)
  if (FIRST) {
    // terminal condition lambda_i^N = seed for every i (psi(T) = dI0/dphi);
    // the seed fields carry no wall slots, so walls are tested here
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const bool wall = (!PERIODIC && push_outside(n, i)) ||
                        (MASKED && ((lm >> opp(i)) & 1u));
      const size_t o = wall ? idx : push_off(n, i);
      nu[i] = seed_u[o];
      nv[i] = seed_v ? seed_v[o] : T(0);
    }
  } else {
    const T* sv = src + 9 * g.plane;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const size_t o = gather_src<PERIODIC>(n, i, g.plane);
      nu[i] = src[o];
      nv[i] = sv[o];
    }
  }
  constexpr bool W3 = VAR == kVarThree;
  if (W3) {
    if (FIRST) {
#pragma unroll
      for (int i = 0; i < 9; ++i) nw[i] = T(0);
    } else {
      const T* sw = src + 18 * g.plane;
#pragma unroll
      for (int i = 0; i < 9; ++i)
        nw[i] = sw[gather_src<PERIODIC>(n, i, g.plane)];
    }
  }
}

// The rest of the adjoint node update after adjoint_gather: sources,
// collision, gradient accumulation and the stores.
template <typename T, bool PERIODIC, bool MASKED, bool FIRST, bool LAST, int VAR = kVarFirst>
__device__ __forceinline__ void adjoint_update(
    const Geometry& g, const NodeIdx& n, const ModelCoef<T>& m, T nu[9], T nv[9], T nw[9],
    T* __restrict__ dst, const T* __restrict__ rec, double* __restrict__ gacc,
    T* __restrict__ adj_u0, T* __restrict__ adj_v0, T* __restrict__ mu, bool step0,
    unsigned lm) {
  const size_t idx = n.r0 + n.x;
  constexpr bool W3 = VAR == kVarThree;
  // weighted sums: sigma = w . nu, p = (tau/Cs^2) sum_i w_i nu_u,i e_i
  const T su_ = T(4.0 / 9.0) * nu[0] +
                T(1.0 / 9.0) * (nu[1] + nu[2] + nu[3] + nu[4]) +
                T(1.0 / 36.0) * (nu[5] + nu[6] + nu[7] + nu[8]);
  const T sv_ = T(4.0 / 9.0) * nv[0] +
                T(1.0 / 9.0) * (nv[1] + nv[2] + nv[3] + nv[4]) +
                T(1.0 / 36.0) * (nv[5] + nv[6] + nv[7] + nv[8]);
  const T px = T(1.0 / 3.0) * (nu[1] - nu[3]) +
               T(1.0 / 12.0) * (nu[5] - nu[6] - nu[7] + nu[8]);
  const T py = T(1.0 / 3.0) * (nu[2] - nu[4]) +
               T(1.0 / 12.0) * (nu[5] + nu[6] - nu[7] - nu[8]);
  constexpr bool LAG = VAR == kVarExplicit;
  constexpr bool IMPL = VAR == kVarImplicit;
  // gradient w.r.t. the control on v: dF_v,i/dc = tau w_i (the implicit
  // form adds its share below)
  if (!IMPL) {
    if (FIRST)
      gacc[idx] = double(sv_);
    else
      gacc[idx] += double(sv_);
  }
  // recorded forward quantities of step n
  const T u = __builtin_nontemporal_load(&rec[idx]);
  const T jx = __builtin_nontemporal_load(&rec[g.plane + idx]);
  const T jy = __builtin_nontemporal_load(&rec[2 * g.plane + idx]);
  const T bjx = m.b00 * jx + m.b01 * jy;
  const T bjy = m.b10 * jx + m.b11 * jy;
  // transposed sources: d(tau S_u + tau Phi_u)/dphi_u is rank one along 1,
  // d(tau S_u)/dphi_v = (tau/Cs^2) diag(w) E u B E^T, dPhi_v/dphi = (a, -b).
  T rho_u = su_, rho_v = sv_;
  if (LAG) {
    const T mu_u = FIRST ? T(0) : mu[idx];
    const T mu_v = FIRST ? T(0) : mu[g.plane + idx];
    if (step0) {
      rho_u = su_ + mu_u;
      rho_v = sv_ + mu_v;
    } else {
      rho_u = T(1.5) * su_ + mu_u;
      rho_v = T(1.5) * sv_ + mu_v;
      mu[idx] = T(-0.5) * su_;
      mu[g.plane + idx] = T(-0.5) * sv_;
    }
  }
  const T qx = u * (m.b00 * px + m.b10 * py);
  const T qy = u * (m.b01 * px + m.b11 * py);
  T wu, wv;
  if (!IMPL) {
    T cu = rho_u * m.r_u * (T(1) - T(2) * u) + px * bjx + py * bjy +
           rho_v * m.a_uv;
    const T cv = -rho_v * m.b_v;
    if (W3) {
      const T kx = __builtin_nontemporal_load(&rec[3 * g.plane + idx]);
      const T ky = __builtin_nontemporal_load(&rec[4 * g.plane + idx]);
      const T sw_ = T(4.0 / 9.0) * nw[0] + T(1.0 / 9.0) * (nw[1] + nw[2] + nw[3] + nw[4]) +
                    T(1.0 / 36.0) * (nw[5] + nw[6] + nw[7] + nw[8]);
      cu += px * (m.bw00 * kx + m.bw01 * ky) + py * (m.bw10 * kx + m.bw11 * ky) +
            sw_ * m.a_w;
      T a1, a2;
      relax(nw, T(0), m.wt, a1, a2);
      const T ww = m.w.e_eq * a1 + m.w.eps_eq * a2 - sw_ * m.b_w;
      const T rx = u * (m.bw00 * px + m.bw10 * py);
      const T ry = u * (m.bw01 * px + m.bw11 * py);
#pragma unroll
      for (int i = 0; i < 9; ++i) nw[i] += ww;
      nw[1] += rx;
      nw[2] += ry;
      nw[3] -= rx;
      nw[4] -= ry;
      nw[5] += rx + ry;
      nw[6] += ry - rx;
      nw[7] -= rx + ry;
      nw[8] += rx - ry;
    }
    // adjoint collision: nu - C^T nu + 1 * weq^T C^T nu  (AEDs with O = 1 weq^T)
    T a1, a2;
    relax(nu, T(0), m.ut, a1, a2);
    wu = m.u.e_eq * a1 + m.u.eps_eq * a2 + cu;
    relax(nv, T(0), m.vt, a1, a2);
    wv = m.v.e_eq * a1 + m.v.eps_eq * a2 + cv;
  } else {
    T a1, a2;
    relax(nu, T(0), m.ut, a1, a2);
    const T eu = m.u.e_eq * a1 + m.u.eps_eq * a2;
    relax(nv, T(0), m.vt, a1, a2);
    const T ev = m.v.e_eq * a1 + m.v.eps_eq * a2;
    T ku = T(0.5) * su_, kv = T(0.5) * sv_;
    if (!step0) {
      // w . A^T nu = w . (relaxed nu) + e (sum_i w_i = 1)
      const T tu = T(4.0 / 9.0) * nu[0] + T(1.0 / 9.0) * (nu[1] + nu[2] + nu[3] + nu[4]) +
                   T(1.0 / 36.0) * (nu[5] + nu[6] + nu[7] + nu[8]) + eu;
      const T tv = T(4.0 / 9.0) * nv[0] + T(1.0 / 9.0) * (nv[1] + nv[2] + nv[3] + nv[4]) +
                   T(1.0 / 36.0) * (nv[5] + nv[6] + nv[7] + nv[8]) + ev;
      ku = T(0.5) * (tu + su_);
      kv = T(0.5) * (tv + sv_);
    }
    const T ubar = ku * m.r_u * (T(1) - T(2) * u) + kv * m.a_uv + px * bjx + py * bjy;
    const T vbar = -kv * m.b_v;
    T gu = ubar, gv = vbar, gc = kv;
    if (!step0) {
      const T beta = T(1) / (T(1) + T(0.5) * m.b_v);
      const T alpha = T(1) / (T(1) - T(0.5) * m.r_u * (T(1) - T(2) * u));
      gv = beta * vbar;
      gu = alpha * (ubar + T(0.5) * m.a_uv * gv);
      gc = kv * beta;
    }
    gacc[idx] += double(gc);  // initialised by the terminal transform
    wu = eu + gu;
    wv = ev + gv;
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    nu[i] += wu;
    nv[i] += wv;
  }
  nv[1] += qx;
  nv[2] += qy;
  nv[3] -= qx;
  nv[4] -= qy;
  nv[5] += qx + qy;
  nv[6] += qy - qx;
  nv[7] -= qx + qy;
  nv[8] += qx - qy;
  if (LAST) {
    // transpose of phi_i^0 = w_i Theta_0
    if (adj_u0)
      adj_u0[idx] = m.u.w_rest * nu[0] +
                    m.u.w_axis * (nu[1] + nu[2] + nu[3] + nu[4]) +
                    m.u.w_diag * (nu[5] + nu[6] + nu[7] + nu[8]);
    if (adj_v0)
      adj_v0[idx] = m.v.w_rest * nv[0] +
                    m.v.w_axis * (nv[1] + nv[2] + nv[3] + nv[4]) +
                    m.v.w_diag * (nv[5] + nv[6] + nv[7] + nv[8]);
  } else if (dst) {
    T* dv = dst + 9 * g.plane;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      __builtin_nontemporal_store(nu[i], &dst[size_t(i) * g.plane + idx]);
      __builtin_nontemporal_store(nv[i], &dv[size_t(i) * g.plane + idx]);
    }
    if (W3) {
      T* dw = dst + 18 * g.plane;
#pragma unroll
      for (int i = 0; i < 9; ++i)
        __builtin_nontemporal_store(nw[i], &dw[size_t(i) * g.plane + idx]);
    }
    if (MASKED && (lm & 0x1FEu)) {
      // wall stores of the adjoint: the next gather in direction i at x
      // reads plane i at the solid node x + e_i and must find lambda_opp(i)(x)
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        if ((lm >> opp(i)) & 1u) {
          const size_t o = size_t(i) * g.plane + push_off(n, i);
          dst[o] = nu[opp(i)];
          dv[o] = nv[opp(i)];
          if (W3) dst[18 * g.plane + o] = nw[opp(i)];
        }
      }
    }
  }
}

template <typename T, bool PERIODIC, bool MASKED, bool FIRST, bool LAST, int VAR = kVarFirst>
__device__ __forceinline__ void adjoint_node(
    const Geometry& g, const NodeIdx& n, const ModelCoef<T>& m, const T* __restrict__ src, T* __restrict__ dst,
    const T* __restrict__ seed_u, const T* __restrict__ seed_v,
    const T* __restrict__ rec, double* __restrict__ gacc,
    T* __restrict__ adj_u0, T* __restrict__ adj_v0, T* __restrict__ mu = nullptr,
    bool step0 = false) {
  const size_t idx = n.r0 + n.x;
  unsigned lm = 0;
  if (MASKED) {
    const unsigned flag = wave_flag(g, n);
    if (FIRST || LAST) {
      // single steps: resolve solid nodes up front, they own outputs
      lm = g.link[idx];
      if (lm & 1u) {
        if (FIRST) gacc[idx] = 0.0;
        if (LAST) {
          if (adj_u0) adj_u0[idx] = T(0);
          if (adj_v0) adj_v0[idx] = T(0);
        }
        return;
      }
    } else {
      if (flag == 2u) return;  // wavefront inside a solid region
      lm = link_of(g, flag, idx);
      // a solid node of a mixed wavefront: no update (taking part in the
      // gradient's read-modify-write with zeros measured 4% slower)
      if (lm & 1u) return;
    }
  }
  T nu[9], nv[9], nw[9];
  adjoint_gather<T, PERIODIC, MASKED, FIRST, VAR>(g, n, src, seed_u, seed_v, lm, nu, nv, nw);
  adjoint_update<T, PERIODIC, MASKED, FIRST, LAST, VAR>(g, n, m, nu, nv, nw, dst, rec, gacc,
                                                        adj_u0, adj_v0, mu, step0, lm);
}

// ------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}

// Block reduction of kRedSlots values (slot 3 is a max, the others sums);
// lane 0 of the block writes the block partial.
__device__ void block_reduce_store(double vals[kRedSlots], double* out) {
  __shared__ double lds[kRedSlots][kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kRedSlots; ++k) {
    double r = (k == 3) ? wave_max(vals[k]) : wave_sum(vals[k]);
    if (lane == 0) lds[k][wave] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kRedSlots; ++k) {
      double r = lds[k][0];
      for (int w = 1; w < kBlock / 64; ++w)
        r = (k == 3) ? fmax(r, lds[k][w]) : r + lds[k][w];
      out[k] = r;
    }
  }
}

}  // namespace dev
}  // namespace mrt
