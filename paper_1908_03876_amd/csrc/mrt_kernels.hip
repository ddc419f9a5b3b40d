// gfx950 kernels of the two-species D2Q9 MRT chemotaxis step, its exact
// discrete adjoint (AMRT) and the cost / gradient / update reductions.
//
// Method: arXiv:1908.03876, Section 3.1 (eq:LBE, S, PhiS, MF, MC, phieq,
// BC11, the relaxation matrix Pi and D = d Cs^2 tau (K^-1 - I/2)) and
// Section 3.2.1 (LIBEG, CAE, AEDs, RFS1, CAEL, gradientLattice).
//
// Design (memory-bound stencil, no MFMA):
//  * One thread per lattice node, 256-thread blocks along x; every
//    population is read once and written once per step in SoA planes, so
//    each wavefront issues 18 coalesced 256-byte loads and 18 stores.
//  * The kernel stores post-collision states and pulls: node x gathers
//    phi*_i(x - e_i) (or its own phi*_opp(i) when x - e_i is solid, halfway
//    bounce-back).  Collision runs in registers in moment space; M0^-1 is
//    applied as M0^T with the row norms folded into the rates.
//  * The adjoint is a gather too: nu_i(x) = lambda_i(x + e_i), or
//    lambda_opp(i)(x) when x + e_i is solid (exact transpose of the pull).
//  * Work-group order is remapped so that each of the 8 XCDs walks a
//    contiguous band of rows (its L2 keeps the shifted-row and edge lines).
//  * State planes and the trajectory record are streamed with non-temporal
//    stores (and non-temporal loads in the adjoint): they are touched once
//    per sweep and would only evict the link mask, control and gradient.
//  * Walls cost no test in the pull: a node whose population streams into
//    a solid neighbour also parks it in that neighbour's (otherwise unused)
//    slot of the opposite plane, where the next pull finds it.
//  * Reductions: wave shuffles (64 lanes), LDS across waves, one partial per
//    block, then a single-block pass in fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "mrt_device.h"
#include "mrt_internal.h"

namespace mrt {
namespace {

using namespace dev;

// -------------------------------------------------------------- link mask

// bit 0: node solid; bit i (1..8): x - e_i is a solid node of the lattice
// (wrapped when periodic; outside a non-periodic lattice is not a node and
// is handled from the coordinates).
__global__ void build_link_kernel(Geometry g, int periodic,
                                  const uint8_t* __restrict__ mask,
                                  uint16_t* __restrict__ link,
                                  uint32_t* __restrict__ wflag) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx) return;
  const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  uint16_t bits = 0;
  for (int i = 0; i < 9; ++i) {
    int xs = x - ex[i], ys = y - ey[i];
    const bool out = xs < 0 || ys < 0 || xs >= g.nx || ys >= g.ny;
    if (out && !periodic) continue;
    xs = (xs + g.nx) % g.nx;
    ys = (ys + g.ny) % g.ny;
    if (mask[size_t(ys) * g.pitch + xs]) bits |= uint16_t(1u << i);
  }
  link[size_t(y) * g.pitch + x] = bits;
  // blocks are 256 wide along x, so each wavefront is one 64-node segment
  const unsigned long long any = __ballot(bits != 0);
  const unsigned long long fluid = __ballot((bits & 1u) == 0);
  if ((threadIdx.x & 63) == 0)
    wflag[size_t(y) * g.nsx + (x >> 6)] = fluid == 0ull ? 2u : (any != 0ull);
}

template <typename T, bool PERIODIC, bool MASKED, bool FIRST, int VAR>
__global__ __launch_bounds__(kBlock) void forward_step_kernel(
    Geometry g, ModelCoef<T> m, const T* __restrict__ src, T* __restrict__ dst,
    const T* __restrict__ u0, const T* __restrict__ v0,
    const T* __restrict__ ctrl, T* __restrict__ rec, T* __restrict__ lag,
    const T* __restrict__ w0) {
  NodeIdx n;
  if (!node_of_block(g, n)) return;
  forward_node<T, PERIODIC, MASKED, FIRST, VAR>(g, n, m, src, dst, u0, v0, ctrl, rec, lag, w0);
}

template <typename T, bool PERIODIC, bool MASKED, bool IMPL, bool W3>
__global__ __launch_bounds__(kBlock) void finalize_kernel(
    Geometry g, ModelCoef<T> m, const T* __restrict__ src, const T* __restrict__ ctrl,
    T* __restrict__ state, T* __restrict__ uN, T* __restrict__ vN) {
  NodeIdx n;
  if (!node_of_block(g, n)) return;
  finalize_node<T, PERIODIC, MASKED, IMPL, W3>(g, n, src, state, uN, vN, &m, ctrl);
}

// Pull of the populations streamed into node n after the last step (zeros
// on solid nodes) and their sums G.
template <typename T, bool PERIODIC, bool MASKED>
__device__ __forceinline__ bool pull_sums(const Geometry& g, const NodeIdx& n,
                                          const T* __restrict__ src, T& Gu, T& Gv) {
  const size_t idx = n.r0 + n.x;
  if (MASKED && (link_of(g, wave_flag(g, n), idx) & 1u)) return false;
  Gu = T(0);
  Gv = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const size_t o = pull_src<PERIODIC>(n, i, g.plane);
    Gu += src[o];
    Gv += src[9 * g.plane + o];
  }
  return true;
}

// Implicit characteristic difference, terminal condition of the adjoint:
// the cost sees Theta^N, a function of the sums G^N of the last state, so
// the seeds (dJ/du^N, dJ/dv^N) = (a, b) become the adjoint of G^N:
// beta b and alpha (a + (tau/2) a_uv beta b), with alpha and beta of the
// node equation at u^N.  v^N also depends on the control (weight tau/2 in
// the node equation): the gradient accumulator starts at (tau/2) beta b.
// Zero on solid nodes.
template <typename T, bool PERIODIC, bool MASKED>
__global__ __launch_bounds__(kBlock) void implicit_terminal_kernel(
    Geometry g, ModelCoef<T> m, const T* __restrict__ src, const T* __restrict__ ctrl,
    const T* __restrict__ seed_u, const T* __restrict__ seed_v, T* __restrict__ out_u,
    T* __restrict__ out_v, double* __restrict__ gacc) {
  NodeIdx n;
  if (!node_of_block(g, n)) return;
  const size_t idx = n.r0 + n.x;
  T Gu, Gv;
  if (!pull_sums<T, PERIODIC, MASKED>(g, n, src, Gu, Gv)) {
    out_u[idx] = T(0);
    out_v[idx] = T(0);
    gacc[idx] = 0.0;
    return;
  }
  T u, v;
  implicit_solve(m, Gu, Gv, ctrl[idx], u, v);
  const T alpha = T(1) / (T(1) - T(0.5) * m.r_u * (T(1) - T(2) * u));
  const T beta = T(1) / (T(1) + T(0.5) * m.b_v);
  const T b = seed_v ? seed_v[idx] : T(0);
  out_v[idx] = beta * b;
  out_u[idx] = alpha * (seed_u[idx] + T(0.5) * m.a_uv * beta * b);
  gacc[idx] = double(T(0.5) * beta * b);
}

// Implicit characteristic difference, end of the tangent sweep: the
// perturbation of Theta^N from that of G^N (node equation linearised at the
// forward's u^N, with the control perturbation).
template <typename T, bool PERIODIC, bool MASKED>
__global__ __launch_bounds__(kBlock) void implicit_tlm_final_kernel(
    Geometry g, ModelCoef<T> m, const T* __restrict__ fsrc, const T* __restrict__ dsrc,
    const T* __restrict__ ctrl, const T* __restrict__ dc, T* __restrict__ duN,
    T* __restrict__ dvN) {
  NodeIdx n;
  if (!node_of_block(g, n)) return;
  const size_t idx = n.r0 + n.x;
  T Gu, Gv, dGu, dGv;
  if (!pull_sums<T, PERIODIC, MASKED>(g, n, fsrc, Gu, Gv)) {
    if (duN) duN[idx] = T(0);
    if (dvN) dvN[idx] = T(0);
    return;
  }
  pull_sums<T, PERIODIC, MASKED>(g, n, dsrc, dGu, dGv);
  T u, v;
  implicit_solve(m, Gu, Gv, ctrl[idx], u, v);
  const T du = dGu / (T(1) - T(0.5) * m.r_u * (T(1) - T(2) * u));
  const T dcc = dc ? dc[idx] : T(0);
  if (duN) duN[idx] = du;
  if (dvN) dvN[idx] = (dGv + T(0.5) * (m.a_uv * du + dcc)) / (T(1) + T(0.5) * m.b_v);
}

template <typename T, bool PERIODIC, bool MASKED, bool FIRST, bool LAST, int VAR>
__global__ __launch_bounds__(kBlock) void adjoint_step_kernel(
    Geometry g, ModelCoef<T> m, const T* __restrict__ src, T* __restrict__ dst,
    const T* __restrict__ seed_u, const T* __restrict__ seed_v,
    const T* __restrict__ rec, double* __restrict__ gacc,
    T* __restrict__ adj_u0, T* __restrict__ adj_v0, T* __restrict__ mu, int step0) {
  NodeIdx n;
  if (!node_of_block(g, n)) return;
  adjoint_node<T, PERIODIC, MASKED, FIRST, LAST, VAR>(g, n, m, src, dst, seed_u, seed_v, rec,
                                                      gacc, adj_u0, adj_v0, mu, step0 != 0);
}

// Tangent-linear step of step n: pulls the perturbation (or, for n = 0,
// the equilibrium of (du0, dv0)), linearised collision at the recorded
// (u, j_v) of step n, streaming stores as the forward.
template <typename T, bool PERIODIC, bool MASKED, bool FIRST, int VAR>
__global__ __launch_bounds__(kBlock) void tlm_step_kernel(
    Geometry g, ModelCoef<T> m, const T* __restrict__ src, T* __restrict__ dst,
    const T* __restrict__ du0, const T* __restrict__ dv0, const T* __restrict__ dc,
    const T* __restrict__ rec, T* __restrict__ dlag) {
  NodeIdx n;
  if (!node_of_block(g, n)) return;
  const size_t idx = n.r0 + n.x;
  unsigned lm = 0;
  if (MASKED) {
    const unsigned flag = wave_flag(g, n);
    if (flag == 2u) return;  // wavefront inside a solid region
    lm = link_of(g, flag, idx);
    if (lm & 1u) return;  // solid node of a mixed wavefront: stores nothing
  }
  T fu[9], fv[9];
  if (FIRST) {
    const T a = du0 ? du0[idx] : T(0), b = dv0 ? dv0[idx] : T(0);
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
  const T c = dc ? dc[idx] : T(0);
  if (VAR == kVarThree) {
    // the third species' perturbation starts at zero (no dw0)
    T fw[9];
    gather_w<T, PERIODIC, FIRST>(g, n, m, src, nullptr, fw);
    tlm_collide_store<T, MASKED, VAR>(g, n, m, fu, fv, c, rec, dst, lm, dlag, FIRST, fw);
  } else {
    tlm_collide_store<T, MASKED, VAR>(g, n, m, fu, fv, c, rec, dst, lm, dlag, FIRST);
  }
}

// Continuous-adjoint step: pulls the adjoint populations (or, for the first
// reversed step, p = seed_u at equilibrium and q = 0), then
// cadj_collide_store with the record of the forward step at this time.
template <typename T, bool PERIODIC, bool MASKED, bool FIRST>
__global__ __launch_bounds__(kBlock) void cadj_step_kernel(
    Geometry g, ModelCoef<T> m, CadjCoef<T> cc, const T* __restrict__ src, T* __restrict__ dst,
    const T* __restrict__ seed_u, const T* __restrict__ rec, double* __restrict__ gacc) {
  NodeIdx n;
  if (!node_of_block(g, n)) return;
  const size_t idx = n.r0 + n.x;
  unsigned lm = 0;
  if (MASKED) {
    if (FIRST) {
      // the first step owns g on every node, solid ones included
      lm = g.link[idx];
      if (lm & 1u) {
        gacc[idx] = 0.0;
        return;
      }
    } else {
      const unsigned flag = wave_flag(g, n);
      if (flag == 2u) return;  // wavefront inside a solid region
      lm = link_of(g, flag, idx);
    }
  }
  T fp[9], fq[9];
  if (FIRST) {
    const T a = seed_u[idx];
    fp[0] = m.u.w_rest * a;
#pragma unroll
    for (int i = 1; i < 5; ++i) fp[i] = m.u.w_axis * a;
#pragma unroll
    for (int i = 5; i < 9; ++i) fp[i] = m.u.w_diag * a;
#pragma unroll
    for (int i = 0; i < 9; ++i) fq[i] = T(0);
  } else {
    const T* sq = src + 9 * g.plane;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const size_t o = pull_src<PERIODIC>(n, i, g.plane);
      fp[i] = src[o];
      fq[i] = sq[o];
    }
  }
  cadj_collide_store<T, MASKED, FIRST>(g, n, m, cc, fp, fq, rec, dst, gacc, lm);
}

// Fluid test on the tape's link word (bit 0 = solid) or, for the calls that
// take no tape, on the caller's byte mask (non-zero = solid).  Null: all fluid.
__device__ __forceinline__ bool is_fluid(const uint16_t* link, size_t idx) {
  return link == nullptr || !(link[idx] & 1u);
}
__device__ __forceinline__ bool is_fluid(const uint8_t* mask, size_t idx) {
  return mask == nullptr || mask[idx] == 0;
}

template <typename T, typename M>
__global__ __launch_bounds__(kBlock) void cost_grad_kernel(
    Geometry g, const M* __restrict__ link, const T* __restrict__ uN, const T* __restrict__ ut,
    const T* __restrict__ ctrl, const double* __restrict__ gacc, T* __restrict__ seed,
    T* __restrict__ grad, double alpha, double* __restrict__ partials) {
  double acc[kRedSlots] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const size_t total = size_t(g.nx) * g.ny;
  for (size_t k = size_t(blockIdx.x) * kBlock + threadIdx.x; k < total;
       k += size_t(gridDim.x) * kBlock) {
    const size_t y = k / g.nx, x = k % g.nx;
    const size_t idx = y * g.pitch + x;
    const bool fl = is_fluid(link, idx);
    double d = 0.0, cc = 0.0, e = 0.0;
    if (fl) {
      d = double(uN[idx]) - double(ut[idx]);
      cc = double(ctrl[idx]);
      acc[0] += 0.5 * d * d;
      acc[1] += 0.5 * alpha * cc * cc;
      if (!isfinite(d) || !isfinite(cc)) acc[4] += 1.0;
    }
    if (seed) seed[idx] = fl ? T(d) : T(0);
    if (gacc) {
      if (fl) {
        e = gacc[idx] + alpha * cc;
        acc[2] += e * e;
        acc[3] = fmax(acc[3], fabs(e));
        if (!isfinite(e)) acc[4] += 1.0;
      }
      grad[idx] = fl ? T(e) : T(0);
    }
  }
  block_reduce_store(acc, partials + size_t(blockIdx.x) * kRedSlots);
}

__global__ __launch_bounds__(kBlock) void finish_reduce_kernel(
    const double* __restrict__ partials, int nblocks,
    double* __restrict__ result) {
  double acc[kRedSlots] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += kBlock) {
#pragma unroll
    for (int k = 0; k < kRedSlots; ++k) {
      double v = partials[size_t(b) * kRedSlots + k];
      acc[k] = (k == 3) ? fmax(acc[k], v) : acc[k] + v;
    }
  }
  block_reduce_store(acc, result);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void grad_max_kernel(
    Geometry g, const T* __restrict__ grad, double* __restrict__ partials) {
  const uint16_t* link = g.link;
  double acc[kRedSlots] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const size_t total = size_t(g.nx) * g.ny;
  for (size_t k = size_t(blockIdx.x) * kBlock + threadIdx.x; k < total;
       k += size_t(gridDim.x) * kBlock) {
    const size_t y = k / g.nx, x = k % g.nx;
    const size_t idx = y * g.pitch + x;
    if (is_fluid(link, idx)) {
      const double e = double(grad[idx]);
      acc[3] = fmax(acc[3], fabs(e));
      if (!isfinite(e)) acc[4] += 1.0;
    }
  }
  block_reduce_store(acc, partials + size_t(blockIdx.x) * kRedSlots);
}

// zeta > 0: fixed step; zeta <= 0: heuristic min(1, 1/||E||_inf) from the
// reduced maximum in result[3] (written by grad_max_kernel on the device).
template <typename T>
__global__ __launch_bounds__(kBlock) void gd_update_kernel(
    Geometry g, T* __restrict__ ctrl, const T* __restrict__ grad, double zeta,
    double lo, double hi, double* __restrict__ result) {
  const uint16_t* link = g.link;
  double z = zeta;
  if (z <= 0.0) {
    const double emax = result[3];
    z = emax > 0.0 ? fmin(1.0, 1.0 / emax) : 1.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) result[kRedSlots] = z;
  const size_t total = size_t(g.nx) * g.ny;
  for (size_t k = size_t(blockIdx.x) * kBlock + threadIdx.x; k < total;
       k += size_t(gridDim.x) * kBlock) {
    const size_t y = k / g.nx, x = k % g.nx;
    const size_t idx = y * g.pitch + x;
    if (!is_fluid(link, idx)) continue;
    double c = double(ctrl[idx]) - z * double(grad[idx]);
    c = fmin(fmax(c, lo), hi);
    ctrl[idx] = T(c);
  }
}

// Partial sums of x . y over the fluid nodes (slot 0), non-finite count
// (slot 4).
template <typename T>
__global__ __launch_bounds__(kBlock) void dot_kernel(Geometry g, const T* __restrict__ x,
                                                     const T* __restrict__ y,
                                                     double* __restrict__ partials) {
  const uint16_t* link = g.link;
  double acc[kRedSlots] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const size_t total = size_t(g.nx) * g.ny;
  for (size_t k = size_t(blockIdx.x) * kBlock + threadIdx.x; k < total;
       k += size_t(gridDim.x) * kBlock) {
    const size_t yy = k / g.nx, xx = k % g.nx;
    const size_t idx = yy * g.pitch + xx;
    if (is_fluid(link, idx)) {
      const double v = double(x[idx]) * double(y[idx]);
      acc[0] += v;
      if (!isfinite(v)) acc[4] += 1.0;
    }
  }
  block_reduce_store(acc, partials + size_t(blockIdx.x) * kRedSlots);
}

// Up to four inner products over the fluid nodes in one pass, each summed
// in the order of dot_kernel (so each equals that kernel's result bit for
// bit): products k = 0, 1, 2, 3 go to slots 0, 1, 2, 4; slot 3 (a maximum)
// flags a non-finite product.
template <typename T>
__global__ __launch_bounds__(kBlock) void dots_kernel(Geometry g, DotPairs<T> d,
                                                      double* __restrict__ partials) {
  const uint16_t* link = g.link;
  double acc[kRedSlots] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const size_t total = size_t(g.nx) * g.ny;
  for (size_t k = size_t(blockIdx.x) * kBlock + threadIdx.x; k < total;
       k += size_t(gridDim.x) * kBlock) {
    const size_t yy = k / g.nx, xx = k % g.nx;
    const size_t idx = yy * g.pitch + xx;
    if (is_fluid(link, idx)) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j < d.n) {
          const double v = double(d.a[j][idx]) * double(d.b[j][idx]);
          acc[j < 3 ? j : 4] += v;
          if (!isfinite(v)) acc[3] = 1.0;
        }
      }
    }
  }
  block_reduce_store(acc, partials + size_t(blockIdx.x) * kRedSlots);
}

// y <- a x + b y on the fluid nodes, 0 on the solid ones.
template <typename T>
__global__ __launch_bounds__(kBlock) void axpby_kernel(Geometry g, const T* __restrict__ x,
                                                       T* __restrict__ y, double a,
                                                       double b) {
  const uint16_t* link = g.link;
  const size_t total = size_t(g.nx) * g.ny;
  for (size_t k = size_t(blockIdx.x) * kBlock + threadIdx.x; k < total;
       k += size_t(gridDim.x) * kBlock) {
    const size_t yy = k / g.nx, xx = k % g.nx;
    const size_t idx = yy * g.pitch + xx;
    y[idx] = is_fluid(link, idx) ? T(a * double(x[idx]) + b * double(y[idx])) : T(0);
  }
}

template <typename M>
__global__ __launch_bounds__(kBlock) void count_fluid_kernel(
    Geometry g, const M* __restrict__ link, double* __restrict__ partials) {
  double acc[kRedSlots] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const size_t total = size_t(g.nx) * g.ny;
  for (size_t k = size_t(blockIdx.x) * kBlock + threadIdx.x; k < total;
       k += size_t(gridDim.x) * kBlock) {
    const size_t y = k / g.nx, x = k % g.nx;
    if (is_fluid(link, y * g.pitch + x)) acc[0] += 1.0;
  }
  block_reduce_store(acc, partials + size_t(blockIdx.x) * kRedSlots);
}

int stencil_blocks(const Geometry& g) {
  return ((g.nx + kBlock - 1) / kBlock) * g.ny;
}

}  // namespace

// ----------------------------------------------------------- launchers

void launch_build_link(const Geometry& g, int periodic, const uint8_t* mask,
                       uint16_t* link_out, uint32_t* wflag_out, hipStream_t s) {
  dim3 grid((g.nx + kBlock - 1) / kBlock, g.ny);
  hipLaunchKernelGGL(build_link_kernel, grid, dim3(kBlock), 0, s, g, periodic,
                     mask, link_out, wflag_out);
}

template <typename T>
void launch_forward_step(const Geometry& g, const ModelCoef<T>& m,
                         const FwdLaunch<T>& a, hipStream_t s) {
  const bool first = a.src == nullptr;
  const int nb = stencil_blocks(g);
#define MRT_FWD2(P, M, F, VR)                                                \
  hipLaunchKernelGGL((forward_step_kernel<T, P, M, F, VR>), dim3(nb),        \
                     dim3(kBlock), 0, s, g, m, a.src, a.dst, a.u0, a.v0,     \
                     a.ctrl, a.rec, a.lag, a.w0)
#define MRT_FWD(P, M, F)                                                     \
  if (a.variant == kVarExplicit) { MRT_FWD2(P, M, F, kVarExplicit); }       \
  else if (a.variant == kVarImplicit) { MRT_FWD2(P, M, F, kVarImplicit); }  \
  else if (a.variant == kVarThree) { MRT_FWD2(P, M, F, kVarThree); }        \
  else { MRT_FWD2(P, M, F, kVarFirst); }
#define MRT_FWD_F(P, M) \
  if (first) { MRT_FWD(P, M, true); } else { MRT_FWD(P, M, false); }
  if (g.periodic) {
    if (g.masked) { MRT_FWD_F(true, true); } else { MRT_FWD_F(true, false); }
  } else {
    if (g.masked) { MRT_FWD_F(false, true); } else { MRT_FWD_F(false, false); }
  }
#undef MRT_FWD_F
#undef MRT_FWD
#undef MRT_FWD2
}

template <typename T>
void launch_finalize(const Geometry& g, const T* src, T* state, T* uN, T* vN,
                     hipStream_t s, const ModelCoef<T>* m, const T* ctrl, bool three) {
  const int nb = stencil_blocks(g);
  const bool impl = m != nullptr;
  const ModelCoef<T> mc = impl ? *m : ModelCoef<T>{};
#define MRT_FIN2(P, M, I, W)                                                 \
  hipLaunchKernelGGL((finalize_kernel<T, P, M, I, W>), dim3(nb),             \
                     dim3(kBlock), 0, s, g, mc, src, ctrl, state, uN, vN)
#define MRT_FIN(P, M)                                                        \
  if (impl) { MRT_FIN2(P, M, true, false); }                                 \
  else if (three) { MRT_FIN2(P, M, false, true); }                           \
  else { MRT_FIN2(P, M, false, false); }
  if (g.periodic) {
    if (g.masked) { MRT_FIN(true, true); } else { MRT_FIN(true, false); }
  } else {
    if (g.masked) { MRT_FIN(false, true); } else { MRT_FIN(false, false); }
  }
#undef MRT_FIN
#undef MRT_FIN2
}

template <typename T>
void launch_implicit_terminal(const Geometry& g, const ModelCoef<T>& m, const T* src,
                              const T* ctrl, const T* seed_u, const T* seed_v, T* out_u,
                              T* out_v, double* gacc, hipStream_t s) {
  const int nb = stencil_blocks(g);
#define MRT_TRM(P, M)                                                        \
  hipLaunchKernelGGL((implicit_terminal_kernel<T, P, M>), dim3(nb),          \
                     dim3(kBlock), 0, s, g, m, src, ctrl, seed_u, seed_v,    \
                     out_u, out_v, gacc)
  if (g.periodic) {
    if (g.masked) { MRT_TRM(true, true); } else { MRT_TRM(true, false); }
  } else {
    if (g.masked) { MRT_TRM(false, true); } else { MRT_TRM(false, false); }
  }
#undef MRT_TRM
}

template <typename T>
void launch_implicit_tlm_final(const Geometry& g, const ModelCoef<T>& m, const T* fsrc,
                               const T* dsrc, const T* ctrl, const T* dc, T* duN, T* dvN,
                               hipStream_t s) {
  const int nb = stencil_blocks(g);
#define MRT_ITF(P, M)                                                        \
  hipLaunchKernelGGL((implicit_tlm_final_kernel<T, P, M>), dim3(nb),         \
                     dim3(kBlock), 0, s, g, m, fsrc, dsrc, ctrl, dc, duN,    \
                     dvN)
  if (g.periodic) {
    if (g.masked) { MRT_ITF(true, true); } else { MRT_ITF(true, false); }
  } else {
    if (g.masked) { MRT_ITF(false, true); } else { MRT_ITF(false, false); }
  }
#undef MRT_ITF
}

template <typename T>
void launch_adjoint_step(const Geometry& g, const ModelCoef<T>& m,
                         const AdjLaunch<T>& a, hipStream_t s) {
  const int nb = stencil_blocks(g);
#define MRT_ADJ2(P, M, F, L, VR)                                             \
  hipLaunchKernelGGL((adjoint_step_kernel<T, P, M, F, L, VR>), dim3(nb),     \
                     dim3(kBlock), 0, s, g, m, a.src, a.dst, a.seed_u,       \
                     a.seed_v, a.rec, a.g, a.adj_u0, a.adj_v0, a.mu,         \
                     a.step0)
#define MRT_ADJ(P, M, F, L)                                                  \
  if (a.variant == kVarExplicit) { MRT_ADJ2(P, M, F, L, kVarExplicit); }    \
  else if (a.variant == kVarImplicit) { MRT_ADJ2(P, M, F, L, kVarImplicit); } \
  else if (a.variant == kVarThree) { MRT_ADJ2(P, M, F, L, kVarThree); }      \
  else { MRT_ADJ2(P, M, F, L, kVarFirst); }
#define MRT_ADJ_L(P, M, F) \
  if (a.last) { MRT_ADJ(P, M, F, true); } else { MRT_ADJ(P, M, F, false); }
#define MRT_ADJ_F(P, M) \
  if (a.first) { MRT_ADJ_L(P, M, true); } else { MRT_ADJ_L(P, M, false); }
  if (g.periodic) {
    if (g.masked) { MRT_ADJ_F(true, true); } else { MRT_ADJ_F(true, false); }
  } else {
    if (g.masked) { MRT_ADJ_F(false, true); } else { MRT_ADJ_F(false, false); }
  }
#undef MRT_ADJ_F
#undef MRT_ADJ_L
#undef MRT_ADJ
#undef MRT_ADJ2
}

template <typename T>
void launch_cost_grad(const Geometry& g, const T* uN, const T* ut,
                      const T* ctrl, const double* gacc, T* seed, T* grad,
                      double alpha, double* partials, double* result,
                      hipStream_t s) {
  hipLaunchKernelGGL((cost_grad_kernel<T, uint16_t>), dim3(kRedBlocks), dim3(kBlock), 0,
                     s, g, g.link, uN, ut, ctrl, gacc, seed, grad, alpha,
                     partials);
  hipLaunchKernelGGL(finish_reduce_kernel, dim3(1), dim3(kBlock), 0, s,
                     partials, kRedBlocks, result);
}

// ---- cost and gradient reduction without a tape or any allocation
//
// The block partials and the two reduced rows live in this file-scope array,
// one copy per device for the life of the process.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in symbol):
// the device address is looked up once per device with hipGetSymbolAddress
// and that pointer is what the kernels receive.  Every block overwrites its
// partial row and the finishing kernel its result row, so nothing needs
// clearing between calls; two calls that overlap on one device share the
// array and race.
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

template <typename T>
hipError_t launch_cost_grad_noalloc(const Geometry& g, const uint8_t* mask, const T* uN,
                                    const T* ut, const T* ctrl, const double* gacc, T* seed,
                                    T* grad, double alpha, double* host_out, hipStream_t s) {
  double* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return e;
  double* partials = base;
  double* result = base + size_t(kRedBlocks) * kRedSlots;  // [2][kRedSlots]
  hipLaunchKernelGGL((cost_grad_kernel<T, uint8_t>), dim3(kRedBlocks), dim3(kBlock), 0,
                     s, g, mask, uN, ut, ctrl, gacc, seed, grad, alpha, partials);
  hipLaunchKernelGGL(finish_reduce_kernel, dim3(1), dim3(kBlock), 0, s,
                     partials, kRedBlocks, result);
  hipLaunchKernelGGL((count_fluid_kernel<uint8_t>), dim3(kRedBlocks), dim3(kBlock), 0, s,
                     g, mask, partials);
  hipLaunchKernelGGL(finish_reduce_kernel, dim3(1), dim3(kBlock), 0, s,
                     partials, kRedBlocks, result + kRedSlots);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(host_out, result, sizeof(double) * 2 * kRedSlots,
                     hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

template <typename T>
void launch_gd_step(const Geometry& g, T* ctrl, const T* grad, double zeta,
                    double lo, double hi, double* partials, double* result,
                    hipStream_t s) {
  if (zeta <= 0.0) {
    hipLaunchKernelGGL((grad_max_kernel<T>), dim3(kRedBlocks), dim3(kBlock), 0,
                       s, g, grad, partials);
    hipLaunchKernelGGL(finish_reduce_kernel, dim3(1), dim3(kBlock), 0, s,
                       partials, kRedBlocks, result);
  }
  hipLaunchKernelGGL((gd_update_kernel<T>), dim3(kRedBlocks), dim3(kBlock), 0,
                     s, g, ctrl, grad, zeta, lo, hi, result);
}

template <typename T>
void launch_tlm_step(const Geometry& g, const ModelCoef<T>& m, const TlmLaunch<T>& a,
                     hipStream_t s) {
  const bool first = a.src == nullptr;
  const int nb = stencil_blocks(g);
#define MRT_TLM2(P, M, F, VR)                                                \
  hipLaunchKernelGGL((tlm_step_kernel<T, P, M, F, VR>), dim3(nb),            \
                     dim3(kBlock), 0, s, g, m, a.src, a.dst, a.du0, a.dv0,   \
                     a.dc, a.rec, a.dlag)
#define MRT_TLM(P, M, F)                                                     \
  if (a.variant == kVarExplicit) { MRT_TLM2(P, M, F, kVarExplicit); }       \
  else if (a.variant == kVarImplicit) { MRT_TLM2(P, M, F, kVarImplicit); }  \
  else if (a.variant == kVarThree) { MRT_TLM2(P, M, F, kVarThree); }        \
  else { MRT_TLM2(P, M, F, kVarFirst); }
#define MRT_TLM_F(P, M) \
  if (first) { MRT_TLM(P, M, true); } else { MRT_TLM(P, M, false); }
  if (g.periodic) {
    if (g.masked) { MRT_TLM_F(true, true); } else { MRT_TLM_F(true, false); }
  } else {
    if (g.masked) { MRT_TLM_F(false, true); } else { MRT_TLM_F(false, false); }
  }
#undef MRT_TLM_F
#undef MRT_TLM
#undef MRT_TLM2
}

template <typename T>
void launch_cadj_step(const Geometry& g, const ModelCoef<T>& m, const CadjCoef<T>& cc,
                      const CadjLaunch<T>& a, hipStream_t s) {
  const int nb = stencil_blocks(g);
#define MRT_CADJ(P, M, F)                                                       \
  hipLaunchKernelGGL((cadj_step_kernel<T, P, M, F>), dim3(nb), dim3(kBlock), 0,  \
                     s, g, m, cc, a.src, a.dst, a.seed_u, a.rec, a.g)
#define MRT_CADJ_F(P, M) \
  if (a.first) { MRT_CADJ(P, M, true); } else { MRT_CADJ(P, M, false); }
  if (g.periodic) {
    if (g.masked) { MRT_CADJ_F(true, true); } else { MRT_CADJ_F(true, false); }
  } else {
    if (g.masked) { MRT_CADJ_F(false, true); } else { MRT_CADJ_F(false, false); }
  }
#undef MRT_CADJ_F
#undef MRT_CADJ
}

template <typename T>
void launch_dot(const Geometry& g, const T* x, const T* y, double* partials, double* result,
                hipStream_t s) {
  hipLaunchKernelGGL((dot_kernel<T>), dim3(kRedBlocks), dim3(kBlock), 0, s, g, x, y,
                     partials);
  hipLaunchKernelGGL(finish_reduce_kernel, dim3(1), dim3(kBlock), 0, s, partials, kRedBlocks,
                     result);
}

template <typename T>
void launch_dots(const Geometry& g, const DotPairs<T>& d, double* partials, double* result,
                 hipStream_t s) {
  hipLaunchKernelGGL((dots_kernel<T>), dim3(kRedBlocks), dim3(kBlock), 0, s, g, d, partials);
  hipLaunchKernelGGL(finish_reduce_kernel, dim3(1), dim3(kBlock), 0, s, partials, kRedBlocks,
                     result);
}

template <typename T>
void launch_axpby(const Geometry& g, const T* x, T* y, double a, double b, hipStream_t s) {
  hipLaunchKernelGGL((axpby_kernel<T>), dim3(kRedBlocks), dim3(kBlock), 0, s, g, x, y, a, b);
}

void launch_count_fluid(const Geometry& g, double* partials, double* result,
                        hipStream_t s) {
  hipLaunchKernelGGL((count_fluid_kernel<uint16_t>), dim3(kRedBlocks), dim3(kBlock), 0, s,
                     g, g.link, partials);
  hipLaunchKernelGGL(finish_reduce_kernel, dim3(1), dim3(kBlock), 0, s,
                     partials, kRedBlocks, result);
}

#define MRT_INSTANTIATE(T)                                                   \
  template void launch_dots<T>(const Geometry&, const DotPairs<T>&, double*, double*,  \
                               hipStream_t);                                          \
  template void launch_forward_step<T>(const Geometry&, const ModelCoef<T>&, \
                                       const FwdLaunch<T>&, hipStream_t);    \
  template void launch_finalize<T>(const Geometry&, const T*, T*, T*, T*,    \
                                   hipStream_t, const ModelCoef<T>*,         \
                                   const T*, bool);                          \
  template void launch_implicit_terminal<T>(const Geometry&,                 \
                                            const ModelCoef<T>&, const T*,   \
                                            const T*, const T*, const T*,    \
                                            T*, T*, double*, hipStream_t);   \
  template void launch_implicit_tlm_final<T>(const Geometry&,                \
                                             const ModelCoef<T>&, const T*,  \
                                             const T*, const T*, const T*,   \
                                             T*, T*, hipStream_t);           \
  template void launch_adjoint_step<T>(const Geometry&, const ModelCoef<T>&, \
                                       const AdjLaunch<T>&, hipStream_t);    \
  template void launch_cost_grad<T>(const Geometry&, const T*, const T*,    \
                                    const T*, const double*, T*, T*, double, \
                                    double*, double*, hipStream_t);          \
  template hipError_t launch_cost_grad_noalloc<T>(                           \
      const Geometry&, const uint8_t*, const T*, const T*, const T*,         \
      const double*, T*, T*, double, double*, hipStream_t);                  \
  template void launch_gd_step<T>(const Geometry&, T*, const T*, double,     \
                                  double, double, double*, double*,          \
                                  hipStream_t);                              \
  template void launch_cadj_step<T>(const Geometry&, const ModelCoef<T>&,    \
                                    const CadjCoef<T>&, const CadjLaunch<T>&, \
                                    hipStream_t);                             \
  template void launch_tlm_step<T>(const Geometry&, const ModelCoef<T>&,     \
                                   const TlmLaunch<T>&, hipStream_t);        \
  template void launch_dot<T>(const Geometry&, const T*, const T*, double*,  \
                              double*, hipStream_t);                         \
  template void launch_axpby<T>(const Geometry&, const T*, T*, double,       \
                                double, hipStream_t);
MRT_INSTANTIATE(float)
MRT_INSTANTIATE(double)
#undef MRT_INSTANTIATE

}  // namespace mrt
