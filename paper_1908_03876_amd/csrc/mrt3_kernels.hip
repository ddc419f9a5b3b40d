// gfx950 kernels of the two-species D3Q19 MRT step, its exact discrete
// adjoint (AMRT) and its tangent.
//
// Method: arXiv:1908.03876, Section 3.1 (eq:LBE with the sources (S),
// (PhiS), the collision (MC) in moment space, (phieq), the relaxation
// matrix with the flux block K, D = d Cs^2 tau (K^-1 - I/2), the D3Q19
// lattice of the Remark on DmQq lattices with (sumWi3)) and Section 3.2.1
// (LIBEG, CAE, AEDs, RFS1, CAEL, gradientLattice), with tau = 1 and
// Cs^2 = 1/3.
//
// Design (as the D2Q9 kernels): one thread per node, 256-node row tiles
// dealt to the 8 XCDs in contiguous bands; structure-of-arrays planes
// [species][19] of the haloed internal layout; pull streaming of
// post-collision states, so each population is read once and written once
// per step; every load is a plane base plus the node's one 32-bit offset
// (a neighbour outside a non-periodic lattice is still an in-bounds address,
// in the halo or at the end of an adjacent row, and its value is discarded
// by the bounce-back); halfway
// bounce-back reads the node's own opposite population where the link word
// marks a wall, so no store is ever scattered and every wavefront writes
// whole cache lines; per 64-node row segment a flag lets all-fluid
// wavefronts skip the link word.
#include "mrt3_internal.h"
#include "mrt_device.h"

namespace mrt3 {
namespace {

using mrt::dev::kBlock;
using mrt::dev::xcd_tile;

struct Node3 {
  int x, y, z;
  uint32_t pub;  // public index (z * ny + y) * pitch + x
  uint32_t in;   // internal index ((z + 1)(ny + 2) + y + 1) * pitchI + x
};

__device__ __forceinline__ void make_node(const Geometry3& g, int x, int y, int z, Node3& n) {
  n.x = x;
  n.y = y;
  n.z = z;
  n.pub = (uint32_t(z) * uint32_t(g.ny) + uint32_t(y)) * uint32_t(g.pitch) + uint32_t(x);
  n.in = (uint32_t(z + 1) * uint32_t(g.ny + 2) + uint32_t(y + 1)) * uint32_t(g.pitchI) +
         uint32_t(x);
}

// Row order of the tiles: z-fastest inside bands of g.band y-rows (the
// last band takes the remainder).  A row shares cache lines with the rows
// at y +- 1 and z +- 1 (its pulls, and the bounce-back reads of the nodes
// next to a wall, hit the lines its neighbours pull); in this order those
// rows run within a band's width of blocks on the same XCD, while the lines
// are still in its L2, where plain z-major order puts a whole (ny x nx)
// slice between z-neighbours.
__device__ __forceinline__ void band_row(const Geometry3& g, int r, int& y, int& z) {
  const int b = g.band;
  const int whole = (g.ny / b) * b;
  int y0, h, q;
  if (r < whole * g.nz) {
    y0 = (r / (b * g.nz)) * b;
    h = b;
    q = r - y0 * g.nz;
  } else {
    y0 = whole;
    h = g.ny - whole;
    q = r - whole * g.nz;
  }
  z = q / h;
  y = y0 + (q - z * h);
}

__device__ __forceinline__ bool node_of_block(const Geometry3& g, Node3& n) {
  const int nbx = (g.nx + kBlock - 1) / kBlock;
  const int ntiles = nbx * g.ny * g.nz;
  const int id = blockIdx.x;
  if (id >= ntiles) return false;
  const int t = xcd_tile(id, ntiles);
  const int x = (t % nbx) * kBlock + int(threadIdx.x);
  if (x >= g.nx) return false;
  int y, z;
  band_row(g, t / nbx, y, z);
  make_node(g, x, y, z, n);
  return true;
}

__device__ __forceinline__ unsigned wave_flag(const Geometry3& g, const Node3& n) {
  const int seg =
      __builtin_amdgcn_readfirstlane((n.z * g.ny + n.y) * g.nsx + (n.x >> 6));
  return g.wflag[seg];
}

// Internal index delta of the displacement (dx, dy, dz) (wave-uniform).
__device__ __forceinline__ int idelta(const Geometry3& g, int dx, int dy, int dz) {
  return (dz * (g.ny + 2) + dy) * g.pitchI + dx;
}

__device__ __forceinline__ int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// Internal index of node x + (dx, dy, dz) on a periodic lattice.
__device__ __forceinline__ uint32_t nb_in_wrapped(const Geometry3& g, const Node3& n, int dx,
                                                  int dy, int dz) {
  const int xx = wrap(n.x + dx, g.nx), yy = wrap(n.y + dy, g.ny), zz = wrap(n.z + dz, g.nz);
  return (uint32_t(zz + 1) * uint32_t(g.ny + 2) + uint32_t(yy + 1)) * uint32_t(g.pitchI) +
         uint32_t(xx);
}

// Public index of the in-lattice node x + (dx, dy, dz) (wrapped when
// periodic).
template <bool PERIODIC>
__device__ __forceinline__ uint32_t nb_pub(const Geometry3& g, const Node3& n, int dx, int dy,
                                           int dz) {
  int xx = n.x + dx, yy = n.y + dy, zz = n.z + dz;
  if (PERIODIC) {
    xx = wrap(xx, g.nx);
    yy = wrap(yy, g.ny);
    zz = wrap(zz, g.nz);
  }
  return (uint32_t(zz) * uint32_t(g.ny) + uint32_t(yy)) * uint32_t(g.pitch) + uint32_t(xx);
}

// Raw buffer accesses to the internal planes: a resource over one plane
// (wave-uniform, its base shifted by the neighbour displacement) plus the
// node's 32-bit byte offset, so that every access is one buffer
// instruction with no per-lane 64-bit address arithmetic.  The resources
// carry no range limit: every access is in bounds by construction (the
// halo rows and slabs cover every neighbour).  Cache policy: kNT =
// non-temporal.
constexpr int kNT = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, -1, 0x00020000);
}

template <int AUX>
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
}
template <int AUX>
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, kNT);
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  using U2 = unsigned __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, off, 0, kNT);
}

// Population node x pulls in direction i: plane i of buf at x - e_i (where
// that neighbour is solid or outside a non-periodic lattice the value read
// is replaced by the wall read).  bo = the node's internal byte offset.
template <typename T, bool PERIODIC, int AUX>
__device__ __forceinline__ T pull_ld(const Geometry3& g, const Node3& n, const T* buf, int i,
                                     uint32_t bo) {
  const Vel e = vel(i);
  const T* pl = buf + size_t(i) * g.planeI;
  if (PERIODIC)
    return bload<AUX>(rsrc_of(pl), nb_in_wrapped(g, n, -e.x, -e.y, -e.z) * uint32_t(sizeof(T)),
                      T(0));
  return bload<AUX>(rsrc_of(pl - idelta(g, e.x, e.y, e.z)), bo, T(0));
}

// Adjoint gather: plane i of buf at x + e_i (the transpose of the pull).
template <typename T, bool PERIODIC, int AUX>
__device__ __forceinline__ T gather_ld(const Geometry3& g, const Node3& n, const T* buf, int i,
                                       uint32_t bo) {
  const Vel e = vel(i);
  const T* pl = buf + size_t(i) * g.planeI;
  if (PERIODIC)
    return bload<AUX>(rsrc_of(pl), nb_in_wrapped(g, n, e.x, e.y, e.z) * uint32_t(sizeof(T)),
                      T(0));
  return bload<AUX>(rsrc_of(pl + idelta(g, e.x, e.y, e.z)), bo, T(0));
}

// acc (+)= r * v for a compile-time integer r (after unrolling): zero terms
// vanish, +-1 become additions.
template <typename T>
__device__ __forceinline__ void madd(T& acc, bool& started, int r, T v) {
  if (r == 0) return;
  const T t = r == 1 ? v : (r == -1 ? -v : T(r) * v);
  if (started) {
    acc += t;
  } else {
    acc = t;
    started = true;
  }
}

__host__ __device__ constexpr bool odd_row(int k) { return (k >= 3 && k <= 8) || k >= 16; }

// D3Q19 weights by shell (sumWi3).
__host__ __device__ constexpr double wgt(int i) {
  return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Relaxation in moment space, f <- f - M^-1 Pi (M f - m_eq(theta)),
// without the conserved density row.  Even rows see only f_0 and the sums
// of opposite pairs, odd rows only their differences; the back-transform
// splits the same way.  TRANS takes K^T: with theta = 0 this is the
// adjoint collision f <- f - C^T f (C^T = M^-1 Pi^T M because the three
// flux rows share one norm).  a1o, a2o: the scaled non-equilibrium parts
// of the energy rows, for the adjoint equilibrium term.
template <typename T, bool TRANS>
__device__ __forceinline__ void relax(T f[Q], T theta, const Species3Coef<T>& c, T& a1o,
                                      T& a2o) {
  T s[9], d[9];
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    s[p] = f[2 * p + 1] + f[2 * p + 2];
    d[p] = f[2 * p + 1] - f[2 * p + 2];
  }
  T m[Q];
#pragma unroll
  for (int k = 1; k < Q; ++k) {
    T acc = T(0);
    bool st = false;
    if (!odd_row(k)) madd(acc, st, mrow(k, 0), f[0]);
#pragma unroll
    for (int p = 0; p < 9; ++p) madd(acc, st, mrow(k, 2 * p + 1), odd_row(k) ? d[p] : s[p]);
    m[k] = acc;
  }
  T a[Q];
  a[1] = c.c[1] * (m[1] - c.e_eq * theta);
  a[2] = c.c[2] * (m[2] - c.eps_eq * theta);
#pragma unroll
  for (int k = 4; k < Q; ++k)
    if (k != 5 && k != 7) a[k] = c.c[k] * m[k];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const T k0 = TRANS ? c.k[r] : c.k[3 * r];
    const T k1 = TRANS ? c.k[3 + r] : c.k[3 * r + 1];
    const T k2 = TRANS ? c.k[6 + r] : c.k[3 * r + 2];
    a[3 + 2 * r] = k0 * m[3] + k1 * m[5] + k2 * m[7];
  }
  {
    T acc = T(0);
    bool st = false;
#pragma unroll
    for (int k = 1; k < Q; ++k)
      if (!odd_row(k)) madd(acc, st, mrow(k, 0), a[k]);
    f[0] -= acc;
  }
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    T ev = T(0), od = T(0);
    bool se = false, so = false;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      if (odd_row(k))
        madd(od, so, mrow(k, 2 * p + 1), a[k]);
      else
        madd(ev, se, mrow(k, 2 * p + 1), a[k]);
    }
    f[2 * p + 1] -= ev + od;
    f[2 * p + 2] -= ev - od;
  }
  a1o = a[1];
  a2o = a[2];
}

// e_p . (ax, ay, az) for the pair representative 2p+1.
template <typename T>
__device__ __forceinline__ T edot(int i, T ax, T ay, T az) {
  const Vel e = vel(i);
  T acc = T(0);
  bool st = false;
  madd(acc, st, e.x, ax);
  madd(acc, st, e.y, ay);
  madd(acc, st, e.z, az);
  return acc;
}

// First moment sum_i e_i f_i.
template <typename T>
__device__ __forceinline__ void first_moment(const T f[Q], T& jx, T& jy, T& jz) {
  T d[9];
#pragma unroll
  for (int p = 0; p < 9; ++p) d[p] = f[2 * p + 1] - f[2 * p + 2];
  jx = T(0), jy = T(0), jz = T(0);
  bool sx = false, sy = false, sz = false;
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    const Vel e = vel(2 * p + 1);
    madd(jx, sx, e.x, d[p]);
    madd(jy, sy, e.y, d[p]);
    madd(jz, sz, e.z, d[p]);
  }
}

template <typename T>
__device__ __forceinline__ T wsum(const T f[Q]) {
  T ax = T(0), dg = T(0);
#pragma unroll
  for (int i = 1; i <= 6; ++i) ax += f[i];
#pragma unroll
  for (int i = 7; i < Q; ++i) dg += f[i];
  return T(1.0 / 3.0) * f[0] + T(1.0 / 18.0) * ax + T(1.0 / 36.0) * dg;
}

// tau S_i + tau w_i Phi (S, PhiS), tau = 1, 1/Cs^2 = 3: on u the
// chemotactic flux a and the kinetics phu; on v the kinetics phv.
template <typename T>
__device__ __forceinline__ void add_sources_u(T fu[Q], T phu, T ax, T ay, T az) {
  fu[0] += phu * T(1.0 / 3.0);
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    const int i = 2 * p + 1;
    const T ea = T(3.0 * wgt(i)) * edot(i, ax, ay, az);
    const T k = phu * T(wgt(i));
    fu[i] += k + ea;
    fu[i + 1] += k - ea;
  }
}
template <typename T>
__device__ __forceinline__ void add_sources_v(T fv[Q], T phv) {
  fv[0] += phv * T(1.0 / 3.0);
#pragma unroll
  for (int i = 1; i < Q; ++i) fv[i] += phv * T(wgt(i));
}

// Halfway bounce-back by own-node reads.  When the neighbour a population
// streams from is solid (or outside a non-periodic lattice), the value is
// the node's own opposite post-collision population of the previous step,
// which the node stored in its own slot of the opposite plane: the pull
// reads it there and no node ever writes into a solid node's slots.  In
// the forward (and tangent) the wall test of direction i is bit i of the
// link word (x - e_i solid); in the adjoint gather it is bit opp(i)
// (x + e_i solid).  The plain pull has already been issued for every lane
// (a solid neighbour's slot holds garbage, which is discarded here).
template <typename T, bool ADJ>
__device__ __forceinline__ void wall_reads(const Geometry3& g, const T* __restrict__ buf,
                                           T f[Q], unsigned lm, uint32_t bo) {
  T own[Q];
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    own[i] = f[i];
    if ((lm >> (ADJ ? opp(i) : i)) & 1u)
      own[i] = bload<0>(rsrc_of(buf + size_t(opp(i)) * g.planeI), bo, T(0));
  }
#pragma unroll
  for (int i = 1; i < Q; ++i) f[i] = own[i];
}

// w~ . f (the transpose of the initialisation phi_i = w~_i Theta_0).
template <typename T>
__device__ __forceinline__ T shell_dot(const T f[Q], const Species3Coef<T>& c) {
  T ax = T(0), dg = T(0);
#pragma unroll
  for (int i = 1; i <= 6; ++i) ax += f[i];
#pragma unroll
  for (int i = 7; i < Q; ++i) dg += f[i];
  return c.w_rest * f[0] + c.w_axis * ax + c.w_diag * dg;
}

// Pre-collision populations: the pull from src, or w~ Theta_0 at step 0.
template <typename T, bool PERIODIC, bool MASKED, bool FIRST>
__device__ __forceinline__ void gather(const Geometry3& g, const Node3& n,
                                       const Model3Coef<T>& m, const T* __restrict__ src,
                                       const T* __restrict__ u0, const T* __restrict__ v0,
                                       T fu[Q], T fv[Q], uint32_t bo, unsigned lm) {
  if (FIRST) {
    const T a = u0 ? u0[n.pub] : T(0), b = v0 ? v0[n.pub] : T(0);
    fu[0] = m.u.w_rest * a;
    fv[0] = m.v.w_rest * b;
#pragma unroll
    for (int i = 1; i <= 6; ++i) {
      fu[i] = m.u.w_axis * a;
      fv[i] = m.v.w_axis * b;
    }
#pragma unroll
    for (int i = 7; i < Q; ++i) {
      fu[i] = m.u.w_diag * a;
      fv[i] = m.v.w_diag * b;
    }
  } else if (MASKED && (lm & 1u)) {
    // a solid lane of a mixed wavefront: its results are never read, so it
    // loads nothing (lines that only solid lanes would touch are not
    // fetched)
#pragma unroll
    for (int i = 0; i < Q; ++i) fu[i] = fv[i] = T(0);
  } else {
    const T* sv = src + size_t(Q) * g.planeI;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      fu[i] = pull_ld<T, PERIODIC, 0>(g, n, src, i, bo);
      fv[i] = pull_ld<T, PERIODIC, 0>(g, n, sv, i, bo);
    }
    if (MASKED && lm != 0u) {
      wall_reads<T, false>(g, src, fu, lm, bo);
      wall_reads<T, false>(g, sv, fv, lm, bo);
    }
  }
}

// Post-collision stores of one species (planes [0, 19) of dst),
// non-temporal (next read a whole sweep later).  Every lane of a wavefront
// stores, solid nodes too (their values are never read by a fluid node), so
// the stores always fill whole cache lines.  Each species is stored as soon
// as it is final, which frees its registers before the other one relaxes.
template <typename T>
__device__ __forceinline__ void store_species(const Geometry3& g, const T f[Q],
                                              T* __restrict__ dst, uint32_t bo) {
#pragma unroll
  for (int i = 0; i < Q; ++i) bstore(rsrc_of(dst + size_t(i) * g.planeI), bo, f[i]);
}

// ------------------------------------------------------------ forward

template <typename T, bool PERIODIC, bool MASKED, bool FIRST>
__global__ __launch_bounds__(kBlock) void forward3_kernel(Geometry3 g, Model3Coef<T> m,
                                                          Fwd3Launch<T> a) {
  Node3 n;
  if (!node_of_block(g, n)) return;
  unsigned lm = 0;
  if (MASKED) {
    const unsigned flag = wave_flag(g, n);
    if (flag == 2u) return;
    lm = flag ? g.link[n.pub] : 0u;
  }
  const uint32_t bo = n.in * uint32_t(sizeof(T));
  T fu[Q], fv[Q];
  gather<T, PERIODIC, MASKED, FIRST>(g, n, m, a.src, a.u0, a.v0, fu, fv, bo, lm);
  const T c = a.ctrl[n.pub];
  T u = T(0), v = T(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    u += fu[i];
    v += fv[i];
  }
  T jx, jy, jz;
  first_moment(fv, jx, jy, jz);
  const bool solid = MASKED && (lm & 1u);
  // every lane stores the record (zeros at the solid lanes of a mixed
  // wavefront, read by nobody), so that the stores fill whole chunks: a
  // store that leaves part of a 64-byte chunk unwritten costs a
  // read-modify-write in memory
  if (a.rec != nullptr) {
    __builtin_nontemporal_store(u, &a.rec[n.pub]);
    __builtin_nontemporal_store(jx, &a.rec[size_t(g.plane) + n.pub]);
    __builtin_nontemporal_store(jy, &a.rec[2 * size_t(g.plane) + n.pub]);
    __builtin_nontemporal_store(jz, &a.rec[3 * size_t(g.plane) + n.pub]);
  }
  // A_u1 grad v = u B j_v with grad v = -K_v j_v / (tau d_v Cs^2)
  const T ax = u * (m.b[0] * jx + m.b[1] * jy + m.b[2] * jz);
  const T ay = u * (m.b[3] * jx + m.b[4] * jy + m.b[5] * jz);
  const T az = u * (m.b[6] * jx + m.b[7] * jy + m.b[8] * jz);
  const T phu = m.r_u * u * (T(1) - u);
  const T phv = m.a_uv * u - m.b_v * v + c;
  // solid nodes of mixed wavefronts compute on values nobody reads; they
  // store them anyway, keeping the wavefront's stores whole
  T t1, t2;
  relax<T, false>(fv, v, m.v, t1, t2);
  add_sources_v(fv, phv);
  store_species<T>(g, fv, a.dst + size_t(Q) * g.planeI, bo);
  relax<T, false>(fu, u, m.u, t1, t2);
  add_sources_u(fu, phu, ax, ay, az);
  store_species<T>(g, fu, a.dst, bo);
}

template <typename T, bool PERIODIC, bool MASKED>
__global__ __launch_bounds__(kBlock) void finalize3_kernel(Geometry3 g, const T* __restrict__ src,
                                                           T* __restrict__ state,
                                                           T* __restrict__ uN,
                                                           T* __restrict__ vN) {
  Node3 n;
  if (!node_of_block(g, n)) return;
  const bool solid = MASKED && (g.link[n.pub] & 1u);
  const uint32_t bo = n.in * uint32_t(sizeof(T));
  T fu[Q], fv[Q];
  if (solid) {
#pragma unroll
    for (int i = 0; i < Q; ++i) fu[i] = fv[i] = T(0);
  } else {
    const T* sv = src + size_t(Q) * g.planeI;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      fu[i] = pull_ld<T, PERIODIC, 0>(g, n, src, i, bo);
      fv[i] = pull_ld<T, PERIODIC, 0>(g, n, sv, i, bo);
    }
    if (MASKED) {
      const unsigned lm = g.link[n.pub];
      if (lm != 0u) {
        wall_reads<T, false>(g, src, fu, lm, bo);
        wall_reads<T, false>(g, sv, fv, lm, bo);
      }
    }
  }
  T u = T(0), v = T(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    u += fu[i];
    v += fv[i];
  }
  if (uN) uN[n.pub] = u;
  if (vN) vN[n.pub] = v;
  if (state) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      state[size_t(i) * g.plane + n.pub] = fu[i];
      state[size_t(Q + i) * g.plane + n.pub] = fv[i];
    }
  }
}

// ------------------------------------------------------------ adjoint

// One reversed step at a node (CAEL): nu = transposed streaming of lambda,
// g += tau sum_i w_i nu_v,i, then lambda = J_n^T nu with the recorded u,
// j_v of step n:
//   lambda_u = nu_u - C_u^T nu_u + 1 [w~_u . C_u^T nu_u + sigma_u r_u (1-2u)
//              + p . (B j_v) + sigma_v a_uv]
//   lambda_v = nu_v - C_v^T nu_v + 1 [w~_v . C_v^T nu_v - sigma_v b_v]
//              + E (u B^T p)
// with sigma = w . nu and p = (tau/Cs^2) sum_i w_i nu_u,i e_i.
template <typename T, bool PERIODIC, bool MASKED, bool FIRST, bool LAST>
__global__ __launch_bounds__(kBlock) void adjoint3_kernel(Geometry3 g, Model3Coef<T> m,
                                                          Adj3Launch<T> a) {
  Node3 n;
  if (!node_of_block(g, n)) return;
  const uint32_t idx = n.pub;
  unsigned lm = 0;
  if (MASKED) {
    if (FIRST || LAST) {
      // single steps: solid nodes own outputs
      lm = g.link[idx];
      if (lm & 1u) {
        if (FIRST) a.g[idx] = 0.0;
        if (LAST) {
          if (a.adj_u0) a.adj_u0[idx] = T(0);
          if (a.adj_v0) a.adj_v0[idx] = T(0);
        }
        return;
      }
    } else {
      const unsigned flag = wave_flag(g, n);
      if (flag == 2u) return;
      lm = flag ? g.link[idx] : 0u;
    }
  }
  const uint32_t bo = n.in * uint32_t(sizeof(T));
  T nu[Q], nv[Q];
  if (FIRST) {
    // lambda_i^N = seed for every i; the seeds carry no wall slots (a wall
    // includes the outside of a non-periodic lattice)
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const Vel e = vel(i);
      const bool wall = MASKED && ((lm >> opp(i)) & 1u);
      const uint32_t s = wall ? idx : nb_pub<PERIODIC>(g, n, e.x, e.y, e.z);
      nu[i] = a.seed_u[s];
      nv[i] = a.seed_v ? a.seed_v[s] : T(0);
    }
  } else if (MASKED && (lm & 1u)) {
    // solid lane of a mixed wavefront: nothing to gather (see gather())
#pragma unroll
    for (int i = 0; i < Q; ++i) nu[i] = nv[i] = T(0);
  } else {
    const T* sv = a.src + size_t(Q) * g.planeI;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      nu[i] = gather_ld<T, PERIODIC, 0>(g, n, a.src, i, bo);
      nv[i] = gather_ld<T, PERIODIC, 0>(g, n, sv, i, bo);
    }
    if (MASKED && lm != 0u) {
      wall_reads<T, true>(g, a.src, nu, lm, bo);
      wall_reads<T, true>(g, sv, nv, lm, bo);
    }
  }
  const bool solid = MASKED && (lm & 1u);
  const T su = wsum(nu), sv = wsum(nv);
  T px, py, pz;
  first_moment(nu, px, py, pz);
  // p = 3 sum_i w_i nu_i e_i: only the axis and diagonal shells carry e_i
  {
    T dxa = nu[1] - nu[2], dya = nu[3] - nu[4], dza = nu[5] - nu[6];
    px = T(1.0 / 6.0) * dxa + T(1.0 / 12.0) * (px - dxa);
    py = T(1.0 / 6.0) * dya + T(1.0 / 12.0) * (py - dya);
    pz = T(1.0 / 6.0) * dza + T(1.0 / 12.0) * (pz - dza);
  }
  // a solid lane of a mixed wavefront adds the 0 of its zero-filled
  // gather, so the gradient stays 0 there and the stores fill whole chunks
  if (FIRST)
    a.g[idx] = solid ? 0.0 : double(sv);
  else
    a.g[idx] += double(sv);
  const T u = __builtin_nontemporal_load(&a.rec[idx]);
  const T jx = __builtin_nontemporal_load(&a.rec[size_t(g.plane) + idx]);
  const T jy = __builtin_nontemporal_load(&a.rec[2 * size_t(g.plane) + idx]);
  const T jz = __builtin_nontemporal_load(&a.rec[3 * size_t(g.plane) + idx]);
  const T bjx = m.b[0] * jx + m.b[1] * jy + m.b[2] * jz;
  const T bjy = m.b[3] * jx + m.b[4] * jy + m.b[5] * jz;
  const T bjz = m.b[6] * jx + m.b[7] * jy + m.b[8] * jz;
  const T cu = su * m.r_u * (T(1) - T(2) * u) + px * bjx + py * bjy + pz * bjz + sv * m.a_uv;
  const T cv = -sv * m.b_v;
  const T qx = u * (m.b[0] * px + m.b[3] * py + m.b[6] * pz);
  const T qy = u * (m.b[1] * px + m.b[4] * py + m.b[7] * pz);
  const T qz = u * (m.b[2] * px + m.b[5] * py + m.b[8] * pz);
  // each species is finished and stored in turn (u first: its adjoint
  // feeds p and q, computed above, and nothing else), which frees its
  // registers before v relaxes; solid nodes of mixed wavefronts store values
  // nobody reads (whole cache lines)
  T a1, a2;
  relax<T, true>(nu, T(0), m.u, a1, a2);
  const T wu = m.u.e_eq * a1 + m.u.eps_eq * a2 + cu;
#pragma unroll
  for (int i = 0; i < Q; ++i) nu[i] += wu;
  if (LAST) {
    // transpose of phi_i^0 = w~_i Theta_0
    if (a.adj_u0) a.adj_u0[idx] = shell_dot(nu, m.u);
  } else if (a.dst) {
    store_species<T>(g, nu, a.dst, bo);
  }
  relax<T, true>(nv, T(0), m.v, a1, a2);
  const T wv = m.v.e_eq * a1 + m.v.eps_eq * a2 + cv;
  nv[0] += wv;
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    const int i = 2 * p + 1;
    const T eq = edot(i, qx, qy, qz);
    nv[i] += wv + eq;
    nv[i + 1] += wv - eq;
  }
  if (LAST) {
    if (a.adj_v0) a.adj_v0[idx] = shell_dot(nv, m.v);
  } else if (a.dst) {
    store_species<T>(g, nv, a.dst + size_t(Q) * g.planeI, bo);
  }
}

// ------------------------------------------------------------ tangent

// Tangent of forward step n (sensitivity LBE, LIBEG-V) at a node, with the
// recorded u, j_v of that step: the relaxation is linear; the sources give
// d(u B j_v) = du B j_v + u B dj_v, dPhi_u = r_u (1-2u) du,
// dPhi_v = a_uv du - b_v dv + dc.
template <typename T, bool PERIODIC, bool MASKED, bool FIRST>
__global__ __launch_bounds__(kBlock) void tlm3_kernel(Geometry3 g, Model3Coef<T> m,
                                                      Tlm3Launch<T> a) {
  Node3 n;
  if (!node_of_block(g, n)) return;
  unsigned lm = 0;
  if (MASKED) {
    const unsigned flag = wave_flag(g, n);
    if (flag == 2u) return;
    lm = flag ? g.link[n.pub] : 0u;
  }
  const uint32_t bo = n.in * uint32_t(sizeof(T));
  T fu[Q], fv[Q];
  gather<T, PERIODIC, MASKED, FIRST>(g, n, m, a.src, a.du0, a.dv0, fu, fv, bo, lm);
  const T dc = a.dc ? a.dc[n.pub] : T(0);
  // solid nodes of mixed wavefronts compute on values nobody reads (their
  // record entries are stale) and store them, keeping the stores whole
  const T u = __builtin_nontemporal_load(&a.rec[n.pub]);
  const T jx = __builtin_nontemporal_load(&a.rec[size_t(g.plane) + n.pub]);
  const T jy = __builtin_nontemporal_load(&a.rec[2 * size_t(g.plane) + n.pub]);
  const T jz = __builtin_nontemporal_load(&a.rec[3 * size_t(g.plane) + n.pub]);
  T du = T(0), dv = T(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    du += fu[i];
    dv += fv[i];
  }
  T djx, djy, djz;
  first_moment(fv, djx, djy, djz);
  const T ax = du * (m.b[0] * jx + m.b[1] * jy + m.b[2] * jz) +
               u * (m.b[0] * djx + m.b[1] * djy + m.b[2] * djz);
  const T ay = du * (m.b[3] * jx + m.b[4] * jy + m.b[5] * jz) +
               u * (m.b[3] * djx + m.b[4] * djy + m.b[5] * djz);
  const T az = du * (m.b[6] * jx + m.b[7] * jy + m.b[8] * jz) +
               u * (m.b[6] * djx + m.b[7] * djy + m.b[8] * djz);
  const T phu = m.r_u * (T(1) - T(2) * u) * du;
  const T phv = m.a_uv * du - m.b_v * dv + dc;
  T t1, t2;
  relax<T, false>(fv, dv, m.v, t1, t2);
  add_sources_v(fv, phv);
  store_species<T>(g, fv, a.dst + size_t(Q) * g.planeI, bo);
  relax<T, false>(fu, du, m.u, t1, t2);
  add_sources_u(fu, phu, ax, ay, az);
  store_species<T>(g, fu, a.dst, bo);
}

// ------------------------------------------------------------ link words

// One thread per node: the link word (bit 0 = solid, bit i = x - e_i solid
// or, on a non-periodic lattice, outside), the 16-bit solid flag the
// reductions read, and per 64-node row segment the wavefront flag.  mask
// may be null (no solid node).
template <bool PERIODIC>
__global__ __launch_bounds__(kBlock) void build_link3_kernel(Geometry3 g,
                                                             const uint8_t* __restrict__ mask,
                                                             uint32_t* __restrict__ link,
                                                             uint32_t* __restrict__ wflag,
                                                             uint16_t* __restrict__ solid16) {
  const int nbx = (g.nx + kBlock - 1) / kBlock;
  const int r = int(blockIdx.x) / nbx;
  const int x = (int(blockIdx.x) % nbx) * kBlock + int(threadIdx.x);
  const bool valid = r < g.ny * g.nz && x < g.nx;
  Node3 n;
  make_node(g, valid ? x : 0, valid ? r % g.ny : 0, valid ? r / g.ny : 0, n);
  unsigned lw = 0;
  bool solid = true;
  if (valid) {
    solid = mask != nullptr && mask[n.pub] != 0;
    lw = solid ? 1u : 0u;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const Vel e = vel(i);
      const int xx = n.x - e.x, yy = n.y - e.y, zz = n.z - e.z;
      const bool out = xx < 0 || xx >= g.nx || yy < 0 || yy >= g.ny || zz < 0 || zz >= g.nz;
      if (!PERIODIC && out) {
        lw |= 1u << i;
      } else if (mask != nullptr && mask[nb_pub<PERIODIC>(g, n, -e.x, -e.y, -e.z)] != 0) {
        lw |= 1u << i;
      }
    }
    link[n.pub] = lw;
    solid16[n.pub] = solid ? 1 : 0;
  }
  const uint64_t any_link = __ballot(valid && lw != 0u);
  const uint64_t any_fluid = __ballot(valid && !solid);
  const int lane = int(threadIdx.x) & 63;
  if (lane == 0 && valid) {
    const unsigned f = any_fluid == 0 ? 2u : (any_link != 0 ? 1u : 0u);
    wflag[r * g.nsx + (x >> 6)] = f;
  }
}

}  // namespace

// ------------------------------------------------------------ launchers

static dim3 grid_of(const Geometry3& g) {
  const int nbx = (g.nx + kBlock - 1) / kBlock;
  return dim3(unsigned(nbx) * unsigned(g.ny) * unsigned(g.nz));
}

void launch_build_link3(const Geometry3& g, const uint8_t* mask, uint32_t* link,
                        uint32_t* wflag, uint16_t* solid16, hipStream_t s) {
  if (g.periodic)
    hipLaunchKernelGGL(build_link3_kernel<true>, grid_of(g), dim3(kBlock), 0, s, g, mask, link,
                       wflag, solid16);
  else
    hipLaunchKernelGGL(build_link3_kernel<false>, grid_of(g), dim3(kBlock), 0, s, g, mask, link,
                       wflag, solid16);
}

// A non-periodic lattice always runs with link words (its edge is a wall).
#define MRT3_DISPATCH_PM(KERNEL, ...)                                                      \
  do {                                                                                     \
    if (g.periodic) {                                                                      \
      if (g.masked)                                                                        \
        hipLaunchKernelGGL((KERNEL<T, true, true, ##__VA_ARGS__>), grid_of(g), dim3(kBlock), \
                           0, s, g, m, a);                                                 \
      else                                                                                 \
        hipLaunchKernelGGL((KERNEL<T, true, false, ##__VA_ARGS__>), grid_of(g),            \
                           dim3(kBlock), 0, s, g, m, a);                                   \
    } else {                                                                               \
      hipLaunchKernelGGL((KERNEL<T, false, true, ##__VA_ARGS__>), grid_of(g), dim3(kBlock),  \
                         0, s, g, m, a);                                                   \
    }                                                                                      \
  } while (0)

template <typename T>
void launch_forward3(const Geometry3& g, const Model3Coef<T>& m, const Fwd3Launch<T>& a,
                     hipStream_t s) {
  if (a.src == nullptr)
    MRT3_DISPATCH_PM(forward3_kernel, true);
  else
    MRT3_DISPATCH_PM(forward3_kernel, false);
}

template <typename T>
void launch_finalize3(const Geometry3& g, const T* src, T* state, T* uN, T* vN,
                      hipStream_t s) {
  if (g.periodic) {
    if (g.masked)
      hipLaunchKernelGGL((finalize3_kernel<T, true, true>), grid_of(g), dim3(kBlock), 0, s, g,
                         src, state, uN, vN);
    else
      hipLaunchKernelGGL((finalize3_kernel<T, true, false>), grid_of(g), dim3(kBlock), 0, s, g,
                         src, state, uN, vN);
  } else {
    hipLaunchKernelGGL((finalize3_kernel<T, false, true>), grid_of(g), dim3(kBlock), 0, s, g,
                       src, state, uN, vN);
  }
}

template <typename T>
void launch_adjoint3(const Geometry3& g, const Model3Coef<T>& m, const Adj3Launch<T>& a,
                     hipStream_t s) {
  if (a.first) {
    if (a.last)
      MRT3_DISPATCH_PM(adjoint3_kernel, true, true);
    else
      MRT3_DISPATCH_PM(adjoint3_kernel, true, false);
  } else {
    if (a.last)
      MRT3_DISPATCH_PM(adjoint3_kernel, false, true);
    else
      MRT3_DISPATCH_PM(adjoint3_kernel, false, false);
  }
}

template <typename T>
void launch_tlm3(const Geometry3& g, const Model3Coef<T>& m, const Tlm3Launch<T>& a,
                 hipStream_t s) {
  if (a.src == nullptr)
    MRT3_DISPATCH_PM(tlm3_kernel, true);
  else
    MRT3_DISPATCH_PM(tlm3_kernel, false);
}

#define MRT3_INSTANTIATE(T)                                                                  \
  template void launch_forward3<T>(const Geometry3&, const Model3Coef<T>&,                   \
                                   const Fwd3Launch<T>&, hipStream_t);                       \
  template void launch_finalize3<T>(const Geometry3&, const T*, T*, T*, T*, hipStream_t);    \
  template void launch_adjoint3<T>(const Geometry3&, const Model3Coef<T>&,                   \
                                   const Adj3Launch<T>&, hipStream_t);                       \
  template void launch_tlm3<T>(const Geometry3&, const Model3Coef<T>&, const Tlm3Launch<T>&, \
                               hipStream_t);

MRT3_INSTANTIATE(float)
MRT3_INSTANTIATE(double)

}  // namespace mrt3
