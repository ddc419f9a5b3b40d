// Internal interface between the D3Q19 C-ABI runtime (mrt3_abi.cpp) and its
// gfx950 kernels (mrt3_kernels.hip).  Not part of the public ABI.
//
// Method: arXiv:1908.03876, Section 3.1 (the D3Q19 lattice of the Remark on
// DmQq lattices with the weights (sumWi3); the MRT collision (MC) in an
// orthogonal moment space, the relaxation matrix with the flux block K,
// D = d Cs^2 tau (K^-1 - I/2), (phieq), the sources (S), (PhiS)) and
// Section 3.2.1 (the exact discrete adjoint, CAE / AEDs / CAEL).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mrt3 {

constexpr int Q = 19;

// D3Q19 velocities, c = 1: rest, the six axis links (+x, -x, +y, -y, +z,
// -z), then the twelve face diagonals in opposite pairs (xy: (1,1,0),
// (-1,-1,0), (1,-1,0), (-1,1,0); xz: (1,0,1), (-1,0,-1), (-1,0,1), (1,0,-1);
// yz: (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1)).  Link 2p+1 and 2p+2 are
// opposite for p = 0..8.
struct Vel {
  int x, y, z;
};

__host__ __device__ constexpr Vel vel(int i) {
  switch (i) {
    case 0: return {0, 0, 0};
    case 1: return {1, 0, 0};
    case 2: return {-1, 0, 0};
    case 3: return {0, 1, 0};
    case 4: return {0, -1, 0};
    case 5: return {0, 0, 1};
    case 6: return {0, 0, -1};
    case 7: return {1, 1, 0};
    case 8: return {-1, -1, 0};
    case 9: return {1, -1, 0};
    case 10: return {-1, 1, 0};
    case 11: return {1, 0, 1};
    case 12: return {-1, 0, -1};
    case 13: return {-1, 0, 1};
    case 14: return {1, 0, -1};
    case 15: return {0, 1, 1};
    case 16: return {0, -1, -1};
    case 17: return {0, 1, -1};
    default: return {0, -1, 1};
  }
}

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Orthogonal D3Q19 moment basis, each row an integer polynomial of e_i
// (the rows are mutually orthogonal over the 19 velocities; their order
// and span are those of Gram-Schmidt applied to the monomials 1, |e|^2,
// |e|^4, e_x, |e|^2 e_x, e_y, |e|^2 e_y, e_z, |e|^2 e_z, 3e_x^2 - |e|^2,
// |e|^2 (3e_x^2 - |e|^2), e_y^2 - e_z^2, |e|^2 (e_y^2 - e_z^2), e_x e_y,
// e_y e_z, e_x e_z, (e_y^2 - e_z^2) e_x, (e_z^2 - e_x^2) e_y,
// (e_x^2 - e_y^2) e_z): density, energy, energy square, j_x, q_x, j_y,
// q_y, j_z, q_z, the five stresses, two fourth-order companions and three
// third-order moments.  Scaling a row does not change the relaxation,
// whose rate is divided by the row's squared norm.
__host__ __device__ constexpr int mrow(int k, int i) {
  const Vel e = vel(i);
  const int x = e.x, y = e.y, z = e.z, e2 = x * x + y * y + z * z;
  switch (k) {
    case 0: return 1;
    case 1: return 19 * e2 - 30;
    case 2: return (21 * e2 * e2 - 53 * e2 + 24) / 2;
    case 3: return x;
    case 4: return (5 * e2 - 9) * x;
    case 5: return y;
    case 6: return (5 * e2 - 9) * y;
    case 7: return z;
    case 8: return (5 * e2 - 9) * z;
    case 9: return 3 * x * x - e2;
    case 10: return (3 * e2 - 5) * (3 * x * x - e2);
    case 11: return y * y - z * z;
    case 12: return (3 * e2 - 5) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
  }
}

// Rows of the free rates s[0..15] of a species: the density (no effect,
// conserved), energy, energy square, the three q's, then rows 9..18.
__host__ __device__ constexpr int free_row(int j) {
  return j < 3 ? j : (j < 6 ? 2 * j - 2 : j + 3);
}

// Relaxation coefficients of one species: c[k] = s_k / |row k|^2 on the
// free rows (0 on the density and flux rows), the flux block K / 10
// (|row 3|^2 = |row 5|^2 = |row 7|^2 = 10) and its transpose, the
// equilibrium moments of rows 1 and 2 per unit Theta, and the equilibrium
// weights w~ by shell (every other row's equilibrium vanishes: w~ depends
// on |e| only and the flux is zero).
template <typename T>
struct Species3Coef {
  T c[Q];
  T k[9];
  T e_eq, eps_eq;
  T w_rest, w_axis, w_diag;
};

template <typename T>
struct Model3Coef {
  Species3Coef<T> u, v;
  T b[9];               // chemotactic source a = u * B * j_v, row-major
  T r_u, a_uv, b_v;     // kinetics
};

// Fields (controls, seeds, records, outputs) use the public layout
// [nz][ny][pitch].  The distribution buffers the library owns use an
// internal layout with halo rows and slabs in y and z: node (x, y, z) at
// ((z + 1)(ny + 2) + y + 1) pitchI + x, pitchI = nx rounded up to 64, so
// that every neighbour x +- e_i of a node, also outside a non-periodic
// lattice, is an in-bounds address (x = -1 and x = nx fall on the end and
// the start of the adjacent rows).  Values read there for a neighbour
// outside the lattice are discarded by the bounce-back (the link word marks
// the outside as a wall), so a pull is a uniform plane base plus one
// per-node offset with no edge test.
struct Geometry3 {
  int nx, ny, nz, pitch;
  int periodic;            // 1: periodic wrap; 0: walls at the lattice edge
  int masked;              // 1: link words in use (a mask, or walls at the
                           // edge of a non-periodic lattice)
  uint32_t plane;          // public plane, nz * ny * pitch elements
  int pitchI;              // internal row stride
  uint32_t planeI;         // internal plane, (nz + 2)(ny + 2) pitchI elements
  const uint32_t* link;    // [nz][ny][pitch] when masked: bit 0 node solid,
                           // bit i = node x - e_i solid or, on a
                           // non-periodic lattice, outside (wrapped when
                           // periodic)
  const uint32_t* wflag;   // [nz][ny][nsx]: 0 = a 64-node row segment and
                           // its neighbours are fluid, 1 = mixed, 2 = solid
  int nsx;                 // ceil(nx / 64)
  int band;                // y-rows per band of the tile order, band_of()
};

// Internal row stride and plane size of a lattice.
inline int internal_pitch(int nx) { return ((nx + 63) / 64) * 64; }
inline size_t internal_plane(int nx, int ny, int nz) {
  return size_t(nz + 2) * size_t(ny + 2) * size_t(internal_pitch(nx));
}

// Height of the y-bands in which the kernels take rows z-fastest.  The 8
// XCDs own equal contiguous ranges of tiles, so a band of ny / 8 rows is
// one XCD's share and the rows on either side of a band edge run at the
// same time on two XCDs.  That share is cut into equal bands when the rows
// between z-neighbours, band * nx nodes at about 336 bytes each, would not
// stay in an XCD's 4 MB L2 (band * nx <= 8192: 32 rows of 256 nodes).
inline int band_of(int nx, int ny) {
  const int share = (ny + 7) / 8;
  const int most = nx >= 8192 ? 1 : 8192 / nx;
  const int nb = (share + most - 1) / most;
  return (share + nb - 1) / nb;
}

void launch_build_link3(const Geometry3& g, const uint8_t* mask, uint32_t* link,
                        uint32_t* wflag, uint16_t* solid16, hipStream_t s);

template <typename T>
struct Fwd3Launch {
  const T* src;   // post-collision state of step n-1, or null (first step)
  T* dst;         // post-collision state of step n (with wall slots)
  const T* u0;    // initial fields (first step only)
  const T* v0;
  const T* ctrl;  // control c(x)
  T* rec;         // record slot [4][plane] (u, j_vx, j_vy, j_vz) or null
};

template <typename T>
void launch_forward3(const Geometry3& g, const Model3Coef<T>& m, const Fwd3Launch<T>& a,
                     hipStream_t s);

// Terminal streaming: state [2][19][plane] in the public layout (may be
// null), u^N, v^N (may be null).
template <typename T>
void launch_finalize3(const Geometry3& g, const T* src, T* state, T* uN, T* vN,
                      hipStream_t s);

template <typename T>
struct Adj3Launch {
  const T* src;     // adjoint state of step n+1, or null (terminal seed)
  T* dst;           // adjoint state of step n, or null (step 0)
  const T* seed_u;  // terminal condition (first step only)
  const T* seed_v;  // may be null (= 0)
  const T* rec;     // record slot of step n
  double* g;        // gradient accumulator
  T* adj_u0;        // dJ/du0, dJ/dv0 (step 0 only, may be null)
  T* adj_v0;
  int first;        // 1: step N-1 (reads the seeds, initialises g)
  int last;         // 1: step 0 with adj_u0 / adj_v0 requested
};

template <typename T>
void launch_adjoint3(const Geometry3& g, const Model3Coef<T>& m, const Adj3Launch<T>& a,
                     hipStream_t s);

template <typename T>
struct Tlm3Launch {
  const T* src;   // perturbation of step n-1 (post-collision), or null (n = 0)
  T* dst;         // perturbation after step n (with wall slots)
  const T* du0;   // initial perturbations (n = 0 only; null = 0)
  const T* dv0;
  const T* dc;    // control perturbation (null = 0)
  const T* rec;   // record slot of step n
};

template <typename T>
void launch_tlm3(const Geometry3& g, const Model3Coef<T>& m, const Tlm3Launch<T>& a,
                 hipStream_t s);

}  // namespace mrt3
