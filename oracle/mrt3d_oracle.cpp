// Plain FP64 CPU oracle for the coupled two-species D3Q19 MRT lattice
// Boltzmann scheme, its exact discrete adjoint (AMRT) and the cost gradient.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark may load this library.  It shares no code,
// header, table or constant with the GPU path and is deliberately slow:
// the moment matrix is built by Gram-Schmidt at run time, the collision is
// a dense 19 x 19 product in moment space, and the adjoint is the transpose
// of a dense local Jacobian.
//
// Paper: A. Belmiloudi, "Optimal Control for Chemotaxis Systems and
// Adjoint-Based Optimization with Multiple-Relaxation-Time Lattice Boltzmann
// Models" (arXiv:1908.03876).  The D3Q19 velocities and weights are those
// of the Remark on DmQq lattices, (sumWi3); Section 3.1 develops the scheme
// on D2Q9 and states that the D3Q19 case follows the same procedure:
//   * M: Gram-Schmidt orthogonalisation (Section 3.1) of the monomials
//     1, |e|^2, |e|^4, e_x, |e|^2 e_x, e_y, |e|^2 e_y, e_z, |e|^2 e_z,
//     3e_x^2 - |e|^2, |e|^2 (3e_x^2 - |e|^2), e_y^2 - e_z^2,
//     |e|^2 (e_y^2 - e_z^2), e_x e_y, e_y e_z, e_x e_z,
//     (e_y^2 - e_z^2) e_x, (e_z^2 - e_x^2) e_y, (e_x^2 - e_y^2) e_z
//     over the 19 velocities; rows 3, 5, 7 are j_x, j_y, j_z.
//   * Pi: diagonal free rates except the 3 x 3 block K on (j_x, j_y, j_z),
//     K = (D / (d Cs^2 tau) + I/2)^-1 (D = d Cs^2 tau (K^-1 - I/2), (PC14)).
//   * (phieq) with zero convective flux and C-tensor: phi_eq_i =
//     w_i (Theta + (d - 1) Cs^2 Theta I:U_i / (2 Cs^4)), I:U_i = |e_i|^2 - 3 Cs^2.
//   * Sources (S), (PhiS): S_u,i = w_i e_i.(A_u1 grad v)/Cs^2, A_u1 =
//     K_u chi u C_chi / tau, grad v = -K_v j_v / (tau d_v Cs^2) (LIBEG);
//     Phi_u = r_u u (1-u), Phi_v = a_uv u - b_v v + c (control on v);
//     first-order source term.
//   * Collide then push-stream along e_i, halfway bounce-back on solid cells
//     (and outside a non-periodic lattice); J = 1/2 sum_F (u^N - u_t)^2 +
//     alpha/2 sum_F c^2; AMRT = transpose of the local Jacobian after the
//     transposed streaming (CAE), (CAEL); gradient sum_n tau sum_i w_i psi_v,i.
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

namespace {

constexpr int Q = 19;
constexpr double TAU = 1.0;
constexpr double CS2 = 1.0 / 3.0;

// (Remark on DmQq lattices, D3Q19), c = 1.
const int EV[Q][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                      {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                      {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {-1, 0, 1}, {1, 0, -1},
                      {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
// (sumWi3)
double wgt(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

int opposite(int i) {
  for (int j = 0; j < Q; ++j)
    if (EV[j][0] == -EV[i][0] && EV[j][1] == -EV[i][1] && EV[j][2] == -EV[i][2]) return j;
  return -1;
}

bool invert(int n, const double* a, double* inv) {
  std::vector<double> m(a, a + n * n);
  for (int i = 0; i < n * n; ++i) inv[i] = 0.0;
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(m[r * n + col]) > std::fabs(m[piv * n + col])) piv = r;
    if (std::fabs(m[piv * n + col]) < 1e-300) return false;
    if (piv != col)
      for (int k = 0; k < n; ++k) {
        std::swap(m[piv * n + k], m[col * n + k]);
        std::swap(inv[piv * n + k], inv[col * n + k]);
      }
    double p = m[col * n + col];
    for (int k = 0; k < n; ++k) {
      m[col * n + k] /= p;
      inv[col * n + k] /= p;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double f = m[r * n + col];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        m[r * n + k] -= f * m[col * n + k];
        inv[r * n + k] -= f * inv[col * n + k];
      }
    }
  }
  return true;
}

// Moment matrix by classical Gram-Schmidt over the monomial list above.
void build_moments(double* M) {
  for (int i = 0; i < Q; ++i) {
    const double x = EV[i][0], y = EV[i][1], z = EV[i][2];
    const double e2 = x * x + y * y + z * z;
    const double p[Q] = {1.0,
                         e2,
                         e2 * e2,
                         x,
                         e2 * x,
                         y,
                         e2 * y,
                         z,
                         e2 * z,
                         3 * x * x - e2,
                         e2 * (3 * x * x - e2),
                         y * y - z * z,
                         e2 * (y * y - z * z),
                         x * y,
                         y * z,
                         x * z,
                         (y * y - z * z) * x,
                         (z * z - x * x) * y,
                         (x * x - y * y) * z};
    for (int k = 0; k < Q; ++k) M[k * Q + i] = p[k];
  }
  for (int k = 0; k < Q; ++k)
    for (int l = 0; l < k; ++l) {
      double num = 0, den = 0;
      for (int i = 0; i < Q; ++i) {
        num += M[k * Q + i] * M[l * Q + i];
        den += M[l * Q + i] * M[l * Q + i];
      }
      for (int i = 0; i < Q; ++i) M[k * Q + i] -= num / den * M[l * Q + i];
    }
}

}  // namespace

extern "C" {

struct Orc3Species {
  double D[9];   // self-diffusion tensor, row-major 3x3
  double d;      // equilibrium parameter d_Theta
  double s[16];  // free rates: s[0] on rho, then moments 1, 2, 4, 6, 8, 9..18
};

struct Orc3Problem {
  int nx, ny, nz;
  int periodic;                // 1: periodic; 0: outside is solid
  const unsigned char* solid;  // nz*ny*nx, 1 = solid, or NULL
  Orc3Species u, v;
  double chi;
  double Cchi[9];
  double r_u, a_uv, b_v;
  double alpha;
};

}  // extern "C"

namespace {

struct Species3Ops {
  double K[9];
  double C[Q * Q];  // M^-1 Pi M
  double weq[Q];
};

struct Ops3 {
  double M[Q * Q], Minv[Q * Q];
  Species3Ops u, v;
  int opp[Q];
};

bool inv3(const double* a, double* r) {
  const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                     a[2] * (a[3] * a[7] - a[4] * a[6]);
  if (std::fabs(det) < 1e-300) return false;
  r[0] = (a[4] * a[8] - a[5] * a[7]) / det;
  r[1] = (a[2] * a[7] - a[1] * a[8]) / det;
  r[2] = (a[1] * a[5] - a[2] * a[4]) / det;
  r[3] = (a[5] * a[6] - a[3] * a[8]) / det;
  r[4] = (a[0] * a[8] - a[2] * a[6]) / det;
  r[5] = (a[2] * a[3] - a[0] * a[5]) / det;
  r[6] = (a[3] * a[7] - a[4] * a[6]) / det;
  r[7] = (a[1] * a[6] - a[0] * a[7]) / det;
  r[8] = (a[0] * a[4] - a[1] * a[3]) / det;
  return true;
}

bool build_species(const Orc3Species& s, const Ops3& ops, Species3Ops& o) {
  double Ki[9];
  for (int k = 0; k < 9; ++k) Ki[k] = s.D[k] / (s.d * CS2 * TAU) + (k % 4 == 0 ? 0.5 : 0.0);
  if (!inv3(Ki, o.K)) return false;
  double Pi[Q * Q] = {0};
  // free rates on the non-conserved, non-flux moments
  const int free_rows[16] = {0, 1, 2, 4, 6, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18};
  for (int k = 0; k < 16; ++k) Pi[free_rows[k] * Q + free_rows[k]] = s.s[k];
  const int jr[3] = {3, 5, 7};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Pi[jr[a] * Q + jr[b]] = o.K[a * 3 + b];
  double PiM[Q * Q];
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j) {
      double acc = 0;
      for (int k = 0; k < Q; ++k) acc += Pi[i * Q + k] * ops.M[k * Q + j];
      PiM[i * Q + j] = acc;
    }
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j) {
      double acc = 0;
      for (int k = 0; k < Q; ++k) acc += ops.Minv[i * Q + k] * PiM[k * Q + j];
      o.C[i * Q + j] = acc;
    }
  for (int i = 0; i < Q; ++i) {
    const double e2 = EV[i][0] * EV[i][0] + EV[i][1] * EV[i][1] + EV[i][2] * EV[i][2];
    o.weq[i] = wgt(i) * (1.0 + (s.d - 1.0) * CS2 * (e2 - 3.0 * CS2) / (2.0 * CS2 * CS2));
  }
  return true;
}

bool build_ops(const Orc3Problem& p, Ops3& ops) {
  build_moments(ops.M);
  if (!invert(Q, ops.M, ops.Minv)) return false;
  for (int i = 0; i < Q; ++i) ops.opp[i] = opposite(i);
  return build_species(p.u, ops, ops.u) && build_species(p.v, ops, ops.v);
}

inline size_t ncell(const Orc3Problem& p) { return size_t(p.nx) * p.ny * p.nz; }

inline bool is_solid(const Orc3Problem& p, int x, int y, int z) {
  if (x < 0 || y < 0 || z < 0 || x >= p.nx || y >= p.ny || z >= p.nz) return true;
  return p.solid && p.solid[(size_t(z) * p.ny + y) * p.nx + x];
}

// Cell x + sign e_i (periodic wrap when periodic), -1 if solid or outside.
inline long neighbour(const Orc3Problem& p, int x, int y, int z, int i, int sign) {
  int xn = x + sign * EV[i][0], yn = y + sign * EV[i][1], zn = z + sign * EV[i][2];
  if (p.periodic) {
    xn = (xn % p.nx + p.nx) % p.nx;
    yn = (yn % p.ny + p.ny) % p.ny;
    zn = (zn % p.nz + p.nz) % p.nz;
  }
  if (is_solid(p, xn, yn, zn)) return -1;
  return long((size_t(zn) * p.ny + yn) * p.nx + xn);
}

// grad Theta = -K j / (tau d Cs^2) with j the first moment.
template <typename T>
void local_grad(const double* K, double d, const T* f, T g[3]) {
  T j[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i)
    for (int a = 0; a < 3; ++a) j[a] += double(EV[i][a]) * f[i];
  for (int a = 0; a < 3; ++a)
    g[a] = -(K[a * 3 + 0] * j[0] + K[a * 3 + 1] * j[1] + K[a * 3 + 2] * j[2]) / (TAU * d * CS2);
}

// A_u1 / u = K_u chi C_chi / tau
void chem_tensor(const Orc3Problem& p, const Ops3& ops, double A[9]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += ops.u.K[a * 3 + k] * p.Cchi[k * 3 + b];
      A[a * 3 + b] = p.chi * acc / TAU;
    }
}

// Local collision at a fluid node: phi [2][Q] -> out [2][Q].
template <typename T>
void collide(const Orc3Problem& p, const Ops3& ops, const T* phi, T c, T* out) {
  const T* fu = phi;
  const T* fv = phi + Q;
  T u = 0, v = 0;
  for (int i = 0; i < Q; ++i) {
    u += fu[i];
    v += fv[i];
  }
  T gv[3];
  local_grad(ops.v.K, p.v.d, fv, gv);
  double A[9];
  chem_tensor(p, ops, A);
  T a[3];
  for (int r = 0; r < 3; ++r) a[r] = u * (A[r * 3] * gv[0] + A[r * 3 + 1] * gv[1] + A[r * 3 + 2] * gv[2]);
  const T Phi[2] = {p.r_u * u * (1.0 - u), p.a_uv * u - p.b_v * v + c};
  for (int s = 0; s < 2; ++s) {
    const Species3Ops& so = s == 0 ? ops.u : ops.v;
    const T* f = phi + s * Q;
    const T theta = s == 0 ? u : v;
    T neq[Q];
    for (int i = 0; i < Q; ++i) neq[i] = f[i] - so.weq[i] * theta;
    for (int i = 0; i < Q; ++i) {
      T acc = 0;
      for (int j = 0; j < Q; ++j) acc += so.C[i * Q + j] * neq[j];
      T S = 0;
      if (s == 0)
        S = wgt(i) * (double(EV[i][0]) * a[0] + double(EV[i][1]) * a[1] + double(EV[i][2]) * a[2]) /
            CS2;
      out[s * Q + i] = f[i] - acc + TAU * S + TAU * wgt(i) * Phi[s];
    }
  }
}

template <typename T>
void init_equilibrium(const Orc3Problem& p, const Ops3& ops, const double* u0, const double* v0,
                      T* f) {
  const size_t nc = ncell(p);
  for (size_t cell = 0; cell < nc; ++cell) {
    const bool sol = p.solid && p.solid[cell];
    for (int i = 0; i < Q; ++i) {
      f[(0 * Q + i) * nc + cell] = sol ? T(0) : T(ops.u.weq[i] * u0[cell]);
      f[(1 * Q + i) * nc + cell] = sol ? T(0) : T(ops.v.weq[i] * v0[cell]);
    }
  }
}

// collide every fluid cell, then push-stream with halfway bounce-back
template <typename T>
void step(const Orc3Problem& p, const Ops3& ops, const T* f, const T* ctrl, T* post, T* fnew) {
  const size_t nc = ncell(p);
#pragma omp parallel for schedule(static)
  for (long cell = 0; cell < long(nc); ++cell) {
    if (p.solid && p.solid[cell]) {
      for (int k = 0; k < 2 * Q; ++k) post[k * nc + cell] = T(0);
      continue;
    }
    T loc[2 * Q], out[2 * Q];
    for (int k = 0; k < 2 * Q; ++k) loc[k] = f[k * nc + cell];
    collide(p, ops, loc, ctrl ? ctrl[cell] : T(0), out);
    for (int k = 0; k < 2 * Q; ++k) post[k * nc + cell] = out[k];
  }
  for (size_t k = 0; k < 2 * Q * nc; ++k) fnew[k] = T(0);
  for (int z = 0; z < p.nz; ++z)
    for (int y = 0; y < p.ny; ++y)
      for (int x = 0; x < p.nx; ++x) {
        const size_t cell = (size_t(z) * p.ny + y) * p.nx + x;
        if (p.solid && p.solid[cell]) continue;
        for (int s = 0; s < 2; ++s)
          for (int i = 0; i < Q; ++i) {
            const long nb = neighbour(p, x, y, z, i, +1);
            const T val = post[(s * Q + i) * nc + cell];
            if (nb >= 0)
              fnew[(s * Q + i) * nc + nb] = val;
            else
              fnew[(s * Q + ops.opp[i]) * nc + cell] = val;
          }
      }
}

// Dense local Jacobian d out / d phi (38 x 38) at a node.
void local_jacobian(const Orc3Problem& p, const Ops3& ops, const double* phi, double* J) {
  const int N2 = 2 * Q;
  for (int k = 0; k < N2 * N2; ++k) J[k] = 0.0;
  const double* fu = phi;
  const double* fv = phi + Q;
  double u = 0;
  for (int i = 0; i < Q; ++i) u += fu[i];
  double gv[3];
  local_grad(ops.v.K, p.v.d, fv, gv);
  double A[9];
  chem_tensor(p, ops, A);
  double Ag[3];
  for (int r = 0; r < 3; ++r) Ag[r] = A[r * 3] * gv[0] + A[r * 3 + 1] * gv[1] + A[r * 3 + 2] * gv[2];
  for (int s = 0; s < 2; ++s) {
    const Species3Ops& so = s == 0 ? ops.u : ops.v;
    // relaxation: I - C + C weq 1^T
    for (int i = 0; i < Q; ++i) {
      double cw = 0;
      for (int k = 0; k < Q; ++k) cw += so.C[i * Q + k] * so.weq[k];
      for (int j = 0; j < Q; ++j)
        J[(s * Q + i) * N2 + s * Q + j] += (i == j ? 1.0 : 0.0) - so.C[i * Q + j] + cw;
    }
  }
  for (int i = 0; i < Q; ++i) {
    const double wi = wgt(i);
    const double ea[3] = {double(EV[i][0]), double(EV[i][1]), double(EV[i][2])};
    const double dSdu = wi * (ea[0] * Ag[0] + ea[1] * Ag[1] + ea[2] * Ag[2]) / CS2;
    for (int j = 0; j < Q; ++j) {
      // through u in the chemotactic flux and in Phi_u; Phi_v through u
      J[(0 * Q + i) * N2 + 0 * Q + j] += TAU * dSdu + TAU * wi * p.r_u * (1.0 - 2.0 * u);
      J[(1 * Q + i) * N2 + 0 * Q + j] += TAU * wi * p.a_uv;
      J[(1 * Q + i) * N2 + 1 * Q + j] += TAU * wi * (-p.b_v);
      // through j_v: d grad v / d phi_v,j = -K_v e_j / (tau d_v Cs^2)
      double dg[3];
      for (int a = 0; a < 3; ++a)
        dg[a] = -(ops.v.K[a * 3] * EV[j][0] + ops.v.K[a * 3 + 1] * EV[j][1] +
                  ops.v.K[a * 3 + 2] * EV[j][2]) / (TAU * p.v.d * CS2);
      double dS = 0;
      for (int r = 0; r < 3; ++r) dS += ea[r] * (A[r * 3] * dg[0] + A[r * 3 + 1] * dg[1] + A[r * 3 + 2] * dg[2]);
      J[(0 * Q + i) * N2 + 1 * Q + j] += TAU * wi * u * dS / CS2;
    }
  }
}

void run_forward(const Orc3Problem& p, const Ops3& ops, int nsteps, const double* u0,
                 const double* v0, const double* c, std::vector<double>& f,
                 std::vector<double>* traj) {
  const size_t nc = ncell(p);
  f.assign(2 * Q * nc, 0.0);
  std::vector<double> post(2 * Q * nc), fnew(2 * Q * nc);
  init_equilibrium(p, ops, u0, v0, f.data());
  if (traj) traj->assign(size_t(nsteps) * 2 * Q * nc, 0.0);
  for (int n = 0; n < nsteps; ++n) {
    if (traj) std::memcpy(traj->data() + size_t(n) * 2 * Q * nc, f.data(), sizeof(double) * 2 * Q * nc);
    step(p, ops, f.data(), c, post.data(), fnew.data());
    f.swap(fnew);
  }
}

}  // namespace

extern "C" {

// Velocities (19 x 3), weights, the Gram-Schmidt moment matrix and its
// inverse (row-major 19 x 19).
int orc3_tables(double* E, double* w, double* M, double* Minv) {
  for (int i = 0; i < Q; ++i) {
    for (int a = 0; a < 3; ++a) E[3 * i + a] = EV[i][a];
    w[i] = wgt(i);
  }
  build_moments(M);
  return invert(Q, M, Minv) ? 0 : -1;
}

// K (3x3), C (19x19) and the equilibrium weights of one species.
int orc3_species_ops(const Orc3Species* s, double* K, double* C, double* weq) {
  Ops3 ops;
  build_moments(ops.M);
  if (!invert(Q, ops.M, ops.Minv)) return -1;
  Species3Ops o;
  if (!build_species(*s, ops, o)) return -1;
  std::memcpy(K, o.K, sizeof o.K);
  std::memcpy(C, o.C, sizeof o.C);
  std::memcpy(weq, o.weq, sizeof o.weq);
  return 0;
}

int orc3_collide(const Orc3Problem* p, const double* phi, double c, double* out) {
  Ops3 ops;
  if (!build_ops(*p, ops)) return -1;
  collide<double>(*p, ops, phi, c, out);
  return 0;
}

int orc3_local_jacobian(const Orc3Problem* p, const double* phi, double* J) {
  Ops3 ops;
  if (!build_ops(*p, ops)) return -1;
  local_jacobian(*p, ops, phi, J);
  return 0;
}

// N steps from the equilibrium of (u0, v0): u^N, v^N and optionally the
// state [2][19][nz][ny][nx].
int orc3_forward(const Orc3Problem* p, int nsteps, const double* u0, const double* v0,
                 const double* c, double* uN, double* vN, double* state) {
  Ops3 ops;
  if (!build_ops(*p, ops) || nsteps < 0) return -1;
  const size_t nc = ncell(*p);
  std::vector<double> f;
  run_forward(*p, ops, nsteps, u0, v0, c, f, nullptr);
  for (size_t cell = 0; cell < nc; ++cell) {
    double u = 0, v = 0;
    for (int i = 0; i < Q; ++i) {
      u += f[(0 * Q + i) * nc + cell];
      v += f[(1 * Q + i) * nc + cell];
    }
    if (uN) uN[cell] = u;
    if (vN) vN[cell] = v;
  }
  if (state) std::memcpy(state, f.data(), sizeof(double) * 2 * Q * nc);
  return 0;
}

// AMRT from psi_u,i(T) = seed_u, psi_v,i(T) = seed_v (may be NULL): g =
// sum_n tau sum_i w_i psi_v,i, and dJ/du0, dJ/dv0 through the equilibrium
// initialisation (may be NULL).
int orc3_adjoint(const Orc3Problem* p, int nsteps, const double* u0, const double* v0,
                 const double* c, const double* seed_u, const double* seed_v, double* g,
                 double* du0, double* dv0) {
  Ops3 ops;
  if (!build_ops(*p, ops) || nsteps < 0) return -1;
  const size_t nc = ncell(*p);
  const int N2 = 2 * Q;
  std::vector<double> f, traj;
  run_forward(*p, ops, nsteps, u0, v0, c, f, &traj);
  std::vector<double> lam(N2 * nc, 0.0), nu(N2 * nc, 0.0);
  for (size_t cell = 0; cell < nc; ++cell) {
    g[cell] = 0.0;
    if (p->solid && p->solid[cell]) continue;
    for (int i = 0; i < Q; ++i) {
      lam[(0 * Q + i) * nc + cell] = seed_u[cell];
      lam[(1 * Q + i) * nc + cell] = seed_v ? seed_v[cell] : 0.0;
    }
  }
  for (int n = nsteps - 1; n >= 0; --n) {
    // transpose of the push streaming with bounce-back
    for (int z = 0; z < p->nz; ++z)
      for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
          const size_t cell = (size_t(z) * p->ny + y) * p->nx + x;
          if (p->solid && p->solid[cell]) continue;
          for (int s = 0; s < 2; ++s)
            for (int i = 0; i < Q; ++i) {
              const long nb = neighbour(*p, x, y, z, i, +1);
              nu[(s * Q + i) * nc + cell] = nb >= 0 ? lam[(s * Q + i) * nc + nb]
                                                    : lam[(s * Q + ops.opp[i]) * nc + cell];
            }
        }
    const double* fn = traj.data() + size_t(n) * N2 * nc;
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < long(nc); ++cell) {
      if (p->solid && p->solid[cell]) continue;
      double loc[2 * Q], nl[2 * Q], J[2 * Q * 2 * Q];
      for (int k = 0; k < N2; ++k) {
        loc[k] = fn[k * nc + cell];
        nl[k] = nu[k * nc + cell];
      }
      double gc = 0.0;
      for (int i = 0; i < Q; ++i) gc += nl[Q + i] * TAU * wgt(i);  // dF_v,i/dc = tau w_i
      g[cell] += gc;
      local_jacobian(*p, ops, loc, J);
      for (int k = 0; k < N2; ++k) {
        double acc = 0;
        for (int r = 0; r < N2; ++r) acc += J[r * N2 + k] * nl[r];
        lam[k * nc + cell] = acc;
      }
    }
  }
  for (size_t cell = 0; cell < nc; ++cell) {
    double a = 0, b = 0;
    if (!(p->solid && p->solid[cell]))
      for (int i = 0; i < Q; ++i) {
        a += ops.u.weq[i] * lam[(0 * Q + i) * nc + cell];
        b += ops.v.weq[i] * lam[(1 * Q + i) * nc + cell];
      }
    if (du0) du0[cell] = a;
    if (dv0) dv0[cell] = b;
  }
  return 0;
}

// Tangent: (du^N, dv^N) for the perturbation (dc, du0, dv0), any NULL = 0.
int orc3_tlm(const Orc3Problem* p, int nsteps, const double* u0, const double* v0,
             const double* c, const double* dc, const double* du0, const double* dv0,
             double* duN, double* dvN) {
  Ops3 ops;
  if (!build_ops(*p, ops) || nsteps < 0) return -1;
  const size_t nc = ncell(*p);
  const int N2 = 2 * Q;
  std::vector<double> f, traj;
  run_forward(*p, ops, nsteps, u0, v0, c, f, &traj);
  std::vector<double> d(N2 * nc, 0.0), dpost(N2 * nc), dnew(N2 * nc);
  for (size_t cell = 0; cell < nc; ++cell) {
    if (p->solid && p->solid[cell]) continue;
    for (int i = 0; i < Q; ++i) {
      d[(0 * Q + i) * nc + cell] = du0 ? ops.u.weq[i] * du0[cell] : 0.0;
      d[(1 * Q + i) * nc + cell] = dv0 ? ops.v.weq[i] * dv0[cell] : 0.0;
    }
  }
  for (int n = 0; n < nsteps; ++n) {
    const double* fn = traj.data() + size_t(n) * N2 * nc;
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < long(nc); ++cell) {
      if (p->solid && p->solid[cell]) {
        for (int k = 0; k < N2; ++k) dpost[k * nc + cell] = 0.0;
        continue;
      }
      double loc[2 * Q], J[2 * Q * 2 * Q];
      for (int k = 0; k < N2; ++k) loc[k] = fn[k * nc + cell];
      local_jacobian(*p, ops, loc, J);
      for (int r = 0; r < N2; ++r) {
        double acc = 0;
        for (int k = 0; k < N2; ++k) acc += J[r * N2 + k] * d[k * nc + cell];
        dpost[r * nc + cell] = acc;
      }
      if (dc)
        for (int i = 0; i < Q; ++i) dpost[(Q + i) * nc + cell] += TAU * wgt(i) * dc[cell];
    }
    std::fill(dnew.begin(), dnew.end(), 0.0);
    for (int z = 0; z < p->nz; ++z)
      for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
          const size_t cell = (size_t(z) * p->ny + y) * p->nx + x;
          if (p->solid && p->solid[cell]) continue;
          for (int s = 0; s < 2; ++s)
            for (int i = 0; i < Q; ++i) {
              const long nb = neighbour(*p, x, y, z, i, +1);
              const double val = dpost[(s * Q + i) * nc + cell];
              if (nb >= 0)
                dnew[(s * Q + i) * nc + nb] = val;
              else
                dnew[(s * Q + ops.opp[i]) * nc + cell] = val;
            }
        }
    d.swap(dnew);
  }
  for (size_t cell = 0; cell < nc; ++cell) {
    double a = 0, b = 0;
    for (int i = 0; i < Q; ++i) {
      a += d[(0 * Q + i) * nc + cell];
      b += d[(1 * Q + i) * nc + cell];
    }
    if (duN) duN[cell] = a;
    if (dvN) dvN[cell] = b;
  }
  return 0;
}

// J at c + i h dc in complex arithmetic (the scheme is polynomial in c).
int orc3_cost_complex_step(const Orc3Problem* p, int nsteps, const double* u0,
                           const double* v0, const double* c, const double* dc, double h,
                           const double* ut, double* J_re, double* J_im) {
  typedef std::complex<double> cd;
  Ops3 ops;
  if (!build_ops(*p, ops) || nsteps < 0) return -1;
  const size_t nc = ncell(*p);
  std::vector<cd> f(2 * Q * nc), post(2 * Q * nc), fnew(2 * Q * nc), cc(nc);
  for (size_t k = 0; k < nc; ++k) cc[k] = cd(c[k], h * dc[k]);
  init_equilibrium<cd>(*p, ops, u0, v0, f.data());
  for (int n = 0; n < nsteps; ++n) {
    step<cd>(*p, ops, f.data(), cc.data(), post.data(), fnew.data());
    f.swap(fnew);
  }
  cd J = 0.0;
  for (size_t cell = 0; cell < nc; ++cell) {
    if (p->solid && p->solid[cell]) continue;
    cd u = 0.0;
    for (int i = 0; i < Q; ++i) u += f[(0 * Q + i) * nc + cell];
    const cd dd = u - ut[cell];
    J += 0.5 * dd * dd + 0.5 * p->alpha * cc[cell] * cc[cell];
  }
  *J_re = J.real();
  *J_im = J.imag();
  return 0;
}

}  // extern "C"
