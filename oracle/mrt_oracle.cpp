// Plain FP64 CPU oracle for the coupled two- or three-species D2Q9 MRT
// lattice Boltzmann scheme, its exact discrete adjoint (AMRT) and the cost
// gradient.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark may load this library.  It shares no code,
// header, table or constant with the GPU path and is deliberately slow:
// explicit 9x9 matrix products, explicit local Jacobians, push streaming,
// a generic Gauss-Jordan inverse of the moment matrix.
//
// Paper: A. Belmiloudi, "Optimal Control for Chemotaxis Systems and
// Adjoint-Based Optimization with Multiple-Relaxation-Time Lattice Boltzmann
// Models" (arXiv:1908.03876).  Equation labels below are the paper's.
//
// Instance computed (two species, Theta in {u, v}, lattice units
// h = tau = c = 1, 3 Cs^2 = c^2 so Cs^2 = 1/3, Section 3.1):
//   * D2Q9 velocities and weights: Remark on DmQq lattices, (sumWi).
//   * Moment matrix M = E0 M0 with E0 = I for c = 1 (Section 3.1, the
//     transportation matrix); relaxation matrix Pi = diag(Lambda1, Lambda2,
//     Lambda3) with the 2x2 K block coupling j_x and j_y.
//   * K_Theta from D_Theta = d_Theta Cs^2 tau (K^-1 - I/2) (parameter
//     choices at the end of the proof of Proposition 1, (PC14)).
//   * Equilibrium (phieq) with convective flux and C-tensor set to zero.
//   * Cross-diffusion source (S): S_u,i = w_i e_i.(A_u1 grad v)/Cs^2 with
//     A_u1 = K_u D_u1 / tau and D_u1 = chi u C_chi (attraction-repulsion
//     example (ARC), chi_k = X u I generalised to a tensor shape C_chi).
//     grad v is computed locally from the distributions (LIBEG): from the
//     first-moment balance (C146), tau Cs^2 d_v grad v = -K_v j_v^neq, and
//     j_v^eq = 0, so grad v = -K_v j_v / (tau d_v Cs^2) with j_v the
//     pre-collision first moment of v.
//   * Reaction source (PhiS) with V = 0: Phi_Theta,i = w_i Phi_Theta,
//     Phi_u = r_u u (1-u), Phi_v = a_uv u - b_v v + c(x) (control on v).
//   * Third species (optional, attraction-repulsion example (ARC)): a
//     repulsive signal w with Phi_w = a_w u - b_w w + s_w and the second
//     cross-diffusion of u, D_u2 = chi_w u C_w (chi_w < 0 repels), whose
//     source A_u2 grad w joins S_u with grad w read from j_w like grad v.
//   * The second-order source term (tau^2/2)(kappa_t d/dt + kappa_x e.grad)
//     of (eq:LBEG): by the explicit or the implicit characteristic
//     difference of the Remark after (eq:LBEG) (source_term 2 or 3, two
//     species), else omitted (source_term 1).
//   * One step = collision (MC) in moment space (MF), then streaming along
//     e_i (eq:LBE); halfway bounce-back on solid cells and, when the lattice
//     is not periodic, outside the domain.
//   * Cost (classicJ)/(EJD-H): J = 1/2 sum_F (u^N - u_t)^2 + alpha/2 sum_F c^2.
//   * Adjoint: AMRT (CAE), (AEDs), (RFS1) with Lambda* = C^T, adjoint
//     streaming along -e_i backward in time (CAEL); terminal condition
//     psi(T) = dI0/dphi; gradient (gradientLattice): sum over steps of
//     sum_i psi_v,i dF_v,i/dc with dF_v,i/dc = tau w_i.
//   * Sensitivity LBE (LIBEG-V) as a forward-mode linearisation (TLM).
//   * Gradient step (Section 2.4, Step 5 and the heuristic step
//     zeta = min(1, 1/||E||_inf)).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

constexpr int Q = 9;
constexpr int NSX = 3;  // at most three species
constexpr double TAU = 1.0;
constexpr double CS2 = 1.0 / 3.0;

// D2Q9: e0 = 0, e1 = (1,0), e2 = (0,1), e3 = -e1, e4 = -e2, e5 = (1,1),
// e6 = (-1,1), e7 = -e5, e8 = -e6.
const int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const double WGT[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                       1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// M0 (Section 3.1): rows are the moments rho, e, epsilon, j_x, q_x, j_y,
// q_y, p_xx, p_xy.
const double M0[Q][Q] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

int opposite(int i) {
  for (int j = 0; j < Q; ++j)
    if (EX[j] == -EX[i] && EY[j] == -EY[i]) return j;
  return -1;
}

// Generic Gauss-Jordan inverse with partial pivoting (n x n, row-major).
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

void matmul(int n, const double* a, const double* b, double* c) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += a[i * n + k] * b[k * n + j];
      c[i * n + j] = s;
    }
}

}  // namespace

extern "C" {

struct OrcSpecies {
  double D[4];  // self-diffusion tensor, row-major 2x2
  double d;     // equilibrium parameter d_Theta
  double s[7];  // free relaxation rates s_0 .. s_6
};

struct OrcProblem {
  int nx, ny;
  int periodic;                // 1: periodic wrap; 0: outside is solid
  const unsigned char* solid;  // ny*nx, 1 = solid, or NULL
  OrcSpecies u, v;
  double chi;
  double Cchi[4];
  double r_u, a_uv, b_v;
  double alpha;
  int control_on_u;  // 0: control enters Phi_v (default); 1: enters Phi_u
  // Source term of (eq:LBEG): 0 or 1: tau F_i; 2: plus (tau^2/2) dF_i/dt
  // by the explicit characteristic difference (kappa_t = 1, kappa_x = 0);
  // 3: plus (tau^2/2)(d/dt + e_i.grad) F_i by the implicit characteristic
  // difference (kappa_t = kappa_x = 1).
  int source_term;
  // Species count: 2 (u, v) or 3 (u, v, w; first-order source term only).
  int nspecies;
  OrcSpecies w;
  double chi_w;      // D_u2 = chi_w u C_w
  double Cw[4];
  double a_w, b_w, s_w;
  const double* w0;  // initial w [ny*nx] (NULL = 0)
};

}  // extern "C"

namespace {

// Per-species precomputed operators.
struct SpeciesOps {
  double K[4];      // 2x2 relaxation block
  double Pi[Q * Q]; // relaxation matrix in moment space
  double C[Q * Q];  // M^-1 Pi M, the collision matrix in velocity space
  double weq[Q];    // phi_eq_i = weq_i * Theta
};

struct Ops {
  double Minv[Q * Q];
  SpeciesOps u, v, w;
  int opp[Q];
};

inline int nspec(const OrcProblem& p) { return p.nspecies == 3 ? 3 : 2; }

inline const SpeciesOps& sops(const Ops& ops, int s) {
  return s == 0 ? ops.u : (s == 1 ? ops.v : ops.w);
}

void k_from_D(const OrcSpecies& s, double K[4]) {
  // K^-1 = D/(d Cs^2 tau) + I/2  (from D = d Cs^2 tau (K^-1 - I/2)).
  double a = s.D[0] / (s.d * CS2 * TAU) + 0.5;
  double b = s.D[1] / (s.d * CS2 * TAU);
  double c = s.D[2] / (s.d * CS2 * TAU);
  double e = s.D[3] / (s.d * CS2 * TAU) + 0.5;
  double det = a * e - b * c;
  K[0] = e / det;
  K[1] = -b / det;
  K[2] = -c / det;
  K[3] = a / det;
}

void build_species(const OrcSpecies& s, const double* Minv, SpeciesOps& o) {
  k_from_D(s, o.K);
  for (int i = 0; i < Q * Q; ++i) o.Pi[i] = 0.0;
  // Lambda1 = diag(s0, s1, s2) on (rho, e, epsilon)
  o.Pi[0 * Q + 0] = s.s[0];
  o.Pi[1 * Q + 1] = s.s[1];
  o.Pi[2 * Q + 2] = s.s[2];
  // Lambda2 = [[k11, 0, k12], [0, s3, 0], [k21, 0, k22]] on (j_x, q_x, j_y)
  o.Pi[3 * Q + 3] = o.K[0];
  o.Pi[3 * Q + 5] = o.K[1];
  o.Pi[4 * Q + 4] = s.s[3];
  o.Pi[5 * Q + 3] = o.K[2];
  o.Pi[5 * Q + 5] = o.K[3];
  // Lambda3 = diag(s4, s5, s6) on (q_y, p_xx, p_xy)
  o.Pi[6 * Q + 6] = s.s[4];
  o.Pi[7 * Q + 7] = s.s[5];
  o.Pi[8 * Q + 8] = s.s[6];
  double PiM[Q * Q];
  matmul(Q, o.Pi, &M0[0][0], PiM);
  matmul(Q, Minv, PiM, o.C);
  // (phieq) with T = 0, C-tensor = 0:
  // phi_eq_i = w_i (Theta + (d Cs^2 Theta - Cs^2 Theta) I:U_i / (2 Cs^4)),
  // U_i = e_i (x) e_i - Cs^2 I, so I:U_i = |e_i|^2 - 2 Cs^2.
  for (int i = 0; i < Q; ++i) {
    double trU = double(EX[i] * EX[i] + EY[i] * EY[i]) - 2.0 * CS2;
    o.weq[i] = WGT[i] * (1.0 + (s.d * CS2 - CS2) * trU / (2.0 * CS2 * CS2));
  }
}

bool build_ops(const OrcProblem& p, Ops& ops) {
  if (!invert(Q, &M0[0][0], ops.Minv)) return false;
  if (p.nspecies == 3 && p.source_term > 1) return false;  // not defined here
  build_species(p.u, ops.Minv, ops.u);
  build_species(p.v, ops.Minv, ops.v);
  build_species(p.nspecies == 3 ? p.w : p.v, ops.Minv, ops.w);
  for (int i = 0; i < Q; ++i) ops.opp[i] = opposite(i);
  return true;
}

inline bool is_solid(const OrcProblem& p, int x, int y) {
  if (x < 0 || y < 0 || x >= p.nx || y >= p.ny) return true;  // non-periodic only
  return p.solid && p.solid[y * p.nx + x];
}

// Neighbour x + e_i (with periodic wrap when periodic); returns -1 if that
// node is solid (or outside a non-periodic domain).
inline int neighbour(const OrcProblem& p, int x, int y, int i, int sign) {
  int xn = x + sign * EX[i], yn = y + sign * EY[i];
  if (p.periodic) {
    xn = (xn % p.nx + p.nx) % p.nx;
    yn = (yn % p.ny + p.ny) % p.ny;
  }
  if (is_solid(p, xn, yn)) return -1;
  return yn * p.nx + xn;
}

// ------------------------------------------------------------------ forward

// Local collision at one fluid node (eq:LBE with (S), (PhiS), (MF), (MC)).
// phi: pre-collision [NS][Q] (species u, v, then w); out: post-collision.
// Second-order source (eq:LBEG with kappa_t = 1, kappa_x = 0): when Fprev
// holds Phi_u, Phi_v of the previous step at this node, the term
// (tau^2/2) dF_i/dt is taken by the explicit characteristic difference
// (F_i(t) - F_i(t - tau)) / tau of the Remark after (eq:LBEG).  Fnow (if
// given) receives Phi_u, Phi_v of this step.
// With `implicit` (kappa_t = kappa_x = 1, implicit characteristic
// difference (F_i(x + e_i tau, t + tau) - F_i(x, t)) / tau), only the
// explicit half -(tau/2) F_i(x, t) is added here; the other half belongs to
// the arrival node and is added by implicit_node after streaming.
template <typename T>
void collide(const OrcProblem& p, const Ops& ops, const T* phi, T c, T* out,
             const T* Fprev = nullptr, T* Fnow = nullptr, bool implicit = false) {
  const int NS = nspec(p);
  const T* fu = phi;
  const T* fv = phi + Q;
  // (UGS): macroscopic values; first moment of v.
  T u = 0, v = 0, jx = 0, jy = 0;
  for (int i = 0; i < Q; ++i) {
    u += fu[i];
    v += fv[i];
    jx += double(EX[i]) * fv[i];
    jy += double(EY[i]) * fv[i];
  }
  // grad v computed locally from the distributions.
  const double* Kv = ops.v.K;
  T gvx = -(Kv[0] * jx + Kv[1] * jy) / (TAU * p.v.d * CS2);
  T gvy = -(Kv[2] * jx + Kv[3] * jy) / (TAU * p.v.d * CS2);
  // D_u1 = chi u C_chi ; A_u1 = K_u D_u1 / tau ; a = A_u1 grad v.
  T D1[4];
  for (int k = 0; k < 4; ++k) D1[k] = p.chi * u * p.Cchi[k];
  const double* Ku = ops.u.K;
  T A[4];
  A[0] = (Ku[0] * D1[0] + Ku[1] * D1[2]) / TAU;
  A[1] = (Ku[0] * D1[1] + Ku[1] * D1[3]) / TAU;
  A[2] = (Ku[2] * D1[0] + Ku[3] * D1[2]) / TAU;
  A[3] = (Ku[2] * D1[1] + Ku[3] * D1[3]) / TAU;
  T ax = A[0] * gvx + A[1] * gvy;
  T ay = A[2] * gvx + A[3] * gvy;
  // Third species: grad w from j_w, D_u2 = chi_w u C_w, A_u2 = K_u D_u2 / tau.
  T wv = 0, Phi_w = 0;
  if (NS == 3) {
    const T* fw = phi + 2 * Q;
    T kx = 0, ky = 0;
    for (int i = 0; i < Q; ++i) {
      wv += fw[i];
      kx += double(EX[i]) * fw[i];
      ky += double(EY[i]) * fw[i];
    }
    const double* Kw = ops.w.K;
    T gwx = -(Kw[0] * kx + Kw[1] * ky) / (TAU * p.w.d * CS2);
    T gwy = -(Kw[2] * kx + Kw[3] * ky) / (TAU * p.w.d * CS2);
    T D2[4], A2[4];
    for (int k = 0; k < 4; ++k) D2[k] = p.chi_w * u * p.Cw[k];
    A2[0] = (Ku[0] * D2[0] + Ku[1] * D2[2]) / TAU;
    A2[1] = (Ku[0] * D2[1] + Ku[1] * D2[3]) / TAU;
    A2[2] = (Ku[2] * D2[0] + Ku[3] * D2[2]) / TAU;
    A2[3] = (Ku[2] * D2[1] + Ku[3] * D2[3]) / TAU;
    ax += A2[0] * gwx + A2[1] * gwy;
    ay += A2[2] * gwx + A2[3] * gwy;
    Phi_w = p.a_w * u - p.b_w * wv + p.s_w;
  }
  // Kinetics.
  T Phi_u = p.r_u * u * (1.0 - u);
  T Phi_v = p.a_uv * u - p.b_v * v;
  if (p.control_on_u)
    Phi_u += c;
  else
    Phi_v += c;
  if (Fnow) {
    Fnow[0] = Phi_u;
    Fnow[1] = Phi_v;
  }
  for (int s = 0; s < NS; ++s) {
    const SpeciesOps& so = sops(ops, s);
    const T* f = phi + s * Q;
    T theta = s == 0 ? u : (s == 1 ? v : wv);
    T Phi = s == 0 ? Phi_u : (s == 1 ? Phi_v : Phi_w);
    // (MF): m = M F, m_eq = M F_eq.
    T feq[Q], m[Q], meq[Q], mcol[Q];
    for (int i = 0; i < Q; ++i) feq[i] = so.weq[i] * theta;
    for (int r = 0; r < Q; ++r) {
      m[r] = 0;
      meq[r] = 0;
      for (int i = 0; i < Q; ++i) {
        m[r] += M0[r][i] * f[i];
        meq[r] += M0[r][i] * feq[i];
      }
    }
    // (MC): m_col = m - Pi (m - m_eq).
    for (int r = 0; r < Q; ++r) {
      T acc = 0;
      for (int k = 0; k < Q; ++k) acc += so.Pi[r * Q + k] * (m[k] - meq[k]);
      mcol[r] = m[r] - acc;
    }
    for (int i = 0; i < Q; ++i) {
      T back = 0;
      for (int r = 0; r < Q; ++r) back += ops.Minv[i * Q + r] * mcol[r];
      // (S): only the u equation carries a cross-diffusion source.
      T S = 0;
      if (s == 0) S = WGT[i] * (double(EX[i]) * ax + double(EY[i]) * ay) / CS2;
      // (PhiS) with V = 0.
      T PhiI = WGT[i] * Phi;
      T second = 0;
      if (Fprev && s < 2) second = (TAU * TAU / 2.0) * (PhiI - WGT[i] * Fprev[s]) / TAU;
      if (implicit) second = -(TAU * TAU / 2.0) * PhiI / TAU;
      out[s * Q + i] = back + TAU * S + TAU * PhiI + second;
    }
  }
}

// State layout: f[(s*Q + i)*ncell + cell], cell = y*nx + x.
template <typename T>
void init_equilibrium(const OrcProblem& p, const Ops& ops, const T* u0,
                      const T* v0, T* f) {
  const int nc = p.nx * p.ny;
  for (int cell = 0; cell < nc; ++cell) {
    bool sol = p.solid && p.solid[cell];
    for (int i = 0; i < Q; ++i) {
      f[(0 * Q + i) * nc + cell] = sol ? T(0) : ops.u.weq[i] * u0[cell];
      f[(1 * Q + i) * nc + cell] = sol ? T(0) : ops.v.weq[i] * v0[cell];
      if (nspec(p) == 3)
        f[(2 * Q + i) * nc + cell] =
            sol || !p.w0 ? T(0) : T(ops.w.weq[i] * p.w0[cell]);
    }
  }
}

// Push streaming along e_i with halfway bounce-back of both species:
// phi_i(x + e_i) = post_i(x), or phi_opp(i)(x) = post_i(x) when x + e_i is
// solid (or outside a non-periodic lattice).
template <typename T>
void stream_push(const OrcProblem& p, const Ops& ops, const T* post, T* fnew) {
  const int nc = p.nx * p.ny;
  const int NS = nspec(p);
  for (int k = 0; k < NS * Q * nc; ++k) fnew[k] = T(0);
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p.ny; ++y)
    for (int x = 0; x < p.nx; ++x) {
      int cell = y * p.nx + x;
      if (p.solid && p.solid[cell]) continue;
      for (int s = 0; s < NS; ++s)
        for (int i = 0; i < Q; ++i) {
          // Streaming into neighbours would race between rows under OpenMP
          // only if two sources targeted one slot; each (target, i) has a
          // unique source, so the writes are disjoint.
          int nb = neighbour(p, x, y, i, +1);
          T val = post[(s * Q + i) * nc + cell];
          if (nb >= 0)
            fnew[(s * Q + i) * nc + nb] = val;
          else
            fnew[(s * Q + ops.opp[i]) * nc + cell] = val;
        }
    }
}

// Implicit half of the characteristic difference at a fluid node y: the
// populations R_i streamed into y give phi_i = R_i + (tau/2) w_i Phi(Theta)
// with Theta = sum_i phi_i, so Theta - (tau/2) Phi(Theta) = sum_i R_i, a
// 2 x 2 nonlinear system (Phi_u depends on u, Phi_v on u and v) solved by
// Newton's method; then phi_i follows.  ph: [2][Q], R in, phi out.
template <typename T>
void implicit_node(const OrcProblem& p, T* ph, T c) {
  const double h = TAU / 2.0;
  const T cu = p.control_on_u ? c : T(0), cv = p.control_on_u ? T(0) : c;
  T Ru = 0, Rv = 0;
  for (int i = 0; i < Q; ++i) {
    Ru += ph[i];
    Rv += ph[Q + i];
  }
  T u = Ru, v = Rv;
  int extra = 0;
  for (int it = 0; it < 100 && extra < 3; ++it) {
    const T fu = u - Ru - h * (p.r_u * u * (1.0 - u) + cu);
    const T fv = v - Rv - h * (p.a_uv * u - p.b_v * v + cv);
    // Jacobian [[1 - h r (1 - 2u), 0], [-h a, 1 + h b]]
    const T j11 = 1.0 - h * p.r_u * (1.0 - 2.0 * u);
    const T j22 = 1.0 + h * p.b_v;
    const T du = fu / j11;
    const T dv = (fv + h * p.a_uv * du) / j22;
    u -= du;
    v -= dv;
    if (std::abs(du) <= 1e-15 * (1.0 + std::abs(u)) &&
        std::abs(dv) <= 1e-15 * (1.0 + std::abs(v)))
      ++extra;  // converged; a few more iterations settle the last bits
  }
  const T Phi_u = p.r_u * u * (1.0 - u) + cu;
  const T Phi_v = p.a_uv * u - p.b_v * v + cv;
  for (int i = 0; i < Q; ++i) {
    ph[i] += h * WGT[i] * Phi_u;
    ph[Q + i] += h * WGT[i] * Phi_v;
  }
}

// One step: collide every fluid node, then push-stream along e_i with
// halfway bounce-back (eq:LBE): phi_i(x + e_i, t+1) = phi*_i(x), or
// phi_opp(i)(x, t+1) = phi*_i(x) when x + e_i is solid.
// With source_term 2, F [2][ncell] holds Phi_u, Phi_v of the previous
// step on entry and those of this step on exit; at the first step (first =
// true) there is no previous value and the difference term is taken as
// zero (F_i(-tau) = F_i(0)).
template <typename T>
void step(const OrcProblem& p, const Ops& ops, const T* f, const T* ctrl,
          T* post, T* fnew, T* F = nullptr, bool first = true) {
  const int nc = p.nx * p.ny;
  const int NQ = nspec(p) * Q;
  const bool second = p.source_term == 2 && F != nullptr;
  const bool implicit = p.source_term == 3;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < p.ny; ++y)
    for (int x = 0; x < p.nx; ++x) {
      int cell = y * p.nx + x;
      if (p.solid && p.solid[cell]) {
        for (int k = 0; k < NQ; ++k) post[k * nc + cell] = T(0);
        continue;
      }
      T loc[NSX * Q], out[NSX * Q];
      for (int k = 0; k < NQ; ++k) loc[k] = f[k * nc + cell];
      T prev[2], now[2];
      if (second) {
        prev[0] = F[cell];
        prev[1] = F[nc + cell];
      }
      collide(p, ops, loc, ctrl ? ctrl[cell] : T(0), out,
              second && !first ? prev : nullptr, second ? now : nullptr, implicit);
      if (second) {
        F[cell] = now[0];
        F[nc + cell] = now[1];
      }
      for (int k = 0; k < NQ; ++k) post[k * nc + cell] = out[k];
    }
  stream_push(p, ops, post, fnew);
  if (implicit) {
#pragma omp parallel for schedule(static)
    for (int cell = 0; cell < nc; ++cell) {
      if (p.solid && p.solid[cell]) continue;
      T ph[2 * Q];
      for (int k = 0; k < 2 * Q; ++k) ph[k] = fnew[k * nc + cell];
      implicit_node(p, ph, ctrl ? ctrl[cell] : T(0));
      for (int k = 0; k < 2 * Q; ++k) fnew[k * nc + cell] = ph[k];
    }
  }
}

// ------------------------------------------------- continuous adjoint

// Collision of the continuous-adjoint system (FVM-PF-Adj-K for the
// two-species instance) solved by the same MRT scheme in reversed time
// s = T - t (Section 3.2.2).  With p the adjoint of u and q that of v:
//   p_s = div(D_u grad p) + chi (C grad v) . grad p + r_u (1 - 2u) p + a_uv q
//   q_s = div(D_v grad q) - b_v q - div(chi u C^T grad p)
// p relaxes like u (K_u, weq_u) and q like v.  The gradients come from the
// first moments as in the forward: grad v = -K_v j_v / (tau d_v Cs^2) from
// the forward populations fw at this time, grad p = -K_u j_p / (tau d_u Cs^2)
// from the adjoint populations.  The cross-diffusion of q by p enters as the
// flux source a_q = K_v (chi u C^T grad p) / tau, the other terms as scalar
// sources.  phi: pre-collision [p (Q), q (Q)]; out: post-collision.
void cadj_collide(const OrcProblem& p, const Ops& ops, const double* fw, const double* phi,
                  double* out) {
  double u = 0, jvx = 0, jvy = 0;
  for (int i = 0; i < Q; ++i) {
    u += fw[i];
    jvx += EX[i] * fw[Q + i];
    jvy += EY[i] * fw[Q + i];
  }
  const double* fp = phi;
  const double* fq = phi + Q;
  double P = 0, Qv = 0, jpx = 0, jpy = 0;
  for (int i = 0; i < Q; ++i) {
    P += fp[i];
    Qv += fq[i];
    jpx += EX[i] * fp[i];
    jpy += EY[i] * fp[i];
  }
  const double* Kv = ops.v.K;
  const double* Ku = ops.u.K;
  const double gvx = -(Kv[0] * jvx + Kv[1] * jvy) / (TAU * p.v.d * CS2);
  const double gvy = -(Kv[2] * jvx + Kv[3] * jvy) / (TAU * p.v.d * CS2);
  const double gpx = -(Ku[0] * jpx + Ku[1] * jpy) / (TAU * p.u.d * CS2);
  const double gpy = -(Ku[2] * jpx + Ku[3] * jpy) / (TAU * p.u.d * CS2);
  const double cgx = p.Cchi[0] * gvx + p.Cchi[1] * gvy;
  const double cgy = p.Cchi[2] * gvx + p.Cchi[3] * gvy;
  const double Phi_p = p.r_u * (1.0 - 2.0 * u) * P + p.a_uv * Qv + p.chi * (cgx * gpx + cgy * gpy);
  const double Phi_q = -p.b_v * Qv;
  // chi u C^T grad p, then K_v / tau
  const double fx = p.chi * u * (p.Cchi[0] * gpx + p.Cchi[2] * gpy);
  const double fy = p.chi * u * (p.Cchi[1] * gpx + p.Cchi[3] * gpy);
  const double aqx = (Kv[0] * fx + Kv[1] * fy) / TAU;
  const double aqy = (Kv[2] * fx + Kv[3] * fy) / TAU;
  for (int s = 0; s < 2; ++s) {
    const SpeciesOps& so = s == 0 ? ops.u : ops.v;
    const double* f = s == 0 ? fp : fq;
    const double theta = s == 0 ? P : Qv;
    const double Phi = s == 0 ? Phi_p : Phi_q;
    double m[Q], meq[Q], mcol[Q], feq[Q];
    for (int i = 0; i < Q; ++i) feq[i] = so.weq[i] * theta;
    for (int r = 0; r < Q; ++r) {
      m[r] = 0;
      meq[r] = 0;
      for (int i = 0; i < Q; ++i) {
        m[r] += M0[r][i] * f[i];
        meq[r] += M0[r][i] * feq[i];
      }
    }
    for (int r = 0; r < Q; ++r) {
      double acc = 0;
      for (int k = 0; k < Q; ++k) acc += so.Pi[r * Q + k] * (m[k] - meq[k]);
      mcol[r] = m[r] - acc;
    }
    for (int i = 0; i < Q; ++i) {
      double back = 0;
      for (int r = 0; r < Q; ++r) back += ops.Minv[i * Q + r] * mcol[r];
      double S = 0;
      if (s == 1) S = WGT[i] * (EX[i] * aqx + EY[i] * aqy) / CS2;
      out[s * Q + i] = back + TAU * S + TAU * WGT[i] * Phi;
    }
  }
}

// Jacobian of the local sources R = tau S + tau Phi of all species with
// respect to the pre-collision node value (NS Q x NS Q, row = output (s,i),
// column = input (s',j)), assembled from the partial derivatives of each
// term of (S) and (PhiS).
void source_jacobian(const OrcProblem& p, const Ops& ops, const double* phi,
                     double* dR, double phi_scale = 1.0) {
  const double* fu = phi;
  const double* fv = phi + Q;
  double u = 0, jx = 0, jy = 0;
  for (int i = 0; i < Q; ++i) {
    u += fu[i];
    jx += EX[i] * fv[i];
    jy += EY[i] * fv[i];
  }
  const int NS = nspec(p);
  const int N2 = NS * Q;
  for (int k = 0; k < N2 * N2; ++k) dR[k] = 0.0;
  const double* Kv = ops.v.K;
  const double* Ku = ops.u.K;
  double gvx = -(Kv[0] * jx + Kv[1] * jy) / (TAU * p.v.d * CS2);
  double gvy = -(Kv[2] * jx + Kv[3] * jy) / (TAU * p.v.d * CS2);
  // A_u1 / u = K_u chi C_chi / tau
  double Au[4];
  Au[0] = p.chi * (Ku[0] * p.Cchi[0] + Ku[1] * p.Cchi[2]) / TAU;
  Au[1] = p.chi * (Ku[0] * p.Cchi[1] + Ku[1] * p.Cchi[3]) / TAU;
  Au[2] = p.chi * (Ku[2] * p.Cchi[0] + Ku[3] * p.Cchi[2]) / TAU;
  Au[3] = p.chi * (Ku[2] * p.Cchi[1] + Ku[3] * p.Cchi[3]) / TAU;
  // third species: A_u2 / u = K_u chi_w C_w / tau and grad w from j_w
  double Aw[4] = {0, 0, 0, 0}, gwx = 0, gwy = 0;
  const double* Kw = ops.w.K;
  if (NS == 3) {
    double kx = 0, ky = 0;
    for (int i = 0; i < Q; ++i) {
      kx += EX[i] * phi[2 * Q + i];
      ky += EY[i] * phi[2 * Q + i];
    }
    gwx = -(Kw[0] * kx + Kw[1] * ky) / (TAU * p.w.d * CS2);
    gwy = -(Kw[2] * kx + Kw[3] * ky) / (TAU * p.w.d * CS2);
    Aw[0] = p.chi_w * (Ku[0] * p.Cw[0] + Ku[1] * p.Cw[2]) / TAU;
    Aw[1] = p.chi_w * (Ku[0] * p.Cw[1] + Ku[1] * p.Cw[3]) / TAU;
    Aw[2] = p.chi_w * (Ku[2] * p.Cw[0] + Ku[3] * p.Cw[2]) / TAU;
    Aw[3] = p.chi_w * (Ku[2] * p.Cw[1] + Ku[3] * p.Cw[3]) / TAU;
  }
  for (int i = 0; i < Q; ++i) {
    double wi = WGT[i];
    double ex = EX[i], ey = EY[i];
    // dS_u,i/dphi_u,j = w_i e_i.(Au grad v + Aw grad w)/Cs^2 (through u)
    double dSdu = wi * (ex * (Au[0] * gvx + Au[1] * gvy + Aw[0] * gwx + Aw[1] * gwy) +
                        ey * (Au[2] * gvx + Au[3] * gvy + Aw[2] * gwx + Aw[3] * gwy)) / CS2;
    for (int j = 0; j < Q; ++j) {
      dR[(0 * Q + i) * N2 + (0 * Q + j)] += TAU * dSdu;
      // dS_u,i/dphi_v,j = w_i e_i.(u Au dgradv/dphi_v,j)/Cs^2 with
      // dgradv/dphi_v,j = -K_v e_j/(tau d_v Cs^2)
      double dgx = -(Kv[0] * EX[j] + Kv[1] * EY[j]) / (TAU * p.v.d * CS2);
      double dgy = -(Kv[2] * EX[j] + Kv[3] * EY[j]) / (TAU * p.v.d * CS2);
      double dS = wi * u * (ex * (Au[0] * dgx + Au[1] * dgy) +
                            ey * (Au[2] * dgx + Au[3] * dgy)) / CS2;
      dR[(0 * Q + i) * N2 + (1 * Q + j)] += TAU * dS;
      // Phi_u = r_u u (1-u): dPhi_u,i/dphi_u,j = w_i r_u (1 - 2u)
      dR[(0 * Q + i) * N2 + (0 * Q + j)] += phi_scale * TAU * wi * p.r_u * (1.0 - 2.0 * u);
      // Phi_v = a u - b v + c
      dR[(1 * Q + i) * N2 + (0 * Q + j)] += phi_scale * TAU * wi * p.a_uv;
      dR[(1 * Q + i) * N2 + (1 * Q + j)] += phi_scale * TAU * wi * (-p.b_v);
      if (NS == 3) {
        // dS_u,i/dphi_w,j through grad w = -K_w j_w / (tau d_w Cs^2)
        double hx = -(Kw[0] * EX[j] + Kw[1] * EY[j]) / (TAU * p.w.d * CS2);
        double hy = -(Kw[2] * EX[j] + Kw[3] * EY[j]) / (TAU * p.w.d * CS2);
        double dSw = wi * u * (ex * (Aw[0] * hx + Aw[1] * hy) +
                               ey * (Aw[2] * hx + Aw[3] * hy)) / CS2;
        dR[(0 * Q + i) * N2 + (2 * Q + j)] += TAU * dSw;
        // Phi_w = a_w u - b_w w + s_w
        dR[(2 * Q + i) * N2 + (0 * Q + j)] += TAU * wi * p.a_w;
        dR[(2 * Q + i) * N2 + (2 * Q + j)] += TAU * wi * (-p.b_w);
      }
    }
  }
}

// Jacobian of the relaxation part phi - C (phi - phi_eq(phi)) of one
// species: I - C + C O^T with O_ij = d phi_eq_j / d phi_i = weq_j (RFS1).
void relaxation_jacobian(const SpeciesOps& so, double* Jr) {
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j) {
      double cw = 0.0;
      for (int k = 0; k < Q; ++k) cw += so.C[i * Q + k] * so.weq[k];
      Jr[i * Q + j] = (i == j ? 1.0 : 0.0) - so.C[i * Q + j] + cw;
    }
}

// Full local Jacobian of the collision map: block-diagonal relaxation part
// plus the source part.
void local_jacobian(const OrcProblem& p, const Ops& ops, const double* phi,
                    double* Jac, double phi_scale = 1.0) {
  const int NS = nspec(p);
  const int N2 = NS * Q;
  source_jacobian(p, ops, phi, Jac, phi_scale);
  for (int s = 0; s < NS; ++s) {
    double Jr[Q * Q];
    relaxation_jacobian(sops(ops, s), Jr);
    for (int i = 0; i < Q; ++i)
      for (int j = 0; j < Q; ++j) Jac[(s * Q + i) * N2 + (s * Q + j)] += Jr[i * Q + j];
  }
}

// Adjoint of the local collision following (CAE)/(AEDs): with
// Lambda* = C^T and O_ij = d phi_eq_j / d phi_i,
//   lambda_i = nu_i - [Lambda* (nu - psi_eq)]_i + R~_i,
//   Lambda* (nu - psi_eq) = Lambda* nu - O Lambda* nu,
//   R~_i = sum_k nu_k dR_k/dphi_i  (R = tau S + tau Phi over both species).
//
// With rho given (source_term 2), the kinetics part of R is left out of
// dR and enters as sum_s rho_s dPhi_s/dphi_i instead, rho_s being the
// adjoint of the node's Phi_s of this step.
void local_adjoint(const OrcProblem& p, const Ops& ops, const double* phi,
                   const double* nu, double* lam, const double* rho = nullptr,
                   double phi_scale = 1.0) {
  const int NS = nspec(p);
  const int N2 = NS * Q;
  double dR[NSX * Q * NSX * Q];
  source_jacobian(p, ops, phi, dR, rho == nullptr ? phi_scale : 0.0);
  double dphi[NSX] = {0.0, 0.0, 0.0};  // sum_s rho_s dPhi_s / dTheta_{s'}
  if (rho) {
    double u = 0.0;
    for (int i = 0; i < Q; ++i) u += phi[i];
    dphi[0] = rho[0] * p.r_u * (1.0 - 2.0 * u) + rho[1] * p.a_uv;
    dphi[1] = -rho[1] * p.b_v;
  }
  for (int s = 0; s < NS; ++s) {
    const SpeciesOps& so = sops(ops, s);
    const double* n = nu + s * Q;
    double Ln[Q];  // Lambda* nu = C^T nu
    for (int i = 0; i < Q; ++i) {
      Ln[i] = 0.0;
      for (int k = 0; k < Q; ++k) Ln[i] += so.C[k * Q + i] * n[k];
    }
    for (int i = 0; i < Q; ++i) {
      double OLn = 0.0;  // (O Lambda* nu)_i = sum_j dphi_eq_j/dphi_i (Lambda* nu)_j
      for (int j = 0; j < Q; ++j) OLn += so.weq[j] * Ln[j];
      double Rt = 0.0;
      for (int k = 0; k < N2; ++k) Rt += nu[k] * dR[k * N2 + (s * Q + i)];
      lam[s * Q + i] = n[i] - (Ln[i] - OLn) + Rt + dphi[s];
    }
  }
}

// Transpose of implicit_node at a node whose solved state is ph (the
// arrival populations of the step): with lam the adjoint of the output
// populations, sigma_s = w . lam_s, J = dPhi/dTheta and
// M = I - (tau/2) J (the Jacobian of the node equation), the adjoint of the
// streamed sum is Sbar = M^-T (tau/2) J^T sigma and lam_s,i += Sbar_s.
// The control enters Phi directly and through Theta; its gradient
// contribution is (tau/2)(sigma + Sbar) of the controlled species.
void implicit_node_adjoint(const OrcProblem& p, const double* ph, double* lam, double* gc) {
  const double h = TAU / 2.0;
  double u = 0.0, su = 0.0, sv = 0.0;
  for (int i = 0; i < Q; ++i) {
    u += ph[i];
    su += WGT[i] * lam[i];
    sv += WGT[i] * lam[Q + i];
  }
  const double tu = h * (su * p.r_u * (1.0 - 2.0 * u) + sv * p.a_uv);
  const double tv = h * (-p.b_v * sv);
  const double Sv = tv / (1.0 + h * p.b_v);
  const double Su = (tu + h * p.a_uv * Sv) / (1.0 - h * p.r_u * (1.0 - 2.0 * u));
  for (int i = 0; i < Q; ++i) {
    lam[i] += Su;
    lam[Q + i] += Sv;
  }
  *gc = p.control_on_u ? h * (su + Su) : h * (sv + Sv);
}

// Tangent of implicit_node: d (in: the perturbation of the streamed
// populations, out: of the solved ones) at a node whose solved state is ph.
void implicit_node_tangent(const OrcProblem& p, const double* ph, double dc, double* d) {
  const double h = TAU / 2.0;
  double u = 0.0, dRu = 0.0, dRv = 0.0;
  for (int i = 0; i < Q; ++i) {
    u += ph[i];
    dRu += d[i];
    dRv += d[Q + i];
  }
  const double dcu = p.control_on_u ? dc : 0.0, dcv = p.control_on_u ? 0.0 : dc;
  const double du = (dRu + h * dcu) / (1.0 - h * p.r_u * (1.0 - 2.0 * u));
  const double dv = (dRv + h * dcv + h * p.a_uv * du) / (1.0 + h * p.b_v);
  const double dPu = p.r_u * (1.0 - 2.0 * u) * du + dcu;
  const double dPv = p.a_uv * du - p.b_v * dv + dcv;
  for (int i = 0; i < Q; ++i) {
    d[i] += h * WGT[i] * dPu;
    d[Q + i] += h * WGT[i] * dPv;
  }
}

void run_forward(const OrcProblem& p, const Ops& ops, int nsteps,
                 const double* u0, const double* v0, const double* c,
                 std::vector<double>& f, std::vector<double>* traj) {
  const size_t nc = size_t(p.nx) * p.ny;
  const size_t NQ = size_t(nspec(p)) * Q;
  f.assign(NQ * nc, 0.0);
  std::vector<double> post(NQ * nc), fnew(NQ * nc);
  std::vector<double> F(2 * nc, 0.0);
  init_equilibrium(p, ops, u0, v0, f.data());
  if (traj) traj->assign(size_t(nsteps) * NQ * nc, 0.0);
  for (int n = 0; n < nsteps; ++n) {
    if (traj) std::memcpy(traj->data() + size_t(n) * NQ * nc, f.data(),
                          sizeof(double) * NQ * nc);
    step(p, ops, f.data(), c, post.data(), fnew.data(), F.data(), n == 0);
    f.swap(fnew);
  }
}

// Bytes of states a Trajectory keeps whole; longer runs are checkpointed.
size_t g_traj_budget = size_t(16) << 30;

// The states phi^n (before step n; phi^N after the last step) of one forward
// solve, as the backward sweep needs them, newest first.  When all of them
// fit in g_traj_budget bytes they are kept from the one forward run.
// Otherwise phi^n (with the previous step's kinetics that source_term 2
// carries) is kept every K = ceil(sqrt(N)) steps, and the K states of a
// segment are computed again from its checkpoint when the sweep first asks
// for one of them.  Each step is a deterministic function of its input, so a
// recomputed state is the stored one bit for bit: this changes the memory,
// not the arithmetic.
class Trajectory {
 public:
  Trajectory(const OrcProblem& p, const Ops& ops, int nsteps, const double* u0,
             const double* v0, const double* c)
      : p_(p), ops_(ops), c_(c), N_(nsteps),
        nc_(size_t(p.nx) * p.ny), NQ_(size_t(nspec(p)) * Q) {
    const size_t sbytes = NQ_ * nc_ * sizeof(double);
    K_ = (size_t(nsteps) + 1) * sbytes <= g_traj_budget
             ? std::max(nsteps, 1)
             : int(std::ceil(std::sqrt(double(nsteps))));
    post_.assign(NQ_ * nc_, 0.0);
    fnew_.assign(NQ_ * nc_, 0.0);
    std::vector<double> f(NQ_ * nc_, 0.0), F(2 * nc_, 0.0);
    init_equilibrium(p, ops, u0, v0, f.data());
    const bool all = K_ >= nsteps;
    if (all) {
      seg_.assign(size_t(std::max(nsteps, 1)) * NQ_ * nc_, 0.0);
      seg_start_ = 0;
    }
    for (int n = 0; n < nsteps; ++n) {
      if (all)
        std::memcpy(seg_.data() + size_t(n) * NQ_ * nc_, f.data(), sbytes);
      else if (n % K_ == 0) {
        ckpt_f_.push_back(f);
        ckpt_F_.push_back(F);
      }
      step(p, ops, f.data(), c, post_.data(), fnew_.data(), F.data(), n == 0);
      std::swap(f, fnew_);
    }
    final_ = f;
  }

  // phi^n, 0 <= n <= N
  const double* state(int n) {
    if (n == N_) return final_.data();
    if (seg_start_ < 0 || n < seg_start_ || n >= seg_start_ + K_) load(n / K_);
    return seg_.data() + size_t(n - seg_start_) * NQ_ * nc_;
  }

 private:
  void load(int s) {
    const int start = s * K_, len = std::min(K_, N_ - start);
    seg_.assign(size_t(len) * NQ_ * nc_, 0.0);
    std::vector<double> f = ckpt_f_[s], F = ckpt_F_[s];
    for (int j = 0; j < len; ++j) {
      std::memcpy(seg_.data() + size_t(j) * NQ_ * nc_, f.data(), NQ_ * nc_ * sizeof(double));
      step(p_, ops_, f.data(), c_, post_.data(), fnew_.data(), F.data(), start + j == 0);
      std::swap(f, fnew_);
    }
    seg_start_ = start;
  }

  const OrcProblem& p_;
  const Ops& ops_;
  const double* c_;
  int N_, K_ = 1, seg_start_ = -1;
  size_t nc_, NQ_;
  std::vector<double> seg_, final_, post_, fnew_;
  std::vector<std::vector<double>> ckpt_f_, ckpt_F_;
};

}  // namespace

extern "C" {

// Largest number of bytes of forward states the adjoint keeps whole before
// it checkpoints (test control; default 16 GiB).
void orc_set_traj_budget(size_t bytes) { g_traj_budget = bytes; }

// Tables for the lattice pins: E (9x2), weights, M0, M0^-1 (Gauss-Jordan).
int orc_tables(double* E, double* w, double* M, double* Minv) {
  for (int i = 0; i < Q; ++i) {
    E[2 * i] = EX[i];
    E[2 * i + 1] = EY[i];
    w[i] = WGT[i];
  }
  std::memcpy(M, &M0[0][0], sizeof(double) * Q * Q);
  return invert(Q, &M0[0][0], Minv) ? 0 : -1;
}

// K, Pi, C = M^-1 Pi M and the equilibrium weights of one species.
int orc_species_ops(const OrcSpecies* s, double* K, double* Pi, double* C,
                    double* weq) {
  double Minv[Q * Q];
  if (!invert(Q, &M0[0][0], Minv)) return -1;
  SpeciesOps o;
  build_species(*s, Minv, o);
  std::memcpy(K, o.K, sizeof o.K);
  std::memcpy(Pi, o.Pi, sizeof o.Pi);
  std::memcpy(C, o.C, sizeof o.C);
  std::memcpy(weq, o.weq, sizeof o.weq);
  return 0;
}

// One local collision: phi[NS*9] pre-collision -> out[NS*9] post-collision.
int orc_collide(const OrcProblem* p, const double* phi, double c, double* out) {
  Ops ops;
  if (!build_ops(*p, ops)) return -1;
  collide<double>(*p, ops, phi, c, out);
  return 0;
}

int orc_local_jacobian(const OrcProblem* p, const double* phi, double* Jac) {
  Ops ops;
  if (!build_ops(*p, ops)) return -1;
  local_jacobian(*p, ops, phi, Jac);
  return 0;
}

int orc_local_adjoint(const OrcProblem* p, const double* phi, const double* nu,
                      double* lam) {
  Ops ops;
  if (!build_ops(*p, ops)) return -1;
  local_adjoint(*p, ops, phi, nu, lam);
  return 0;
}

// Forward solve: N steps from the equilibrium of (u0, v0) (and w0).
// Outputs u^N and v^N (after the last streaming) and optionally the full
// distribution state state[NS][9][ny][nx] and the per-step pre-collision
// trajectory of u and j_v (traj_u[N][ny*nx], traj_j[N][2][ny*nx]).
int orc_forward(const OrcProblem* p, int nsteps, const double* u0,
                const double* v0, const double* c, double* uN, double* vN,
                double* state, double* traj_u, double* traj_j) {
  Ops ops;
  if (!build_ops(*p, ops) || nsteps < 0) return -1;
  const size_t nc = size_t(p->nx) * p->ny;
  const size_t NQ = size_t(nspec(*p)) * Q;
  std::vector<double> f(NQ * nc), post(NQ * nc), fnew(NQ * nc), F(2 * nc, 0.0);
  init_equilibrium(*p, ops, u0, v0, f.data());
  for (int n = 0; n < nsteps; ++n) {
    if (traj_u || traj_j)
      for (size_t cell = 0; cell < nc; ++cell) {
        double u = 0, jx = 0, jy = 0;
        for (int i = 0; i < Q; ++i) {
          u += f[(0 * Q + i) * nc + cell];
          jx += EX[i] * f[(1 * Q + i) * nc + cell];
          jy += EY[i] * f[(1 * Q + i) * nc + cell];
        }
        if (traj_u) traj_u[size_t(n) * nc + cell] = u;
        if (traj_j) {
          traj_j[(size_t(n) * 2 + 0) * nc + cell] = jx;
          traj_j[(size_t(n) * 2 + 1) * nc + cell] = jy;
        }
      }
    step<double>(*p, ops, f.data(), c, post.data(), fnew.data(), F.data(), n == 0);
    f.swap(fnew);
  }
  for (size_t cell = 0; cell < nc; ++cell) {
    double u = 0, v = 0;
    for (int i = 0; i < Q; ++i) {
      u += f[(0 * Q + i) * nc + cell];
      v += f[(1 * Q + i) * nc + cell];
    }
    if (uN) uN[cell] = u;
    if (vN) vN[cell] = v;
  }
  if (state) std::memcpy(state, f.data(), sizeof(double) * NQ * nc);
  return 0;
}

// Cost (classicJ) on fluid nodes: J = 1/2 sum (uN - ut)^2 + alpha/2 sum c^2.
double orc_cost(const OrcProblem* p, const double* uN, const double* ut,
                const double* c, double* J_track, double* J_reg) {
  const size_t nc = size_t(p->nx) * p->ny;
  double jt = 0.0, jr = 0.0;
  for (size_t cell = 0; cell < nc; ++cell) {
    if (p->solid && p->solid[cell]) continue;
    double d = uN[cell] - ut[cell];
    jt += 0.5 * d * d;
    if (c) jr += 0.5 * p->alpha * c[cell] * c[cell];
  }
  if (J_track) *J_track = jt;
  if (J_reg) *J_reg = jr;
  return jt + jr;
}

// Discrete adjoint sweep (AMRT) with terminal condition
// psi_u,i(T) = seed_u, psi_v,i(T) = seed_v (seed_v may be NULL = 0).
// Outputs g[cell] = sum_n tau sum_i w_i psi_v,i (the adjoint part of the
// gradient w.r.t. the control; the control enters Phi_u instead when
// control_on_u), and optionally dJ/du0, dJ/dv0 through the equilibrium
// initialisation.
//
// g_theta (may be NULL; first source form, nsteps >= 1): the paper's
// trapezoid form of the same gradient (JD-H-B) as a diagnostic.  Its
// integrand at t_n is the control derivative of step n paired with the
// adjoint that carries it, h_n = tau sum_i w_i nu_c,i^n (the terms the exact
// gradient g sums over n = 0 .. N-1), and at t_N the terminal adjoint at the
// node, h_N = tau sum_i w_i psi_c,i^N; with theta_0 = theta_N = 1/2,
//   g_theta = g - h_0 / 2 + h_N / 2,
// an O(1/N) departure from the exact transpose.
static int adjoint_impl(const OrcProblem* p, int nsteps, const double* u0,
                        const double* v0, const double* c, const double* seed_u,
                        const double* seed_v, double* g, double* du0, double* dv0,
                        double* g_theta) {
  Ops ops;
  if (!build_ops(*p, ops) || nsteps < 0) return -1;
  if (g_theta && (p->source_term != 1 || nsteps < 1)) return -1;
  const size_t nc = size_t(p->nx) * p->ny;
  const int NS = nspec(*p);
  const size_t NQ = size_t(NS) * Q;
  Trajectory traj(*p, ops, nsteps, u0, v0, c);
  std::vector<double> lam(NQ * nc, 0.0), nu(NQ * nc, 0.0);
  for (size_t cell = 0; cell < nc; ++cell) {
    if (p->solid && p->solid[cell]) continue;
    for (int i = 0; i < Q; ++i) {
      lam[(0 * Q + i) * nc + cell] = seed_u[cell];
      lam[(1 * Q + i) * nc + cell] = seed_v ? seed_v[cell] : 0.0;
    }
  }
  for (size_t cell = 0; cell < nc; ++cell) g[cell] = 0.0;
  const int cs = p->control_on_u ? 0 : 1;
  if (g_theta) {
    // theta_N h_N from the terminal condition held in lam
    for (size_t cell = 0; cell < nc; ++cell) {
      double s = 0.0;
      if (!(p->solid && p->solid[cell]))
        for (int i = 0; i < Q; ++i) s += WGT[i] * lam[(cs * Q + i) * nc + cell];
      g_theta[cell] = 0.5 * TAU * s;
    }
  }
  // source_term 2: the state of the scheme also holds F(t - tau), i.e.
  // Phi_u, Phi_v of the previous step; mu [2][ncell] is its adjoint (the
  // adjoint of the Phi stored by step n, read by step n + 1; 0 after the
  // last step, which nothing reads).
  const bool so2 = p->source_term == 2;
  std::vector<double> mu(so2 ? 2 * nc : 0, 0.0);
  // source_term 3: each step ends with the implicit node solve at the
  // arrival nodes, whose transpose comes first
  const bool implicit = p->source_term == 3;
  for (int n = nsteps - 1; n >= 0; --n) {
    if (implicit) {
      const double* fa = traj.state(n + 1);
#pragma omp parallel for schedule(static)
      for (int cell = 0; cell < int(nc); ++cell) {
        if (p->solid && p->solid[cell]) continue;
        double ph[2 * Q], lm[2 * Q], gc;
        for (int k = 0; k < 2 * Q; ++k) {
          ph[k] = fa[k * nc + cell];
          lm[k] = lam[k * nc + cell];
        }
        implicit_node_adjoint(*p, ph, lm, &gc);
        for (int k = 0; k < 2 * Q; ++k) lam[k * nc + cell] = lm[k];
        g[cell] += gc;
      }
    }
    // Adjoint streaming along -e_i (transpose of push + bounce-back):
    // nu_i(x) = lambda_i(x + e_i) if x + e_i is fluid, else lambda_opp(i)(x).
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        int cell = y * p->nx + x;
        if (p->solid && p->solid[cell]) continue;
        for (int s = 0; s < NS; ++s)
          for (int i = 0; i < Q; ++i) {
            int nb = neighbour(*p, x, y, i, +1);
            nu[(s * Q + i) * nc + cell] =
                nb >= 0 ? lam[(s * Q + i) * nc + nb]
                        : lam[(s * Q + ops.opp[i]) * nc + cell];
          }
      }
    const double* fn = traj.state(n);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        int cell = y * p->nx + x;
        if (p->solid && p->solid[cell]) continue;
        double loc[NSX * Q], nl[NSX * Q], out[NSX * Q];
        for (int k = 0; k < int(NQ); ++k) {
          loc[k] = fn[k * nc + cell];
          nl[k] = nu[k * nc + cell];
        }
        if (!so2) {
          // (gradientLattice): dF_Theta,i/dc = tau w_i (tau/2 for the
          // explicit half of the implicit characteristic difference).
          const double kphi = implicit ? 0.5 : 1.0;
          double gc = 0.0;
          for (int i = 0; i < Q; ++i) gc += nl[cs * Q + i] * kphi * TAU * WGT[i];
          g[cell] += gc;
          if (g_theta) g_theta[cell] += (n == 0 ? 0.5 : 1.0) * gc;  // theta_n h_n
          local_adjoint(*p, ops, loc, nl, out, nullptr, kphi);
        } else {
          // out_i = ... + tau w_i Phi + (tau/2) w_i (Phi - F_prev) (n >= 1):
          // d out_i / d Phi = (tau + tau/2) w_i, d out_i / d F_prev =
          // -(tau/2) w_i; Phi of this step is also stored for step n + 1.
          double sig[2] = {0.0, 0.0}, rho[2];
          for (int q = 0; q < 2; ++q)
            for (int i = 0; i < Q; ++i) sig[q] += nl[q * Q + i] * WGT[i];
          const double kdir = TAU + (n >= 1 ? TAU / 2.0 : 0.0);
          for (int q = 0; q < 2; ++q) {
            rho[q] = kdir * sig[q] + mu[q * nc + cell];
            mu[q * nc + cell] = n >= 1 ? -(TAU / 2.0) * sig[q] : 0.0;
          }
          g[cell] += rho[cs];  // dPhi_cs / dc = 1
          local_adjoint(*p, ops, loc, nl, out, rho);
        }
        for (int k = 0; k < int(NQ); ++k) lam[k * nc + cell] = out[k];
      }
  }
  // Transpose of the equilibrium initialisation phi_i^0 = weq_i Theta_0.
  for (size_t cell = 0; cell < nc; ++cell) {
    double a = 0.0, b = 0.0;
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

int orc_adjoint(const OrcProblem* p, int nsteps, const double* u0, const double* v0,
                const double* c, const double* seed_u, const double* seed_v, double* g,
                double* du0, double* dv0) {
  return adjoint_impl(p, nsteps, u0, v0, c, seed_u, seed_v, g, du0, dv0, nullptr);
}

// The diagnostic g_theta of adjoint_impl alone.
int orc_adjoint_theta(const OrcProblem* p, int nsteps, const double* u0, const double* v0,
                      const double* c, const double* seed_u, const double* seed_v,
                      double* g_theta) {
  std::vector<double> g(size_t(p->nx) * p->ny);
  return adjoint_impl(p, nsteps, u0, v0, c, seed_u, seed_v, g.data(), nullptr, nullptr,
                      g_theta);
}

// Sensitivity LBE (LIBEG-V), forward mode: directional derivative of
// (u^N, v^N) for a perturbation (dc, du0, dv0) (any may be NULL = 0).
int orc_tlm(const OrcProblem* p, int nsteps, const double* u0,
            const double* v0, const double* c, const double* dc,
            const double* du0, const double* dv0, double* duN, double* dvN) {
  Ops ops;
  if (!build_ops(*p, ops) || nsteps < 0) return -1;
  const size_t nc = size_t(p->nx) * p->ny;
  const int NS = nspec(*p);
  const size_t NQ = size_t(NS) * Q;
  std::vector<double> f, traj;
  run_forward(*p, ops, nsteps, u0, v0, c, f, &traj);
  std::vector<double> d(NQ * nc, 0.0), dpost(NQ * nc), dnew(NQ * nc);
  for (size_t cell = 0; cell < nc; ++cell) {
    if (p->solid && p->solid[cell]) continue;
    for (int i = 0; i < Q; ++i) {
      d[(0 * Q + i) * nc + cell] = du0 ? ops.u.weq[i] * du0[cell] : 0.0;
      d[(1 * Q + i) * nc + cell] = dv0 ? ops.v.weq[i] * dv0[cell] : 0.0;
    }
  }
  const int cs = p->control_on_u ? 0 : 1;
  const int N2 = int(NQ);
  // source_term 2: dF [2][ncell] is the perturbation of the stored Phi of
  // the previous step.
  const bool so2 = p->source_term == 2;
  std::vector<double> dF(so2 ? 2 * nc : 0, 0.0);
  const bool implicit = p->source_term == 3;
  for (int n = 0; n < nsteps; ++n) {
    const double* fn = traj.data() + size_t(n) * NQ * nc;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        int cell = y * p->nx + x;
        if (p->solid && p->solid[cell]) {
          for (int k = 0; k < N2; ++k) dpost[k * nc + cell] = 0.0;
          continue;
        }
        double loc[NSX * Q], Jac[NSX * Q * NSX * Q];
        for (int k = 0; k < N2; ++k) loc[k] = fn[k * nc + cell];
        local_jacobian(*p, ops, loc, Jac, so2 ? 0.0 : (implicit ? 0.5 : 1.0));
        for (int r = 0; r < N2; ++r) {
          double acc = 0.0;
          for (int k = 0; k < N2; ++k) acc += Jac[r * N2 + k] * d[k * nc + cell];
          dpost[r * nc + cell] = acc;
        }
        if (!so2) {
          const double kphi = implicit ? 0.5 : 1.0;
          if (dc)
            for (int i = 0; i < Q; ++i)
              dpost[(cs * Q + i) * nc + cell] += kphi * TAU * WGT[i] * dc[cell];
        } else {
          // perturbation of Phi_u, Phi_v (with the control) of this step
          double u = 0.0, du = 0.0, dv = 0.0;
          for (int i = 0; i < Q; ++i) {
            u += loc[i];
            du += d[(0 * Q + i) * nc + cell];
            dv += d[(1 * Q + i) * nc + cell];
          }
          const double dcc = dc ? dc[cell] : 0.0;
          double dphi[2];
          dphi[0] = p->r_u * (1.0 - 2.0 * u) * du + (cs == 0 ? dcc : 0.0);
          dphi[1] = p->a_uv * du - p->b_v * dv + (cs == 1 ? dcc : 0.0);
          for (int q = 0; q < 2; ++q) {
            for (int i = 0; i < Q; ++i) {
              double add = TAU * WGT[i] * dphi[q];
              if (n >= 1) add += (TAU / 2.0) * WGT[i] * (dphi[q] - dF[q * nc + cell]);
              dpost[(q * Q + i) * nc + cell] += add;
            }
            dF[q * nc + cell] = dphi[q];
          }
        }
      }
    std::fill(dnew.begin(), dnew.end(), 0.0);
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        int cell = y * p->nx + x;
        if (p->solid && p->solid[cell]) continue;
        for (int s = 0; s < NS; ++s)
          for (int i = 0; i < Q; ++i) {
            int nb = neighbour(*p, x, y, i, +1);
            double val = dpost[(s * Q + i) * nc + cell];
            if (nb >= 0)
              dnew[(s * Q + i) * nc + nb] = val;
            else
              dnew[(s * Q + ops.opp[i]) * nc + cell] = val;
          }
      }
    if (implicit) {
      const double* fa = n + 1 < nsteps ? traj.data() + size_t(n + 1) * NQ * nc : f.data();
      for (size_t cell = 0; cell < nc; ++cell) {
        if (p->solid && p->solid[cell]) continue;
        double ph[NSX * Q], dl[NSX * Q];
        for (int k = 0; k < N2; ++k) {
          ph[k] = fa[k * nc + cell];
          dl[k] = dnew[k * nc + cell];
        }
        implicit_node_tangent(*p, ph, dc ? dc[cell] : 0.0, dl);
        for (int k = 0; k < N2; ++k) dnew[k * nc + cell] = dl[k];
      }
    }
    d.swap(dnew);
  }
  for (size_t cell = 0; cell < nc; ++cell) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < Q; ++i) {
      a += d[(0 * Q + i) * nc + cell];
      b += d[(1 * Q + i) * nc + cell];
    }
    if (duN) duN[cell] = a;
    if (dvN) dvN[cell] = b;
  }
  return 0;
}

// Complex-step evaluation of J at c + i h dc: the scheme is polynomial in
// c (bounce-back is a fixed permutation), so Im J / h is the exact
// directional derivative up to O(h^2).
int orc_cost_complex_step(const OrcProblem* p, int nsteps, const double* u0,
                          const double* v0, const double* c, const double* dc,
                          double h, const double* ut, double* J_re,
                          double* J_im) {
  typedef std::complex<double> cd;
  Ops ops;
  if (!build_ops(*p, ops) || nsteps < 0) return -1;
  const size_t nc = size_t(p->nx) * p->ny;
  const size_t NQ = size_t(nspec(*p)) * Q;
  std::vector<cd> f(NQ * nc), post(NQ * nc), fnew(NQ * nc);
  std::vector<cd> cu0(nc), cv0(nc), cc(nc);
  for (size_t k = 0; k < nc; ++k) {
    cu0[k] = u0[k];
    cv0[k] = v0[k];
    cc[k] = cd(c[k], h * dc[k]);
  }
  std::vector<cd> F(2 * nc);
  init_equilibrium<cd>(*p, ops, cu0.data(), cv0.data(), f.data());
  for (int n = 0; n < nsteps; ++n) {
    step<cd>(*p, ops, f.data(), cc.data(), post.data(), fnew.data(), F.data(), n == 0);
    f.swap(fnew);
  }
  cd J = 0.0;
  for (size_t cell = 0; cell < nc; ++cell) {
    if (p->solid && p->solid[cell]) continue;
    cd u = 0.0;
    for (int i = 0; i < Q; ++i) u += f[(0 * Q + i) * nc + cell];
    cd dd = u - ut[cell];
    J += 0.5 * dd * dd + 0.5 * p->alpha * cc[cell] * cc[cell];
  }
  *J_re = J.real();
  *J_im = J.imag();
  return 0;
}

// Full gradient (gradientLattice) of J: E = g + alpha c on fluid nodes and
// 0 on solid nodes, from the adjoint seeded with dI0/dphi_u,i = u^N - u_t.
// Also returns J and its two parts.
int orc_cost_gradient(const OrcProblem* p, int nsteps, const double* u0,
                      const double* v0, const double* c, const double* ut,
                      double* grad, double* J, double* J_track, double* J_reg,
                      double* uN_out) {
  const size_t nc = size_t(p->nx) * p->ny;
  std::vector<double> uN(nc), vN(nc), seed(nc, 0.0);
  int rc = orc_forward(p, nsteps, u0, v0, c, uN.data(), vN.data(), nullptr,
                       nullptr, nullptr);
  if (rc) return rc;
  *J = orc_cost(p, uN.data(), ut, c, J_track, J_reg);
  for (size_t cell = 0; cell < nc; ++cell)
    if (!(p->solid && p->solid[cell])) seed[cell] = uN[cell] - ut[cell];
  rc = orc_adjoint(p, nsteps, u0, v0, c, seed.data(), nullptr, grad, nullptr,
                   nullptr);
  if (rc) return rc;
  for (size_t cell = 0; cell < nc; ++cell)
    grad[cell] = (p->solid && p->solid[cell]) ? 0.0 : grad[cell] + p->alpha * c[cell];
  if (uN_out) std::memcpy(uN_out, uN.data(), sizeof(double) * nc);
  return 0;
}

// Continuous-adjoint gradient: the forward trajectory, then the system of
// cadj_collide in reversed time from p = seed_u (equilibrium populations),
// q = 0, with streaming and bounce-back as the forward; reversed step k
// uses the forward state of step N-1-k.  g[cell] = tau sum_k q^k (the
// pre-collision q of each reversed step), the time integral of q in the
// gradient (DJRW) of a control entering Phi_v.
int orc_cadjoint(const OrcProblem* p, int nsteps, const double* u0, const double* v0,
                 const double* c, const double* seed_u, double* g) {
  Ops ops;
  if (!build_ops(*p, ops) || nsteps < 0 || nspec(*p) != 2) return -1;
  const size_t nc = size_t(p->nx) * p->ny;
  std::vector<double> f, traj;
  run_forward(*p, ops, nsteps, u0, v0, c, f, &traj);
  std::vector<double> d(2 * Q * nc, 0.0), post(2 * Q * nc), dnew(2 * Q * nc);
  for (size_t cell = 0; cell < nc; ++cell) {
    g[cell] = 0.0;
    if (p->solid && p->solid[cell]) continue;
    for (int i = 0; i < Q; ++i) d[(0 * Q + i) * nc + cell] = ops.u.weq[i] * seed_u[cell];
  }
  for (int k = 0; k < nsteps; ++k) {
    const double* fn = traj.data() + size_t(nsteps - 1 - k) * 2 * Q * nc;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x) {
        const int cell = y * p->nx + x;
        if (p->solid && p->solid[cell]) {
          for (int q = 0; q < 2 * Q; ++q) post[q * nc + cell] = 0.0;
          continue;
        }
        double fw[2 * Q], loc[2 * Q], out[2 * Q];
        for (int q = 0; q < 2 * Q; ++q) {
          fw[q] = fn[q * nc + cell];
          loc[q] = d[q * nc + cell];
        }
        double qv = 0.0;
        for (int i = 0; i < Q; ++i) qv += loc[Q + i];
        g[cell] += TAU * qv;
        cadj_collide(*p, ops, fw, loc, out);
        for (int q = 0; q < 2 * Q; ++q) post[q * nc + cell] = out[q];
      }
    stream_push(*p, ops, post.data(), dnew.data());
    d.swap(dnew);
  }
  return 0;
}

// Gradient step (Step 5): c <- clamp(c - zeta E, lo, hi); zeta <= 0 selects
// the heuristic zeta = min(1, 1/||E||_inf).  Returns the zeta used.
double orc_gd_step(int n, double* c, const double* E, double zeta, double lo,
                   double hi) {
  if (zeta <= 0.0) {
    double emax = 0.0;
    for (int k = 0; k < n; ++k) emax = std::fmax(emax, std::fabs(E[k]));
    zeta = emax > 0.0 ? std::fmin(1.0, 1.0 / emax) : 1.0;
  }
  for (int k = 0; k < n; ++k) {
    double x = c[k] - zeta * E[k];
    if (x < lo) x = lo;
    if (x > hi) x = hi;
    c[k] = x;
  }
  return zeta;
}

}  // extern "C"
