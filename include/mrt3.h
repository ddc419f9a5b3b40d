/*
 * mrt3.h - C-ABI of the MI355X (gfx950) D3Q19 variant of the hot path: the
 * two-species chemotaxis control problem of mrt.h on a three-dimensional
 * lattice, with its exact discrete adjoint (AMRT) and tangent.
 *
 * Method: A. Belmiloudi, "Optimal Control for Chemotaxis Systems and
 * Adjoint-Based Optimization with Multiple-Relaxation-Time Lattice Boltzmann
 * Models", arXiv:1908.03876.  Section 3.1 develops the MRT scheme on D2Q9
 * and extends it to the DmQq lattices of its Remark, here D3Q19 with the
 * weights (sumWi3); Section 3.2.1 gives the adjoint algorithm.
 *
 * Problem solved (Section 1, (ReacDiff), two species, null-flux walls (E2)
 * as halfway bounce-back):
 *   du/dt - div(D_u grad u) = r_u u (1-u) - div(chi u C_chi grad v)
 *   dv/dt - div(D_v grad v) = a_uv u - b_v v + c(x)
 * with 3x3 tensors, the static control c(x) on v and the cost (classicJ)
 * J(c) = 1/2 sum (u^N - u_target)^2 + alpha/2 sum c^2 over fluid nodes.
 * Lattice units: h = tau = 1, Cs^2 = 1/3; first-order source term.
 *
 * Conventions (as mrt.h, whose return codes, mrt_last_error(), mrt_scalars,
 * mrt_tape_info and the mrt_timing_* calls this interface shares):
 *   - Array arguments are DEVICE pointers owned by the caller.
 *   - Fields are [nz][ny][pitch]: node (x, y, z) at (z*ny + y)*pitch + x;
 *     only x < nx is read or written.
 *   - Floating-point fields have the grid's dtype (MRT_F32 / MRT_F64),
 *     grad_accum is always double.
 *   - The distribution state is SoA: population i of species s (0 = u,
 *     1 = v) at node (x, y, z) is at ((s*19 + i)*nz*ny + z*ny + y)*pitch + x,
 *     with the velocity order e0 = 0; e1..e6 = +x, -x, +y, -y, +z, -z;
 *     e7..e10 = (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0); e11..e14 =
 *     (1,0,1), (-1,0,-1), (-1,0,1), (1,0,-1); e15..e18 = (0,1,1),
 *     (0,-1,-1), (0,1,-1), (0,-1,1) (links 2p+1 and 2p+2 are opposite).
 *   - The moment basis is orthogonal, in the order density, energy,
 *     energy square, j_x, q_x, j_y, q_y, j_z, q_z, then 3e_x^2 - |e|^2,
 *     its |e|^2 companion, e_y^2 - e_z^2, its |e|^2 companion, e_x e_y,
 *     e_y e_z, e_x e_z and the three third-order moments
 *     (e_y^2 - e_z^2) e_x, (e_z^2 - e_x^2) e_y, (e_x^2 - e_y^2) e_z (the
 *     span and order of Gram-Schmidt on the corresponding monomials).
 *   - Solid nodes (mask = 1) carry no populations; every output is 0 there.
 *   - Asynchronous calls enqueue on `stream` (a hipStream_t; NULL = the
 *     default stream); calls returning host scalars synchronise it.  On an
 *     error no work is enqueued, except MRT_EHIP and MRT_ENONFINITE.
 *   - One tape must not be used by two calls at the same time.
 */
#ifndef MRT3_H
#define MRT3_H

#include "mrt.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Lattice: nx, ny, nz in 1..4096, pitch >= nx, nz*ny*pitch < 2^31. */
typedef struct mrt3_grid {
  int32_t nx, ny, nz;
  int32_t pitch;       /* x stride of every field, in elements */
  int32_t periodic;    /* 1: periodic wrap; 0: outside the grid is a wall */
  int32_t dtype;       /* MRT_F32 or MRT_F64 */
  int32_t nsteps;      /* N >= 1 */
  int32_t reserved;    /* must be 0 */
  const uint8_t* mask; /* device [nz][ny][pitch], 1 = solid; NULL = none */
} mrt3_grid;

/* One species: self-diffusion tensor D (3x3 row-major, symmetric positive
 * definite), the equilibrium parameter d > 0 of (phieq) and the free rates
 * s[0..15] in (0, 2) on the density (no effect: conserved), energy, energy
 * square, q_x, q_y, q_z and the ten moments after the q's, in the order
 * above.  The 3x3 block K on (j_x, j_y, j_z) follows from
 * D = d Cs^2 tau (K^-1 - I/2). */
typedef struct mrt3_species {
  double D[9];
  double d;
  double s[16];
} mrt3_species;

typedef struct mrt3_problem {
  mrt3_grid grid;
  mrt3_species u, v;
  double chi;       /* chemotactic sensitivity */
  double Cchi[9];   /* 3x3 row-major shape of D_{u,1} = chi u Cchi */
  double r_u;       /* Phi_u = r_u u (1 - u) */
  double a_uv;      /* Phi_v = a_uv u - b_v v + c */
  double b_v;
  double alpha;     /* control penalty weight, >= 0 */
} mrt3_problem;

typedef struct mrt3_tape mrt3_tape;

/* Host-only check: MRT_EINVAL for a grid outside the limits above, an
 * unknown dtype, nsteps < 1, a D not symmetric positive definite, d <= 0, a
 * rate outside (0, 2), a non-finite coefficient or alpha < 0. */
int mrt3_validate(const mrt3_problem* p);

/* Host-only: device bytes of a tape (ckpt_every: 0 forward only, >= nsteps
 * store-all, else a checkpoint every ckpt_every steps). */
int mrt3_tape_bytes(const mrt3_problem* p, int32_t ckpt_every, size_t* bytes);

/* Device workspace: ping-pong states, the link words built from grid.mask,
 * reduction buffers and, for the adjoint, the tape: u and j_v of every node
 * and step of a segment (16 or 32 bytes per node and step), and the states
 * at the segment starts.  mem_budget > 0: MRT_ENOMEM above that many
 * bytes.  grid.mask is read here only. */
int mrt3_tape_create(const mrt3_problem* p, int32_t ckpt_every, size_t mem_budget,
                     mrt3_tape** out);
void mrt3_tape_destroy(mrt3_tape* t);
int mrt3_tape_query(const mrt3_tape* t, mrt_tape_info* info /* host */);

/* Forward MRT solve (eq:LBE with (S), (PhiS), the collision (MC) in moment
 * space, halfway bounce-back), N steps from the equilibrium of (u0, v0)
 * (phieq).  Writes u^N, v^N (may be NULL) and, if not NULL, the state
 * [2][19][nz][ny][pitch] after the last streaming.  Records the tape when
 * it was created for the adjoint.  Asynchronous. */
int mrt3_forward(const mrt3_problem* p, mrt3_tape* t, const void* u0, const void* v0,
                 const void* control, void* state, void* uN, void* vN, void* stream);

/* Adjoint sweep (CAE, AEDs, CAEL; streaming along -e_i backward in time) of
 * the last mrt3_forward on this tape from psi_u,i(T) = seed_u,
 * psi_v,i(T) = seed_v (NULL = 0).  u0, v0, control must be the buffers of
 * that forward call.  Overwrites grad_accum (double) with
 * sum_n tau sum_i w_i psi_v,i (gradientLattice) and, if not NULL, writes
 * dJ/du0, dJ/dv0.  MRT_ESTATE without an adjoint tape or a forward.
 * Asynchronous. */
int amrt3_adjoint(const mrt3_problem* p, mrt3_tape* t, const void* u0, const void* v0,
                  const void* control, const void* seed_u, const void* seed_v,
                  double* grad_accum, void* adj_u0, void* adj_v0, void* stream);

/* Tangent-linear sweep (sensitivity LBE, LIBEG-V) about the last forward:
 * (du^N, dv^N) for the perturbation (dc, du0, dv0) (each NULL = 0; duN or
 * dvN may be NULL, not both).  Asynchronous. */
int mrt3_tlm(const mrt3_problem* p, mrt3_tape* t, const void* u0, const void* v0,
             const void* control, const void* dc, const void* du0, const void* dv0,
             void* duN, void* dvN, void* stream);

/* Cost and gradient reduction (classicJ, gradientLattice) as cost_gradient
 * of mrt.h on the 3-D fields: phase 1 (grad_accum NULL) returns J and, if
 * seed_out is not NULL, writes the seed u^N - u_target; phase 2 also
 * writes grad_out = grad_accum + alpha c and the gradient norms.
 * Synchronises the stream; MRT_ENONFINITE on a NaN or Inf. */
int mrt3_cost_gradient(const mrt3_problem* p, mrt3_tape* t, const void* uN,
                       const void* u_target, const void* control, const double* grad_accum,
                       void* seed_out, void* grad_out, mrt_scalars* out /* host */,
                       void* stream);

/* Gradient step c <- clamp(c - zeta E, lo, hi) on fluid nodes (zeta <= 0:
 * min(1, 1/||E||_inf)).  With zeta_used (host) not NULL, synchronises and
 * returns the step taken. */
int mrt3_gd_step(const mrt3_problem* p, mrt3_tape* t, void* control, const void* grad,
                 double zeta, double lo, double hi, double* zeta_used, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MRT3_H */
