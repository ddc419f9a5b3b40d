/*
 * mrt.h - C-ABI of the MI355X (gfx950) hot path for adjoint-based optimal
 * control of a coupled anisotropic chemotaxis system with a two-species
 * (optionally three-species) D2Q9 multiple-relaxation-time lattice
 * Boltzmann model (MRT) and its adjoint (AMRT).
 *
 * Method: A. Belmiloudi, "Optimal Control for Chemotaxis Systems and
 * Adjoint-Based Optimization with Multiple-Relaxation-Time Lattice Boltzmann
 * Models", arXiv:1908.03876 (equation labels below are the paper's).
 *
 * Problem solved (Section 1, (ReacDiff) with two species u = cells,
 * v = chemical, null-flux walls (E2) as halfway bounce-back):
 *   du/dt - div(D_u grad u) = r_u u (1-u) - div(chi u C_chi grad v)
 *   dv/dt - div(D_v grad v) = a_uv u - b_v v + c(x)
 * with a static distributed control c(x) on the v equation, and the cost
 * (classicJ) J(c) = 1/2 sum (u(T) - u_target)^2 + alpha/2 sum c^2 over the
 * fluid nodes.  Lattice units: h = tau = 1, Cs^2 = 1/3 (Section 3.1).
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer unless marked "host".  The
 *     caller allocates and owns it; the library never frees it.
 *   - Fields are [ny][pitch] row-major, element (x, y) at y*pitch + x.
 *     Only x < nx is read or written.
 *   - Floating-point fields have the grid's dtype (MRT_F32: float,
 *     MRT_F64: double), except grad_accum, which is always double.
 *   - The distribution state is SoA: population i of species s (0 = u,
 *     1 = v, 2 = w with three species) of node (x, y) is at
 *     ((s*9 + i)*ny + y)*pitch + x, with the D2Q9
 *     velocity order e0 = 0, e1 = (1,0), e2 = (0,1), e3 = -e1, e4 = -e2,
 *     e5 = (1,1), e6 = (-1,1), e7 = -e5, e8 = -e6 (Remark on DmQq lattices).
 *   - Solid nodes (mask = 1) carry no populations: every output is 0 there.
 *   - Asynchronous calls enqueue work on `stream` (a hipStream_t; NULL is the
 *     default stream) and return at once.  Calls that return host scalars
 *     synchronise that stream.
 *   - Return codes: MRT_OK or a negative MRT_E*; mrt_last_error() gives a
 *     thread-local message.  On an error no work has been enqueued, except
 *     MRT_EHIP (a HIP call failed) and MRT_ENONFINITE (work done, result
 *     not finite).
 *   - Calls are re-entrant given distinct tapes; one tape must not be used
 *     by two calls at the same time.
 */
#ifndef MRT_H
#define MRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MRT_OK = 0,
  MRT_EINVAL = -1,     /* invalid argument or parameter set */
  MRT_ENOMEM = -2,     /* device allocation failed or over the budget */
  MRT_EHIP = -3,       /* a HIP runtime call failed */
  MRT_ENONFINITE = -4, /* a reduced scalar is NaN or Inf */
  MRT_ESTATE = -5      /* tape does not match the problem or call order */
};

enum { MRT_F32 = 0, MRT_F64 = 1 };

/* Lattice (Section 3.1: uniform grid of spacing h, time step tau = T/N,
 * DmQq velocity set). */
typedef struct mrt_grid {
  int32_t nx, ny;   /* nodes per axis, 1..32768 */
  int32_t pitch;    /* row stride of every field, in elements, >= nx */
  int32_t q;        /* velocity set size; must be 9 (D2Q9) */
  int32_t periodic; /* 1: periodic wrap; 0: outside the grid is a wall */
  int32_t dtype;    /* MRT_F32 or MRT_F64 */
  int32_t nsteps;   /* N time steps, >= 1 */
  int32_t reserved; /* must be 0 */
  const uint8_t* mask; /* device [ny][pitch], 1 = solid node; NULL = none */
} mrt_grid;

/* One species Theta (Section 3.1): self-diffusion tensor D_Theta, the
 * equilibrium parameter d_Theta of (phieq) and the free relaxation rates of
 * Pi_Theta = diag(Lambda1, Lambda2, Lambda3): s[0..2] on (rho, e, epsilon),
 * s[3] on q_x, s[4] on q_y, s[5] on p_xx, s[6] on p_xy.  The 2x2 block K
 * coupling j_x and j_y follows from D_Theta = d_Theta Cs^2 tau (K^-1 - I/2)
 * (end of the proof of Proposition 1). */
typedef struct mrt_species {
  double D[4];  /* row-major 2x2, symmetric positive definite */
  double d;     /* > 0 */
  double s[7];  /* each in (0, 2) */
} mrt_species;

/* The control problem.  Cross-diffusion of u by v is the chemotactic tensor
 * D_{u,1} = chi u Cchi (example (ARC)); D_{v,1} = 0. */
typedef struct mrt_problem {
  mrt_grid grid;
  mrt_species u, v;
  double chi;      /* chemotactic sensitivity */
  double Cchi[4];  /* row-major 2x2 shape of the chemotactic tensor */
  double r_u;      /* Phi_u = r_u u (1 - u) */
  double a_uv;     /* Phi_v = a_uv u - b_v v + c */
  double b_v;
  double alpha;    /* control penalty weight, >= 0 */
  /* Source term of the LBE (eq:LBEG): 0 or 1 = tau F_i (first order, the
   * default); 2 = tau F_i + (tau^2/2) dF_i/dt, i.e. kappa_t = 1 and
   * kappa_x = 0, with the time derivative taken by the explicit
   * characteristic difference (F_i(t) - F_i(t - tau)) / tau of the Remark
   * after (eq:LBEG) and F_i(-tau) = F_i(0).  Order 2 adds the previous
   * step's kinetics to the scheme's state (two planes, carried by the tape
   * and its checkpoints).  It is a two-step (Adams-Bashforth-like) rule:
   * stable for slow kinetics, unstable when tau dPhi/dTheta reaches -1.
   * The batched engine accepts order 0 or 1 only. */
  int32_t source_term;
  /* Species: 0 or 2 = u and v; 3 adds a repulsive chemical signal w (the
   * attraction-repulsion example (ARC)): Phi_w = a_w u - b_w w + s_w and a
   * second cross-diffusion of u, D_{u,2} = chi_w u C_w (chi_w < 0 repels),
   * whose gradient is read from the first moment of w as that of v.  The
   * state is then [3][9][ny][pitch]; the second-order source terms, the
   * continuous adjoint and the batched engine take two species only. */
  int32_t nspecies;
  mrt_species w;
  double chi_w;
  double Cw[4];      /* row-major 2x2 shape of the repulsive tensor */
  double a_w, b_w, s_w;
  const void* w0;    /* device [ny][pitch] initial w, grid dtype; NULL = 0 */
} mrt_problem;

/* Reduced scalars returned by cost_gradient (host struct). */
typedef struct mrt_scalars {
  double J;        /* J_track + J_reg */
  double J_track;  /* 1/2 sum_F (u^N - u_target)^2 */
  double J_reg;    /* alpha/2 sum_F c^2 */
  double grad_inf; /* ||E||_inf (phase 2 only, else 0) */
  double grad_l2;  /* ||E||_2   (phase 2 only, else 0) */
  int64_t n_fluid; /* number of fluid nodes */
} mrt_scalars;

/* Description of a tape (host struct). */
typedef struct mrt_tape_info {
  int32_t mode;        /* 0 forward only, 1 store-all, 2 checkpointed */
  int32_t ckpt_every;  /* segment length K in steps */
  int32_t n_segments;  /* ceil(N / K) */
  int32_t reserved;
  int64_t n_fluid;     /* fluid nodes */
  size_t device_bytes; /* device memory held by the tape */
} mrt_tape_info;

typedef struct mrt_tape mrt_tape;

/* Host-only check of a problem (no device call).  Returns MRT_EINVAL when
 * q != 9, nx or ny outside 1..32768, pitch < nx, nsteps < 1, dtype unknown,
 * a D not symmetric positive definite, d <= 0, a rate outside (0, 2), a
 * non-finite coefficient or alpha < 0 (Remark on the CFL-type condition of
 * the explicit scheme: the derived K must have eigenvalues in (0, 2)). */
int mrt_validate(const mrt_problem* p);

/* Host-only: device bytes a tape for `p` with segment length ckpt_every
 * would hold (ckpt_every: 0 forward only, >= nsteps store-all, else
 * checkpoints every ckpt_every steps). */
int mrt_tape_bytes(const mrt_problem* p, int32_t ckpt_every, size_t* bytes);

/* Create the device workspace of a problem: ping-pong distribution
 * buffers, the link mask built from grid.mask, reduction buffers and, for
 * the adjoint, the trajectory tape.  The forward records the quantities the
 * adjoint needs (u and the first moment j_v of every node and step, the
 * state trajectory being an input of the backward solve, Section 3); when
 * the whole record does not fit, states are checkpointed every ckpt_every
 * steps and segments are recomputed in the adjoint.  mem_budget > 0 makes
 * the call fail with MRT_ENOMEM if the tape would need more device bytes.
 * The library owns the tape's memory; grid.mask is read here only. */
int mrt_tape_create(const mrt_problem* p, int32_t ckpt_every,
                    size_t mem_budget, mrt_tape** out);
void mrt_tape_destroy(mrt_tape* t);
int mrt_tape_query(const mrt_tape* t, mrt_tape_info* info /* host */);

/* Forward MRT solve (eq:LBEG with the sources (S), (PhiS); collision (MC) in
 * moment space (MF); streaming with halfway bounce-back), N steps from the
 * equilibrium of (u0, v0) (phieq).  Writes u^N, v^N after the last
 * streaming and, if `state` is not NULL, the distribution state [2][9][ny]
 * [pitch].  u^N / v^N may be NULL.  Records the adjoint tape when the tape
 * was created for the adjoint.  Asynchronous. */
int mrt_forward(const mrt_problem* p, mrt_tape* t, const void* u0,
                const void* v0, const void* control, void* state, void* uN,
                void* vN, void* stream);

/* Adjoint MRT sweep (CAE, AEDs, RFS1; streaming along -e_i backward in time,
 * CAEL) of the last mrt_forward on this tape, from the terminal condition
 * psi_u,i(T) = seed_u, psi_v,i(T) = seed_v (seed_v NULL = 0), i.e. the
 * gradient of a terminal functional of u^N, v^N.  u0, v0, control must be
 * the same buffers (and contents) as in that forward call (they seed the
 * segment recomputation).  Writes grad_accum[ny][pitch] (double) =
 * sum_n tau sum_i w_i psi_v,i, the adjoint part of the gradient
 * (gradientLattice), overwriting it.  If adj_u0 / adj_v0 are not NULL they
 * receive dJ/du0 and dJ/dv0 (transpose of the equilibrium initialisation).
 * MRT_ESTATE if the tape has no adjoint record or no forward ran.
 * Asynchronous. */
int amrt_adjoint(const mrt_problem* p, mrt_tape* t, const void* u0,
                 const void* v0, const void* control, const void* seed_u,
                 const void* seed_v, double* grad_accum, void* adj_u0,
                 void* adj_v0, void* stream);

/* Cost and gradient reduction (classicJ, EJD-H terminal term, gradient
 * (gradientLattice)).  Phase 1 (grad_accum NULL): J, J_track, J_reg over the
 * fluid nodes and, if seed_out is not NULL, the adjoint seed
 * seed_out = u^N - u_target (0 on solids).  Phase 2 (grad_accum given): also
 * grad_out = grad_accum + alpha * control on fluid nodes (0 on solids) and
 * its norms.  Reductions are in double, deterministic (fixed order).
 * Synchronises `stream`; MRT_ENONFINITE if a scalar is NaN or Inf. */
int cost_gradient(const mrt_problem* p, mrt_tape* t, const void* uN,
                  const void* u_target, const void* control,
                  const double* grad_accum, void* seed_out, void* grad_out,
                  mrt_scalars* out /* host */, void* stream);

/* Allocation-free variant of cost_gradient, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * errors as cost_gradient without the tape: solid nodes come from
 * p->grid.mask directly (non-zero = solid; NULL = none) and the fluid count
 * is reduced in the same call.  The block partials live in a static device
 * array of about 41 KB that each device holds until the process ends; the
 * call allocates nothing and its results equal cost_gradient's bit for bit.
 * Maximum size: nx * ny <= 2^30 nodes (MRT_EINVAL beyond).  Calls that
 * overlap on one device share that array and race: serialise them (one
 * stream, or host-side ordering).  Synchronises `stream`. */
int cost_gradient_noalloc(const mrt_problem* p, const void* uN,
                          const void* u_target, const void* control,
                          const double* grad_accum, void* seed_out,
                          void* grad_out, mrt_scalars* out /* host */,
                          void* stream);

/* Gradient step (Section 2.4, Step 5): control <- clamp(control - zeta *
 * grad, lo, hi) on fluid nodes.  zeta <= 0 selects the heuristic step
 * zeta = min(1, 1/||grad||_inf) (Remark after Step 6), computed on the
 * device.  lo/hi = -/+INFINITY for no box constraint.  If zeta_used is not
 * NULL the stream is synchronised and the step used is returned there. */
int gd_step(const mrt_problem* p, mrt_tape* t, void* control,
            const void* grad, double zeta, double lo, double hi,
            double* zeta_used /* host, NULL ok */, void* stream);

/* Tangent-linear model (sensitivity LBE, LIBEG-V; Section 2.4 uses it in
 * the linearised line minimisation LMA): the derivative of (u^N, v^N) of the
 * last mrt_forward on this tape in the direction (dc, du0, dv0), each NULL =
 * 0.  It applies, step by step, the Jacobian of the collision at the
 * recorded forward state (the record (u, j_v) of every step, re-recorded
 * segment by segment from the checkpoints in checkpointed mode) followed by
 * the streaming with bounce-back, from the equilibrium of (du0, dv0).
 * u0, v0, control must be the buffers of that forward call.  Writes duN
 * and/or dvN [ny][pitch] (0 on solids).  Uses the tape's adjoint buffers:
 * do not overlap with amrt_adjoint on the same tape.  MRT_ESTATE if the
 * tape has no record or no forward ran.  Asynchronous. */
int mrt_tlm(const mrt_problem* p, mrt_tape* t, const void* u0, const void* v0,
            const void* control, const void* dc, const void* du0,
            const void* dv0, void* duN, void* dvN, void* stream);

/* Continuous-adjoint variant of the gradient (Section 3.2.2): the continuous
 * adjoint system (FVM-PF-Adj-K) of the two-species problem, reversed in
 * time s = T - t and solved by the same MRT scheme, with p (adjoint of u)
 * and q (adjoint of v):
 *   p_s = div(D_u grad p) + chi (Cchi grad v) . grad p + r_u (1 - 2u) p + a_uv q
 *   q_s = div(D_v grad q) - b_v q - div(chi u Cchi^T grad p)
 * from p = seed_u, q = 0, with the forward state of the last mrt_forward on
 * this tape (re-recorded per segment when checkpointed) and bounce-back
 * walls.  Writes grad_accum[ny][pitch] (double) = tau sum over the
 * reversed steps of q (0 on solids); cost_gradient phase 2 then adds
 * alpha * control, as after amrt_adjoint.  It approximates the exact
 * discrete gradient of amrt_adjoint to the discretisation error.  Uses the
 * tape's adjoint buffers.  Asynchronous. */
int mrt_cadjoint(const mrt_problem* p, mrt_tape* t, const void* u0,
                 const void* v0, const void* control, const void* seed_u,
                 double* grad_accum, void* stream);

/* out = sum over the fluid nodes of x * y, accumulated in double in a fixed
 * order (x, y: [ny][pitch] of the grid's dtype).  The inner product of
 * the line searches and conjugate-gradient rules of Section 2.4.
 * Synchronises `stream`; MRT_ENONFINITE if the result is not finite. */
int mrt_dot(const mrt_problem* p, mrt_tape* t, const void* x, const void* y,
            double* out /* host */, void* stream);

/* y <- a x + b y on the fluid nodes, 0 on the solid ones (search
 * directions and control updates of Section 2.4).  Asynchronous. */
int mrt_axpby(const mrt_problem* p, mrt_tape* t, const void* x, void* y,
              double a, double b, void* stream);

/* Linearised line minimisation (LMA, Section 2.4): the minimiser of the
 * quadratic model of the cost along a direction d,
 *   J(c - zeta d) ~ 1/2 |r - zeta P|^2 + alpha/2 |c - zeta d|^2,
 * i.e. zeta = (<r, P> + alpha <c, d>) / (<P, P> + alpha <d, d>), with
 * r = u^N - u_target (the seed of cost_gradient), P = F'(c) d the
 * tangent-linear response of u^N (mrt_tlm) and inner products over the fluid
 * nodes, accumulated in double in a fixed order.  For the gradient step,
 * d = grad and c <- c - zeta grad; along a search direction D stepped as
 * c + s D, s = -zeta.  zeta = 0 if the denominator is not positive.
 * Synchronises `stream`; MRT_ENONFINITE if a product is not finite. */
int mrt_lma_step(const mrt_problem* p, mrt_tape* t, const void* control,
                 const void* dir, const void* resid, const void* P,
                 double* zeta /* host */, void* stream);

/* Nonlinear conjugate-gradient direction (Section 2.4, Remark after Step 6,
 * item 2): D <- -G + beta D with beta by the Fletcher-Reeves, Polak-Ribiere
 * (clipped at 0), Hestenes-Stiefel (clipped at 0) or Dai-Yuan rule, from
 * the new gradient G, the previous gradient Gprev and direction D (in/out),
 * gg_old = <Gprev, Gprev> and dg_old = <D, Gprev> of the previous iteration.
 * A restart (D = -G) is taken at the first iteration, when
 * |<G, Gprev>| >= 0.2 <G, G> (Powell), or when the new D is not a descent
 * direction.  Returns <G, G>, beta, the restart flag and dg = <D, G> of the
 * new direction (the gg_old and dg_old of the next call).  Synchronises
 * `stream`. */
enum { MRT_CG_FR = 0, MRT_CG_PR = 1, MRT_CG_HS = 2, MRT_CG_DY = 3 };
typedef struct mrt_cg_info {
  double gg;       /* <G, G> */
  double beta;     /* the rule's value (0 at the first iteration); not
                      applied when restart is set */
  double dg;       /* <D, G> of the returned direction (< 0) */
  int32_t restart; /* 1 if D = -G was taken */
  int32_t reserved;
} mrt_cg_info;
int mrt_cg_direction(const mrt_problem* p, mrt_tape* t, int32_t rule,
                     int32_t first, const void* G, const void* Gprev, void* D,
                     double gg_old, double dg_old, mrt_cg_info* out /* host */,
                     void* stream);

/* Thread-local text of the last error. */
const char* mrt_last_error(void);

/* Kernel timing with HIP events recorded on the caller's stream around the
 * step loops.  kind: 0 forward steps, 1 adjoint steps, 2 recompute steps,
 * 3 tangent-linear steps, 4 continuous-adjoint steps.
 * mrt_timing_read synchronises on the recorded events and returns the
 * summed milliseconds and the number of kernel launches since the last
 * reset. */
int mrt_timing_enable(int32_t on);
int mrt_timing_reset(void);
int mrt_timing_read(int32_t kind, double* ms /* host */,
                    int64_t* launches /* host */);


/* Streaming probe, for measurement: out[w][i] = sum_r in[r][i] + w over
 * `reads` planes of in and `writes` planes of out, each [n] FP32, with the
 * non-temporal loads and stores of the step kernels, over 256-element
 * tiles taken in launch order (order = 0) or XCD-banded as in the
 * single-lattice step kernels (order = 1: XCD k takes a contiguous range).
 * It reproduces a step kernel's HBM access mix without its arithmetic, so
 * the better of the two orders' bandwidths is the practical ceiling for
 * that mix.  Built mixes (reads, writes): (19, 18), (19, 21), (23, 20)
 * (the D2Q9 forward without and with the record, and the AMRT step),
 * (39, 42), (44, 40) (the D3Q19 forward and AMRT step); others, another
 * order, a NULL buffer or a negative n, and n of 2^31 or more 256-element
 * tiles, return MRT_EINVAL (checked on the host; n = 0 launches nothing).
 * Caller-owned device buffers of reads * n and writes * n floats.
 * Asynchronous on `stream`. */
int mrt_stream_probe(int32_t reads, int32_t writes, int32_t order, const float* in, float* out,
                     int64_t n, void* stream);

/* ------------------------------------------------------------------------
 * Batched form: many independent control problems of uneven size advanced
 * together.  Each gradient iteration (forward, cost and seed, AMRT sweep,
 * gradient and norms, gradient step, for every instance; Section 3.2.1's
 * discrete optimisation loop) runs the forward pass and the adjoint pass as
 * one persistent launch each, with a grid barrier between time steps, and
 * can be captured once in a HIP graph and replayed.  Problems must be
 * periodic, unmasked and square with pitch == nx, and share dtype and
 * nsteps; chi, tensors, rates, reactions and alpha may differ.  The batch
 * owns every field of every instance (instance-major, [L][L] each).
 * ---------------------------------------------------------------------- */

typedef struct mrt_batch mrt_batch;

enum {
  MRT_FIELD_U0 = 0,
  MRT_FIELD_V0 = 1,
  MRT_FIELD_CONTROL = 2,
  MRT_FIELD_TARGET = 3,
  MRT_FIELD_UN = 4,
  MRT_FIELD_VN = 5,
  MRT_FIELD_GRAD = 6
};

/* Launch shape of the persistent kernels: tiles of tile_w x (256/tile_w)
 * nodes (tile_w 64, 128 or 256) and blocks_per_cu resident work-groups per
 * compute unit (1..max_blocks_per_cu, the occupancy limit, so that every
 * work-group of a persistent launch is resident). */
typedef struct mrt_batch_tiles {
  int32_t tile_w;
  int32_t blocks_per_cu;
  int32_t max_blocks_per_cu; /* output only */
  int32_t reserved;
  double ms_per_step;        /* output of mrt_batch_tune */
} mrt_batch_tiles;

/* ckpt_every: segment length of the checkpointed record (0 or >= nsteps:
 * record every step; < 0: forward solves only, mrt_batch_forward, no
 * adjoint buffers).  MRT_ENOMEM if mem_budget > 0 is exceeded. */
int mrt_batch_create(const mrt_problem* problems, int32_t count,
                     int32_t ckpt_every, size_t mem_budget, mrt_batch** out);
void mrt_batch_destroy(mrt_batch* b);

/* Device pointer of field `which` of instance k ([L][L], grid dtype). */
int mrt_batch_field(mrt_batch* b, int32_t k, int32_t which, void** ptr);

/* Device-to-device copy of field `which` of instance k from (to_batch = 1)
 * or to (to_batch = 0) the caller's buffer `data` ([L][L]).  Asynchronous. */
int mrt_batch_copy(mrt_batch* b, int32_t k, int32_t which, int32_t to_batch,
                   void* data, void* stream);

int mrt_batch_set_tiles(mrt_batch* b, const mrt_batch_tiles* tiles);
int mrt_batch_get_tiles(mrt_batch* b, mrt_batch_tiles* tiles /* host */);

/* Autotuner: times a `steps`-step forward pass for every tile width and
 * power-of-two residency (the fastest of three passes after a warm-up),
 * keeps the fastest shape and returns it.  Synchronises
 * `stream`; overwrites the forward work buffers (not the fields). */
int mrt_batch_tune(mrt_batch* b, int32_t steps, mrt_batch_tiles* best /* host */,
                   void* stream);

/* Limit of a grid-barrier wait (default 2 s).  A wait beyond it aborts the
 * persistent launch (it always terminates) and mrt_batch_scalars reports
 * MRT_EHIP.  Exists so that the failure path can be exercised. */
int mrt_batch_set_timeout(mrt_batch* b, double seconds);

/* One gradient iteration for every instance: controls are updated in place
 * with zeta (<= 0: per-instance min(1, 1/||E_k||_inf)).  use_graph = 1
 * captures the iteration in a HIP graph on first use (and after a change of
 * zeta or tiles) and replays it.  Asynchronous on `stream`. */
int mrt_batch_iteration(mrt_batch* b, double zeta, int32_t use_graph,
                        void* stream);

/* Per-instance scalars of the last iteration (out[count], host): J and its
 * parts at the control before the update, gradient norms, and the step
 * used (zeta_used[count], NULL ok).  Synchronises `stream`; MRT_EHIP if a
 * grid barrier timed out, MRT_ENONFINITE if a value is not finite. */
int mrt_batch_scalars(mrt_batch* b, mrt_scalars* out, double* zeta_used,
                      void* stream);

/* Forward solves only (no record, no adjoint) of every instance from its
 * current u0, v0, control: writes the MRT_FIELD_UN / MRT_FIELD_VN fields.
 * One persistent launch plus the terminal streaming.  Synchronises
 * `stream`; MRT_EHIP if a grid barrier timed out (the outputs are then not
 * valid). */
int mrt_batch_forward(mrt_batch* b, void* stream);

/* ------------------------------------------------------------------------
 * Convolutional surrogate of the control-to-state map c -> u(T) - u_base:
 * four periodic 3x3 convolution layers (1 -> 32 -> 32 -> 32 -> 1 channels,
 * tanh between them), BF16 weights with FP32 accumulation and FP32 master
 * weights trained with Adam.  A layer computes z = oscale (W * (iscale x)
 * + b); the first layer uses iscale = in_scale, the last oscale = out_scale.
 * Fields are float [B][H][W] (periodic).  It proposes warm starts and step
 * sizes for the optimisation loop; MRT solves verify what it proposes.
 * ---------------------------------------------------------------------- */

typedef struct mrt_srg mrt_srg;

/* Work buffers hold max_batch * max_h * max_w pixels (at most 2^28, else
 * MRT_EINVAL); any call with B * H * W within that (H, W >= 3, W <= 2^24)
 * is accepted. */
int mrt_srg_create(int32_t channels /* 32 */, int32_t max_batch, int32_t max_h,
                   int32_t max_w, float in_scale, float out_scale, mrt_srg** out);
void mrt_srg_destroy(mrt_srg* s);

/* Device pointer and element count of a parameter of layer 0..3: kind 0
 * FP32 master weights [cout][cin][3][3], 1 biases [cout], 2 weight
 * gradients, 3 bias gradients (of the last backward / training step). */
int mrt_srg_param(mrt_srg* s, int32_t layer, int32_t kind, void** ptr,
                  int64_t* count /* host, NULL ok */);

/* Device-to-device copy of a parameter (kinds as above) from (to_srg = 1)
 * or to (to_srg = 0) the caller's float buffer.  Asynchronous. */
int mrt_srg_copy_param(mrt_srg* s, int32_t layer, int32_t kind, int32_t to_srg,
                       void* data, void* stream);

/* After writing the FP32 masters: refresh the BF16 copies and reset the
 * Adam moments.  Asynchronous. */
int mrt_srg_sync(mrt_srg* s, void* stream);

/* y = surrogate(x) for B fields of H x W.  Asynchronous. */
int mrt_srg_forward(mrt_srg* s, const float* x, float* y, int32_t B, int32_t H,
                    int32_t W, void* stream);

/* Backward of the last mrt_srg_forward on x from dy = dL/dy: dx = dL/dx
 * (NULL: not computed) and, if weight_grads, the parameter gradients.
 * Asynchronous. */
int mrt_srg_backward(mrt_srg* s, const float* x, const float* dy, float* dx,
                     int32_t weight_grads, int32_t B, int32_t H, int32_t W,
                     void* stream);

/* Mean squared error of surrogate(x) against target over the interior
 * (border pixels excluded).  Synchronises `stream`. */
int mrt_srg_loss(mrt_srg* s, const float* x, const float* target, int32_t B,
                 int32_t H, int32_t W, int32_t border, double* loss /* host */,
                 void* stream);

/* One Adam step (b1 = 0.9, b2 = 0.999) on the interior MSE of a batch.
 * loss (host) NULL: asynchronous; else synchronises and returns the loss
 * before the step. */
int mrt_srg_train_step(mrt_srg* s, const float* x, const float* target,
                       int32_t B, int32_t H, int32_t W, int32_t border,
                       float lr, double* loss /* host, NULL ok */, void* stream);

/* Periodic crops: out[i] = h x w window at (oy[i], ox[i]) of the L x L field
 * src[idx[i]] (idx, oy, ox: device int32 arrays of n entries), minus the
 * same window of the L x L field `sub` when sub is not NULL (training
 * targets u(T) - u_base).  Asynchronous. */
int mrt_srg_gather(const float* src, int32_t L, const int32_t* idx,
                   const int32_t* oy, const int32_t* ox, const float* sub,
                   float* out, int32_t n, int32_t h, int32_t w, void* stream);

/* Surrogate cost of B <= 32 candidate controls x_b [B][H][W] of one control
 * problem (classicJ with u(T) replaced by u_base + surrogate(x_b)):
 *   J_b = 1/2 sum (u_base + S(x_b) - u_target)^2 + alpha/2 sum x_b^2,
 * u_base and u_target [H][W], sums in double.  J (host, B entries) NULL:
 * asynchronous, else synchronises and fills it.  dx (NULL: not computed)
 * receives dJ_b/dx_b = S'(x_b)^T (u_base + S(x_b) - u_target) + alpha x_b.
 * MRT_ENONFINITE if a J_b is not finite. */
int mrt_srg_objective(mrt_srg* s, const float* x, const float* u_base,
                      const float* u_target, double alpha, int32_t B, int32_t H,
                      int32_t W, double* J /* host, NULL ok */, float* dx,
                      void* stream);

/* Surrogate-scored step sizes of a gradient step (Section 2.4: the step
 * zeta_k of c - zeta E; the surrogate stands in for the exact line
 * minimisation (LM)): J[k] = the surrogate cost above of c - lambdas[k] E
 * for k < n <= 32 (lambdas and J on the host; n * H * W within the
 * surrogate's work buffers).  Synchronises the stream. */
int mrt_srg_score_steps(mrt_srg* s, const float* c, const float* E,
                        const double* lambdas /* host */, int32_t n,
                        const float* u_base, const float* u_target, double alpha,
                        int32_t H, int32_t W, double* J /* host */, void* stream);

/* Warm start of the control: `iters` Adam steps (b1 = 0.9, b2 = 0.999,
 * eps = 1e-8, learning rate lr) on the surrogate cost of the single field
 * c [H][W] (H * W <= max_h * max_w), starting from the values c holds.
 * Asynchronous; c is updated in place. */
int mrt_srg_warm_start(mrt_srg* s, const float* u_base, const float* u_target,
                       double alpha, int32_t H, int32_t W, int32_t iters, float lr,
                       float* c, void* stream);

/* Warm start of the control by steepest descent on the surrogate cost with
 * Barzilai-Borwein steps: c <- c - eta_k g_k with g_k the input gradient of
 * the cost above at c, eta_0 = step0 / RMS(g_0) (a first move of RMS size
 * step0) and eta_k = <s, s>/<s, y> for s = c_k - c_{k-1}, y = g_k - g_{k-1}
 * when that is positive (else the previous step), for `iters` iterations;
 * c ends as the iterate of least surrogate cost.  One step length for the
 * whole field, computed on the device.  Asynchronous; c is updated in
 * place; H * W <= max_h * max_w. */
int mrt_srg_warm_start_bb(mrt_srg* s, const float* u_base, const float* u_target,
                          double alpha, int32_t H, int32_t W, int32_t iters,
                          float step0, float* c, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MRT_H */
