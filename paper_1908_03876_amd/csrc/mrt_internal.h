// Internal interface between the C-ABI runtime (mrt_abi.cpp) and the gfx950
// kernels (mrt_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mrt {

// Relaxation coefficients of one species, pre-scaled by the inverse squared
// row norms of M0 (M0^-1 = M0^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12,
// 1/4, 1/4), the rows of M0 being orthogonal).
template <typename T>
struct SpeciesCoef {
  T s1, s2;               // s1/36, s2/36       on (e, epsilon)
  T s3, s4;               // s3/12, s4/12       on (q_x, q_y)
  T s5, s6;               // s5/4,  s6/4        on (p_xx, p_xy)
  T k00, k01, k10, k11;   // K/6                on (j_x, j_y)
  T e_eq, eps_eq;         // m_eq = Theta * (1, e_eq, eps_eq, 0, ..., 0)
  T w_rest, w_axis, w_diag;  // phi_eq_i = w_i * Theta by velocity shell
};

// Per-step model coefficients (kernel argument, passed by value).
template <typename T>
struct ModelCoef {
  SpeciesCoef<T> u, v;   // forward relaxation
  SpeciesCoef<T> ut, vt; // adjoint relaxation: K transposed
  T b00, b01, b10, b11;  // chemotactic source a = u * B * j_v
  T r_u, a_uv, b_v;      // kinetics
  // third species (three-species problems only)
  SpeciesCoef<T> w, wt;
  T bw00, bw01, bw10, bw11;  // repulsive source a += u * Bw * j_w
  T a_w, b_w, s_w;           // Phi_w = a_w u - b_w w + s_w
};

struct Geometry {
  int nx, ny, pitch;
  int periodic;          // 1: periodic wrap; 0: walls at the lattice edge
  int masked;            // 1: solid nodes given by a mask (link mask in use)
  size_t plane;          // ny * pitch elements
  const uint16_t* link;  // link mask [ny][pitch] when masked, else null
  const uint32_t* wflag; // [ny][nsx]: 1 if a 64-node row segment touches a
                         // solid node (itself or a neighbour), when masked
  int nsx;               // 64-node segments per row, ceil(nx / 64)
};

// Link mask: bit 0 = node solid, bit i (1..8) = node x - e_i solid (wrapped
// when periodic; outside a non-periodic lattice is handled from the node
// coordinates, not by the mask).
void launch_build_link(const Geometry& g, int periodic, const uint8_t* mask,
                       uint16_t* link_out, uint32_t* wflag_out, hipStream_t s);

template <typename T>
struct FwdLaunch {
  const T* src;      // post-collision state of step n-1, or null (first)
  T* dst;            // post-collision state of step n (with wall slots)
  const T* u0;       // initial fields (first step only)
  const T* v0;
  const T* ctrl;     // control c(x)
  T* rec;            // record slot [3][plane] (u, j_vx, j_vy) or null
  int variant;       // scheme variant: 1 first-order source, 2 explicit,
                     // 3 implicit characteristic difference, 4 three species
  T* lag;            // variant 2: kinetics of the previous step [2][plane],
                     // overwritten with this step's
  const T* w0;       // variant 4: initial w (first step only; null = 0)
};

template <typename T>
void launch_forward_step(const Geometry& g, const ModelCoef<T>& m,
                         const FwdLaunch<T>& a, hipStream_t s);

// Terminal streaming: state (may be null), u^N, v^N (may be null).  With m
// given (implicit characteristic difference), Theta^N comes from the node
// solve with the control ctrl and the state is phi^N.
template <typename T>
void launch_finalize(const Geometry& g, const T* src, T* state, T* uN, T* vN,
                     hipStream_t s, const ModelCoef<T>* m = nullptr,
                     const T* ctrl = nullptr, bool three = false);

// Implicit characteristic difference: adjoint seeds of the sums G^N from
// (dJ/du^N, dJ/dv^N) (seed_v may be null), initialising the gradient
// accumulator with the control's share in v^N; and the tangent of Theta^N
// from that of G^N (fsrc: the forward's last post-collision state, dsrc:
// the tangent's).
template <typename T>
void launch_implicit_terminal(const Geometry& g, const ModelCoef<T>& m, const T* src,
                              const T* ctrl, const T* seed_u, const T* seed_v, T* out_u,
                              T* out_v, double* gacc, hipStream_t s);
template <typename T>
void launch_implicit_tlm_final(const Geometry& g, const ModelCoef<T>& m, const T* fsrc,
                               const T* dsrc, const T* ctrl, const T* dc, T* duN, T* dvN,
                               hipStream_t s);

template <typename T>
struct AdjLaunch {
  const T* src;      // adjoint state of step n+1, or null (terminal seed)
  T* dst;            // adjoint state of step n, or null (last step)
  const T* seed_u;   // terminal condition (first step only)
  const T* seed_v;   // may be null (= 0)
  const T* rec;      // record slot of step n
  double* g;         // gradient accumulator
  T* adj_u0;         // dJ/du0 (last step only, may be null)
  T* adj_v0;
  int first;         // 1: step N-1 (reads seeds, initialises g)
  int last;          // 1: step 0 and adj_u0/adj_v0 requested
  int variant;       // scheme variant (as FwdLaunch)
  T* mu;             // variant 2: adjoint of the stored kinetics [2][plane]
  int step0;         // 1: step 0
};

template <typename T>
void launch_adjoint_step(const Geometry& g, const ModelCoef<T>& m,
                         const AdjLaunch<T>& a, hipStream_t s);

// Coefficients of the continuous-adjoint system (p adjoint of u, q of v):
// advection chi (C grad v) . grad p = j_p^T M j_v and the cross-diffusion
// flux of q, a_q = u Bq j_p, with grad Theta = -K_Theta j / (tau d Cs^2).
template <typename T>
struct CadjCoef {
  T m00, m01, m10, m11;
  T q00, q01, q10, q11;
};

template <typename T>
struct CadjLaunch {
  const T* src;      // continuous-adjoint state of the previous reversed step, or null
  T* dst;            // state after this reversed step (with wall slots)
  const T* seed_u;   // p at s = 0 (first reversed step only)
  const T* rec;      // record slot of the forward step at this time
  double* g;         // time integral of q
  int first;         // 1: first reversed step (initialises g)
};

template <typename T>
void launch_cadj_step(const Geometry& g, const ModelCoef<T>& m, const CadjCoef<T>& cc,
                      const CadjLaunch<T>& a, hipStream_t s);

template <typename T>
struct TlmLaunch {
  const T* src;      // perturbation of step n-1 (post-collision), or null (n = 0)
  T* dst;            // perturbation after step n (with wall slots)
  const T* du0;      // initial perturbations (n = 0 only; null = 0)
  const T* dv0;
  const T* dc;       // control perturbation (null = 0)
  const T* rec;      // record slot of step n (forward u, j_vx, j_vy)
  int variant;       // scheme variant (as FwdLaunch)
  T* dlag;           // variant 2: perturbed kinetics of the previous step
                     // [2][plane]
};

template <typename T>
void launch_tlm_step(const Geometry& g, const ModelCoef<T>& m, const TlmLaunch<T>& a,
                     hipStream_t s);

// result[0] = sum over fluid nodes of x * y (double), result[4] = number of
// non-finite products.
template <typename T>
void launch_dot(const Geometry& g, const T* x, const T* y, double* partials, double* result,
                hipStream_t s);
// Up to four inner products <a_k, b_k> over the fluid nodes in one pass:
// result slots 0, 1, 2, 4 (k = 0..3), slot 3 > 0 if a product is not finite.
template <typename T>
struct DotPairs {
  const T* a[4];
  const T* b[4];
  int n;
};
template <typename T>
void launch_dots(const Geometry& g, const DotPairs<T>& d, double* partials, double* result,
                 hipStream_t s);
// y <- a x + b y on fluid nodes, 0 on solid nodes.
template <typename T>
void launch_axpby(const Geometry& g, const T* x, T* y, double a, double b, hipStream_t s);

// Deterministic two-pass reductions in double.
// Result slots (double): [0] sum 1/2 (uN-ut)^2, [1] sum alpha/2 c^2,
// [2] sum E^2, [3] max |E|, [4] count of non-finite values.
constexpr int kRedSlots = 5;
constexpr int kRedBlocks = 1024;

template <typename T>
void launch_cost_grad(const Geometry& g, const T* uN,
                      const T* ut, const T* ctrl, const double* gacc,
                      T* seed, T* grad, double alpha, double* partials,
                      double* result, hipStream_t s);

template <typename T>
void launch_gd_step(const Geometry& g, T* ctrl,
                    const T* grad, double zeta, double lo, double hi,
                    double* partials, double* result, hipStream_t s);

void launch_count_fluid(const Geometry& g, double* partials, double* result,
                        hipStream_t s);

// Cost and gradient reduction of launch_cost_grad without a tape: solid
// nodes from the caller's byte mask (null = none), the block partials and
// results in a device-resident static array of kNoallocScratchDoubles
// doubles (no allocation).  Writes host_out[0..4] = the reduced slots above
// and host_out[5] = the fluid node count, and synchronises the stream.
constexpr int kNoallocScratchDoubles = kRedBlocks * kRedSlots + 2 * kRedSlots;
constexpr size_t kNoallocMaxNodes = size_t(1) << 30;
template <typename T>
hipError_t launch_cost_grad_noalloc(const Geometry& g, const uint8_t* mask, const T* uN,
                                    const T* ut, const T* ctrl, const double* gacc, T* seed,
                                    T* grad, double alpha, double* host_out, hipStream_t s);

// Host helpers of the runtime (mrt_abi.cpp), shared with the batch runtime.
}  // namespace mrt

struct mrt_problem;
namespace mrt {
namespace host {
int validate(const mrt_problem* p);        // MRT_OK or MRT_EINVAL, sets the error
int set_error(int code, const char* msg);  // records a message, returns code
template <typename T>
ModelCoef<T> model_coef(const mrt_problem* p);
template <typename T>
CadjCoef<T> cadj_coef(const mrt_problem* p);
}  // namespace host
}  // namespace mrt
