// C-ABI runtime of the MRT/AMRT hot path: parameter validation, the
// device workspace ("tape"), the forward / adjoint step loops with the
// checkpoint schedule, reductions and the gradient step.  See include/mrt.h
// for the contract of every entry point.
#include "mrt.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mrt_host.h"
#include "mrt_internal.h"
#include "probe_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                        \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return fail(MRT_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));  \
  } while (0)

constexpr double kCs2 = 1.0 / 3.0;  // 3 Cs^2 = c^2, c = 1
constexpr double kTau = 1.0;

bool finite_all(const double* a, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// K = (D/(d Cs^2 tau) + I/2)^-1, from D = d Cs^2 tau (K^-1 - I/2).
void k_block(const mrt_species& s, double K[4]) {
  const double f = 1.0 / (s.d * kCs2 * kTau);
  const double a = s.D[0] * f + 0.5, b = s.D[1] * f;
  const double c = s.D[2] * f, e = s.D[3] * f + 0.5;
  const double det = a * e - b * c;
  K[0] = e / det;
  K[1] = -b / det;
  K[2] = -c / det;
  K[3] = a / det;
}

int check_species(const mrt_species& s, const char* name) {
  if (!finite_all(s.D, 4) || !std::isfinite(s.d) || !finite_all(s.s, 7))
    return fail(MRT_EINVAL, "species %s: non-finite coefficient", name);
  const double scale = std::max({std::fabs(s.D[0]), std::fabs(s.D[3]), 1e-300});
  if (std::fabs(s.D[1] - s.D[2]) > 1e-12 * scale)
    return fail(MRT_EINVAL, "species %s: D must be symmetric", name);
  if (!(s.D[0] > 0.0) || !(s.D[0] * s.D[3] - s.D[1] * s.D[2] > 0.0))
    return fail(MRT_EINVAL, "species %s: D must be positive definite", name);
  if (!(s.d > 0.0)) return fail(MRT_EINVAL, "species %s: d must be > 0", name);
  for (int j = 0; j < 7; ++j)
    if (!(s.s[j] > 0.0 && s.s[j] < 2.0))
      return fail(MRT_EINVAL, "species %s: rate s%d = %g outside (0, 2)", name,
                  j, s.s[j]);
  // eigenvalues of the symmetric K lie in (0, 2) for SPD D; checked anyway
  double K[4];
  k_block(s, K);
  const double tr = K[0] + K[3], det = K[0] * K[3] - K[1] * K[2];
  const double disc = std::sqrt(std::max(0.0, 0.25 * tr * tr - det));
  const double lmin = 0.5 * tr - disc, lmax = 0.5 * tr + disc;
  if (!(lmin > 0.0 && lmax < 2.0))
    return fail(MRT_EINVAL, "species %s: K eigenvalues (%g, %g) outside (0, 2)",
                name, lmin, lmax);
  return MRT_OK;
}

int validate(const mrt_problem* p) {
  if (!p) return fail(MRT_EINVAL, "problem is NULL");
  const mrt_grid& g = p->grid;
  if (g.q != 9) return fail(MRT_EINVAL, "q = %d: only D2Q9 (q = 9)", g.q);
  if (g.nx < 1 || g.ny < 1 || g.nx > 32768 || g.ny > 32768)
    return fail(MRT_EINVAL, "grid %d x %d outside 1..32768", g.nx, g.ny);
  if (g.pitch < g.nx) return fail(MRT_EINVAL, "pitch %d < nx %d", g.pitch, g.nx);
  if (g.nsteps < 1) return fail(MRT_EINVAL, "nsteps %d < 1", g.nsteps);
  if (g.dtype != MRT_F32 && g.dtype != MRT_F64)
    return fail(MRT_EINVAL, "unknown dtype %d", g.dtype);
  if (g.periodic != 0 && g.periodic != 1)
    return fail(MRT_EINVAL, "periodic must be 0 or 1");
  if (g.reserved != 0) return fail(MRT_EINVAL, "grid.reserved must be 0");
  int rc = check_species(p->u, "u");
  if (rc) return rc;
  rc = check_species(p->v, "v");
  if (rc) return rc;
  const double sc[8] = {p->chi, p->Cchi[0], p->Cchi[1], p->Cchi[2],
                        p->Cchi[3], p->r_u, p->a_uv, p->b_v};
  if (!finite_all(sc, 8) || !std::isfinite(p->alpha))
    return fail(MRT_EINVAL, "non-finite model coefficient");
  if (p->alpha < 0.0) return fail(MRT_EINVAL, "alpha < 0");
  if (p->source_term < 0 || p->source_term > 3)
    return fail(MRT_EINVAL, "source_term %d: must be 0, 1, 2 or 3", p->source_term);
  if (p->source_term == 3 && !(0.5 * p->r_u < 1.0 && 0.5 * p->b_v > -1.0))
    return fail(MRT_EINVAL,
                "implicit source term needs tau r_u / 2 < 1 and tau b_v / 2 > -1 "
                "(a solvable node equation)");
  if (p->nspecies != 0 && p->nspecies != 2 && p->nspecies != 3)
    return fail(MRT_EINVAL, "nspecies %d: must be 0, 2 or 3", p->nspecies);
  if (p->nspecies == 3) {
    if (p->source_term > 1)
      return fail(MRT_EINVAL, "three species take the first-order source term only");
    rc = check_species(p->w, "w");
    if (rc) return rc;
    const double wc[8] = {p->chi_w, p->Cw[0], p->Cw[1], p->Cw[2], p->Cw[3],
                          p->a_w, p->b_w, p->s_w};
    if (!finite_all(wc, 8)) return fail(MRT_EINVAL, "non-finite coefficient of w");
  }
  return MRT_OK;
}

template <typename T>
mrt::SpeciesCoef<T> species_coef(const mrt_species& s, bool transpose_k) {
  double K[4];
  k_block(s, K);
  if (transpose_k) std::swap(K[1], K[2]);
  mrt::SpeciesCoef<T> c;
  c.s1 = T(s.s[1] / 36.0);
  c.s2 = T(s.s[2] / 36.0);
  c.s3 = T(s.s[3] / 12.0);
  c.s4 = T(s.s[4] / 12.0);
  c.s5 = T(s.s[5] / 4.0);
  c.s6 = T(s.s[6] / 4.0);
  c.k00 = T(K[0] / 6.0);
  c.k01 = T(K[1] / 6.0);
  c.k10 = T(K[2] / 6.0);
  c.k11 = T(K[3] / 6.0);
  // m_eq (before (BC11)) with B = d Cs^2 Theta I: e = (2d - 4) Theta,
  // epsilon = (3 - 2d) Theta
  c.e_eq = T(2.0 * s.d - 4.0);
  c.eps_eq = T(3.0 - 2.0 * s.d);
  // phi_eq = M0^-1 m_eq by shell: rest 4(2-d)/9, axis (1+d)/18,
  // diagonal (2d-1)/36
  c.w_rest = T(4.0 * (2.0 - s.d) / 9.0);
  c.w_axis = T((1.0 + s.d) / 18.0);
  c.w_diag = T((2.0 * s.d - 1.0) / 36.0);
  return c;
}

template <typename T>
mrt::ModelCoef<T> model_coef(const mrt_problem* p) {
  mrt::ModelCoef<T> m{};
  m.u = species_coef<T>(p->u, false);
  m.v = species_coef<T>(p->v, false);
  m.ut = species_coef<T>(p->u, true);
  m.vt = species_coef<T>(p->v, true);
  // A_u1 grad v = (K_u chi u Cchi / tau) (-K_v j_v / (tau d_v Cs^2))
  //             = u * B * j_v
  double Ku[4], Kv[4], KC[4], B[4];
  k_block(p->u, Ku);
  k_block(p->v, Kv);
  KC[0] = Ku[0] * p->Cchi[0] + Ku[1] * p->Cchi[2];
  KC[1] = Ku[0] * p->Cchi[1] + Ku[1] * p->Cchi[3];
  KC[2] = Ku[2] * p->Cchi[0] + Ku[3] * p->Cchi[2];
  KC[3] = Ku[2] * p->Cchi[1] + Ku[3] * p->Cchi[3];
  const double f = -p->chi / (kTau * kTau * p->v.d * kCs2);
  B[0] = f * (KC[0] * Kv[0] + KC[1] * Kv[2]);
  B[1] = f * (KC[0] * Kv[1] + KC[1] * Kv[3]);
  B[2] = f * (KC[2] * Kv[0] + KC[3] * Kv[2]);
  B[3] = f * (KC[2] * Kv[1] + KC[3] * Kv[3]);
  m.b00 = T(B[0]);
  m.b01 = T(B[1]);
  m.b10 = T(B[2]);
  m.b11 = T(B[3]);
  m.r_u = T(p->r_u);
  m.a_uv = T(p->a_uv);
  m.b_v = T(p->b_v);
  if (p->nspecies == 3) {
    // A_u2 grad w = (K_u chi_w u C_w / tau) (-K_w j_w / (tau d_w Cs^2))
    //             = u * Bw * j_w
    double Kw[4], KW[4], Bw[4];
    k_block(p->w, Kw);
    KW[0] = Ku[0] * p->Cw[0] + Ku[1] * p->Cw[2];
    KW[1] = Ku[0] * p->Cw[1] + Ku[1] * p->Cw[3];
    KW[2] = Ku[2] * p->Cw[0] + Ku[3] * p->Cw[2];
    KW[3] = Ku[2] * p->Cw[1] + Ku[3] * p->Cw[3];
    const double fw = -p->chi_w / (kTau * kTau * p->w.d * kCs2);
    Bw[0] = fw * (KW[0] * Kw[0] + KW[1] * Kw[2]);
    Bw[1] = fw * (KW[0] * Kw[1] + KW[1] * Kw[3]);
    Bw[2] = fw * (KW[2] * Kw[0] + KW[3] * Kw[2]);
    Bw[3] = fw * (KW[2] * Kw[1] + KW[3] * Kw[3]);
    m.w = species_coef<T>(p->w, false);
    m.wt = species_coef<T>(p->w, true);
    m.bw00 = T(Bw[0]);
    m.bw01 = T(Bw[1]);
    m.bw10 = T(Bw[2]);
    m.bw11 = T(Bw[3]);
    m.a_w = T(p->a_w);
    m.b_w = T(p->b_w);
    m.s_w = T(p->s_w);
  }
  return m;
}

// ---------------------------------------------------------------- timing

struct TimedSpan {
  int kind;
  hipEvent_t a, b;
  int64_t launches;
};

struct Timing {
  std::mutex mu;
  bool on = false;
  std::vector<TimedSpan> pending;
  double ms[5] = {0, 0, 0, 0, 0};
  int64_t launches[5] = {0, 0, 0, 0, 0};
};

Timing& timing() {
  static Timing t;
  return t;
}

struct SpanGuard {
  bool active = false;
  TimedSpan span{};
  hipStream_t s;
  SpanGuard(int kind, hipStream_t st) : s(st) {
    Timing& t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    if (!t.on) return;
    span.kind = kind;
    if (hipEventCreate(&span.a) != hipSuccess) return;
    if (hipEventCreate(&span.b) != hipSuccess) {
      (void)hipEventDestroy(span.a);
      return;
    }
    (void)hipEventRecord(span.a, s);
    active = true;
  }
  void count() { ++span.launches; }
  ~SpanGuard() {
    if (!active) return;
    (void)hipEventRecord(span.b, s);
    Timing& t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    t.pending.push_back(span);
  }
};

}  // namespace

namespace mrt {
namespace host {
int validate(const mrt_problem* p) { return ::validate(p); }
int set_error(int code, const char* msg) { return fail(code, "%s", msg); }
int failf(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
void* span_begin(int kind, hipStream_t s) {
  SpanGuard* g = new SpanGuard(kind, s);
  if (!g->active) {
    delete g;
    return nullptr;
  }
  return g;
}
void span_end(void* span, int64_t launches) {
  if (!span) return;
  SpanGuard* g = static_cast<SpanGuard*>(span);
  g->span.launches = launches;
  delete g;
}
template <typename T>
ModelCoef<T> model_coef(const mrt_problem* p) {
  return ::model_coef<T>(p);
}
template <typename T>
CadjCoef<T> cadj_coef(const mrt_problem* p) {
  // grad Theta = G_Theta j with G_Theta = -K_Theta / (tau d_Theta Cs^2)
  double Ku[4], Kv[4], Gu[4], Gv[4];
  k_block(p->u, Ku);
  k_block(p->v, Kv);
  for (int k = 0; k < 4; ++k) {
    Gu[k] = -Ku[k] / (kTau * p->u.d * kCs2);
    Gv[k] = -Kv[k] / (kTau * p->v.d * kCs2);
  }
  auto mul = [](const double* a, const double* b, double* c) {
    c[0] = a[0] * b[0] + a[1] * b[2];
    c[1] = a[0] * b[1] + a[1] * b[3];
    c[2] = a[2] * b[0] + a[3] * b[2];
    c[3] = a[2] * b[1] + a[3] * b[3];
  };
  const double chiC[4] = {p->chi * p->Cchi[0], p->chi * p->Cchi[1], p->chi * p->Cchi[2],
                          p->chi * p->Cchi[3]};
  const double GuT[4] = {Gu[0], Gu[2], Gu[1], Gu[3]};
  const double chiCT[4] = {chiC[0], chiC[2], chiC[1], chiC[3]};
  double t[4], M[4], Bq[4];
  mul(GuT, chiC, t);  // M = G_u^T (chi C) G_v
  mul(t, Gv, M);
  mul(Kv, chiCT, t);  // Bq = K_v (chi C^T) G_u / tau
  mul(t, Gu, Bq);
  CadjCoef<T> c;
  c.m00 = T(M[0]);
  c.m01 = T(M[1]);
  c.m10 = T(M[2]);
  c.m11 = T(M[3]);
  c.q00 = T(Bq[0] / kTau);
  c.q01 = T(Bq[1] / kTau);
  c.q10 = T(Bq[2] / kTau);
  c.q11 = T(Bq[3] / kTau);
  return c;
}
template CadjCoef<float> cadj_coef<float>(const mrt_problem*);
template CadjCoef<double> cadj_coef<double>(const mrt_problem*);
template ModelCoef<float> model_coef<float>(const mrt_problem*);
template ModelCoef<double> model_coef<double>(const mrt_problem*);
}  // namespace host
}  // namespace mrt

// ------------------------------------------------------------------ tape

struct mrt_tape {
  int nx, ny, pitch, nsteps, dtype, periodic, masked, device;
  int mode, K, nseg;
  int ns;                   // species: 2 or 3
  int so2;                  // explicit second-order source term (source_term 2)
  int impl;                 // implicit second-order source term (source_term 3)
  size_t plane, elem, state_bytes, rec_slot_bytes, total_bytes;
  void* buf[2] = {nullptr, nullptr};
  void* abuf[2] = {nullptr, nullptr};
  std::vector<void*> ckpt;  // ckpt[s] (s >= 1): post-collision state of step sK-1
  // so2: kinetics of the previous step [2][plane] (forward), its adjoint or
  // its perturbation (adjoint and tangent sweeps), and per checkpoint the
  // kinetics stored by step sK-1
  void* lag = nullptr;
  void* alag = nullptr;
  std::vector<void*> ckpt_lag;
  // impl: adjoint seeds of the last state's sums [2][plane]
  void* tseed = nullptr;
  void* rec = nullptr;      // record slots [K][3][plane]
  uint16_t* link = nullptr;
  uint32_t* wflag = nullptr;
  double* partials = nullptr;
  double* result = nullptr;
  double* host = nullptr;   // pinned
  int64_t n_fluid = 0;
  // last forward
  bool fwd_done = false;
  int rec_seg = -1;         // segment whose (u, j_v) record the slots hold
  const void* f_u0 = nullptr;
  const void* f_v0 = nullptr;
  const void* f_ctrl = nullptr;
  std::vector<void*> allocs;
};

namespace {

size_t elem_size(int dtype) { return dtype == MRT_F64 ? 8 : 4; }

struct Layout {
  int mode, K, nseg;
  size_t plane, elem, state_bytes, rec_slot_bytes, lag_bytes, tseed_bytes, total;
};

Layout plan(const mrt_problem* p, int ckpt_every) {
  Layout L{};
  const mrt_grid& g = p->grid;
  L.plane = size_t(g.ny) * size_t(g.pitch);
  L.elem = elem_size(g.dtype);
  const int ns = p->nspecies == 3 ? 3 : 2;
  L.state_bytes = size_t(9 * ns) * L.plane * L.elem;
  L.rec_slot_bytes = size_t(ns == 3 ? 5 : 3) * L.plane * L.elem;
  L.lag_bytes = p->source_term == 2 ? 2 * L.plane * L.elem : 0;
  L.tseed_bytes = p->source_term == 3 ? 2 * L.plane * L.elem : 0;
  if (ckpt_every <= 0) {
    L.mode = 0;
    L.K = g.nsteps;
    L.nseg = 1;
  } else if (ckpt_every >= g.nsteps) {
    L.mode = 1;
    L.K = g.nsteps;
    L.nseg = 1;
  } else {
    L.mode = 2;
    L.K = ckpt_every;
    L.nseg = (g.nsteps + ckpt_every - 1) / ckpt_every;
  }
  const bool masked = g.mask != nullptr;
  size_t t = 2 * L.state_bytes + L.lag_bytes;  // forward ping-pong, lag
  if (masked)
    t += L.plane * sizeof(uint16_t) +
         size_t(g.ny) * ((g.nx + 63) / 64) * sizeof(uint32_t);
  t += (size_t(mrt::kRedBlocks) * mrt::kRedSlots + 16) * sizeof(double);
  if (L.mode > 0) {
    t += 2 * L.state_bytes + L.lag_bytes + L.tseed_bytes;  // adjoint ping-pong, lag, seeds
    t += size_t(L.nseg - 1) * (L.state_bytes + L.lag_bytes);  // checkpoints
    t += size_t(L.K) * L.rec_slot_bytes;              // record slots
  }
  L.total = t;
  return L;
}

int check_tape(const mrt_problem* p, const mrt_tape* t) {
  if (!t) return fail(MRT_EINVAL, "tape is NULL");
  const mrt_grid& g = p->grid;
  const int masked = g.mask != nullptr ? 1 : 0;
  if (g.nx != t->nx || g.ny != t->ny || g.pitch != t->pitch ||
      g.nsteps != t->nsteps || g.dtype != t->dtype ||
      g.periodic != t->periodic || masked != t->masked)
    return fail(MRT_ESTATE, "tape was created for another grid");
  if ((p->source_term == 2 ? 1 : 0) != t->so2 || (p->source_term == 3 ? 1 : 0) != t->impl)
    return fail(MRT_ESTATE, "tape was created for another source term");
  if ((p->nspecies == 3 ? 3 : 2) != t->ns)
    return fail(MRT_ESTATE, "tape was created for another number of species");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != t->device)
    return fail(MRT_ESTATE, "tape belongs to device %d, current is %d",
                t->device, dev);
  return MRT_OK;
}

mrt::Geometry geometry(const mrt_tape* t) {
  mrt::Geometry g;
  g.nx = t->nx;
  g.ny = t->ny;
  g.pitch = t->pitch;
  g.periodic = t->periodic;
  g.masked = t->masked;
  g.plane = t->plane;
  g.link = t->masked ? t->link : nullptr;
  g.wflag = t->masked ? t->wflag : nullptr;
  g.nsx = (t->nx + 63) / 64;
  return g;
}

template <typename T>
T* slot(const mrt_tape* t, int k) {
  return reinterpret_cast<T*>(static_cast<char*>(t->rec) +
                              size_t(k) * t->rec_slot_bytes);
}

int last_launch_error() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(MRT_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
  return MRT_OK;
}

// Forward steps [n0, n1) starting from `src` (null = equilibrium of u0, v0).
// The output of step n goes to ckpt[(n+1)/K] when that step closes a
// segment (checkpointed mode, forward pass), else to a ping-pong buffer.
// Returns the buffer holding the last written state through *last.
//
// Second-order source: the kinetics of the previous step live in t->lag;
// a step that closes a segment also saves them beside its checkpoint, and
// a recomputation that starts from checkpoint `seg` (restore_lag) first
// restores them.
template <typename T>
int run_forward_steps(mrt_tape* t, const mrt::ModelCoef<T>& m,
                      const mrt::Geometry& g, int n0, int n1, const T* src,
                      const T* u0, const T* v0, const T* ctrl, bool record,
                      bool write_ckpt, int kind, hipStream_t s,
                      const T** last, bool restore_lag = false, const T* w0 = nullptr) {
  SpanGuard span(kind, s);
  const int seg = n0 / t->K;
  if (t->so2 && restore_lag && n0 > 0)
    HIP_TRY(hipMemcpyAsync(t->lag, t->ckpt_lag[seg], 2 * t->plane * t->elem,
                           hipMemcpyDeviceToDevice, s));
  for (int n = n0; n < n1; ++n) {
    mrt::FwdLaunch<T> a;
    a.src = src;
    a.u0 = u0;
    a.v0 = v0;
    a.ctrl = ctrl;
    a.rec = record ? slot<T>(t, n - seg * t->K) : nullptr;
    a.variant = t->ns == 3 ? 4 : (t->so2 ? 2 : (t->impl ? 3 : 1));
    a.lag = t->so2 ? static_cast<T*>(t->lag) : nullptr;
    a.w0 = w0;
    T* dst = static_cast<T*>(t->buf[n & 1]);
    const bool closes = write_ckpt && t->mode == 2 && (n + 1) % t->K == 0 && n + 1 < t->nsteps;
    if (closes) dst = static_cast<T*>(t->ckpt[(n + 1) / t->K]);
    a.dst = dst;
    mrt::launch_forward_step<T>(g, m, a, s);
    span.count();
    int rc = last_launch_error();
    if (rc) return rc;
    if (closes && t->so2)
      HIP_TRY(hipMemcpyAsync(t->ckpt_lag[(n + 1) / t->K], t->lag, 2 * t->plane * t->elem,
                             hipMemcpyDeviceToDevice, s));
    src = dst;
  }
  *last = src;
  return MRT_OK;
}

template <typename T>
int forward_impl(const mrt_problem* p, mrt_tape* t, const void* u0,
                 const void* v0, const void* control, void* state, void* uN,
                 void* vN, hipStream_t s) {
  const mrt::ModelCoef<T> m = model_coef<T>(p);
  const mrt::Geometry g = geometry(t);
  const int N = t->nsteps;
  const bool adj = t->mode > 0;
  const int last_seg = t->nseg - 1;
  const T* cur = nullptr;
  const T* tu0 = static_cast<const T*>(u0);
  const T* tv0 = static_cast<const T*>(v0);
  const T* tc = static_cast<const T*>(control);
  t->fwd_done = false;
  int rc;
  // segments before the last: no record; the last one records the tape
  const int rec_start = adj ? last_seg * t->K : N;
  const T* tw0 = static_cast<const T*>(p->nspecies == 3 ? p->w0 : nullptr);
  if (rec_start > 0) {
    rc = run_forward_steps<T>(t, m, g, 0, rec_start, nullptr, tu0, tv0, tc,
                              false, true, 0, s, &cur, false, tw0);
    if (rc) return rc;
  }
  if (rec_start < N) {
    rc = run_forward_steps<T>(t, m, g, rec_start, N, cur, tu0, tv0, tc, true,
                              true, 0, s, &cur, false, tw0);
    if (rc) return rc;
  }
  mrt::launch_finalize<T>(g, cur, static_cast<T*>(state), static_cast<T*>(uN),
                          static_cast<T*>(vN), s, t->impl ? &m : nullptr, tc, t->ns == 3);
  rc = last_launch_error();
  if (rc) return rc;
  t->fwd_done = true;
  t->rec_seg = adj ? last_seg : -1;
  t->f_u0 = u0;
  t->f_v0 = v0;
  t->f_ctrl = control;
  return MRT_OK;
}

template <typename T>
int adjoint_impl(const mrt_problem* p, mrt_tape* t, const void* u0,
                 const void* v0, const void* control, const void* seed_u,
                 const void* seed_v, double* gacc, void* adj_u0, void* adj_v0,
                 hipStream_t s) {
  const mrt::ModelCoef<T> m = model_coef<T>(p);
  const mrt::Geometry g = geometry(t);
  const int N = t->nsteps, K = t->K;
  const T* tu0 = static_cast<const T*>(u0);
  const T* tv0 = static_cast<const T*>(v0);
  const T* tc = static_cast<const T*>(control);
  const bool want0 = adj_u0 != nullptr || adj_v0 != nullptr;
  const T* asrc = nullptr;
  for (int seg = t->nseg - 1; seg >= 0; --seg) {
    const int n0 = seg * K, n1 = std::min(N, n0 + K);
    if (t->rec_seg != seg) {
      // recompute the segment from its checkpoint, recording u and j_v
      // (also the last one when an earlier sweep overwrote its record)
      const T* src = seg == 0 ? nullptr : static_cast<const T*>(t->ckpt[seg]);
      const T* dummy = nullptr;
      t->rec_seg = -1;
      int rc = run_forward_steps<T>(t, m, g, n0, n1, src, tu0, tv0, tc, true,
                                    false, 2, s, &dummy, true,
                                    static_cast<const T*>(p->nspecies == 3 ? p->w0 : nullptr));
      if (rc) return rc;
      t->rec_seg = seg;
    }
    const T* su = static_cast<const T*>(seed_u);
    const T* sv = static_cast<const T*>(seed_v);
    if (t->impl && seg == t->nseg - 1) {
      // the cost sees Theta^N, a function of the sums of the last state,
      // which buf[(N-1) & 1] holds (the last step never closes a segment,
      // and the last segment was the most recent one run or recomputed)
      T* tu = static_cast<T*>(t->tseed);
      T* tv = tu + t->plane;
      mrt::launch_implicit_terminal<T>(g, m, static_cast<const T*>(t->buf[(N - 1) & 1]), tc,
                                       su, sv, tu, tv, gacc, s);
      int rc = last_launch_error();
      if (rc) return rc;
      su = tu;
      sv = tv;
    }
    SpanGuard span(1, s);
    for (int n = n1 - 1; n >= n0; --n) {
      mrt::AdjLaunch<T> a;
      a.src = asrc;
      a.first = n == N - 1;
      a.last = (n == 0 && want0) ? 1 : 0;
      a.dst = n == 0 ? nullptr : static_cast<T*>(t->abuf[n & 1]);
      a.seed_u = su;
      a.seed_v = sv;
      a.variant = t->ns == 3 ? 4 : (t->so2 ? 2 : (t->impl ? 3 : 1));
      a.rec = slot<T>(t, n - n0);
      a.g = gacc;
      a.adj_u0 = static_cast<T*>(adj_u0);
      a.adj_v0 = static_cast<T*>(adj_v0);
      a.mu = t->so2 ? static_cast<T*>(t->alag) : nullptr;
      a.step0 = n == 0 ? 1 : 0;
      mrt::launch_adjoint_step<T>(g, m, a, s);
      span.count();
      int rc = last_launch_error();
      if (rc) return rc;
      asrc = a.dst;
    }
  }
  return MRT_OK;
}

// Tangent-linear sweep: segments in forward order, each re-recorded from
// its checkpoint when the record slots hold another one, then the TLM
// steps of the segment into the adjoint ping-pong buffers.
template <typename T>
int tlm_impl(const mrt_problem* p, mrt_tape* t, const void* u0, const void* v0,
             const void* control, const void* dc, const void* du0, const void* dv0,
             void* duN, void* dvN, hipStream_t s) {
  const mrt::ModelCoef<T> m = model_coef<T>(p);
  const mrt::Geometry g = geometry(t);
  const int N = t->nsteps, K = t->K;
  const T* tu0 = static_cast<const T*>(u0);
  const T* tv0 = static_cast<const T*>(v0);
  const T* tc = static_cast<const T*>(control);
  const T* dsrc = nullptr;
  for (int seg = 0; seg < t->nseg; ++seg) {
    const int n0 = seg * K, n1 = std::min(N, n0 + K);
    if (t->rec_seg != seg) {
      const T* src = seg == 0 ? nullptr : static_cast<const T*>(t->ckpt[seg]);
      const T* dummy = nullptr;
      t->rec_seg = -1;
      int rc = run_forward_steps<T>(t, m, g, n0, n1, src, tu0, tv0, tc, true, false, 2, s,
                                    &dummy, true,
                                    static_cast<const T*>(p->nspecies == 3 ? p->w0 : nullptr));
      if (rc) return rc;
      t->rec_seg = seg;
    }
    SpanGuard span(3, s);
    for (int n = n0; n < n1; ++n) {
      mrt::TlmLaunch<T> a;
      a.src = dsrc;
      a.dst = static_cast<T*>(t->abuf[n & 1]);
      a.du0 = static_cast<const T*>(du0);
      a.dv0 = static_cast<const T*>(dv0);
      a.dc = static_cast<const T*>(dc);
      a.rec = slot<T>(t, n - n0);
      a.variant = t->ns == 3 ? 4 : (t->so2 ? 2 : (t->impl ? 3 : 1));
      a.dlag = t->so2 ? static_cast<T*>(t->alag) : nullptr;
      mrt::launch_tlm_step<T>(g, m, a, s);
      span.count();
      int rc = last_launch_error();
      if (rc) return rc;
      dsrc = a.dst;
    }
  }
  if (t->impl)
    // the last segment ran last, so buf[(N-1) & 1] holds the forward's last state
    mrt::launch_implicit_tlm_final<T>(g, m, static_cast<const T*>(t->buf[(N - 1) & 1]), dsrc,
                                      tc, static_cast<const T*>(dc), static_cast<T*>(duN),
                                      static_cast<T*>(dvN), s);
  else
    mrt::launch_finalize<T>(g, dsrc, nullptr, static_cast<T*>(duN), static_cast<T*>(dvN), s);
  return last_launch_error();
}

// Continuous-adjoint sweep: reversed steps k = 0..N-1 use the forward
// record of step N-1-k, so segments run in reverse as in the AMRT sweep.
template <typename T>
int cadjoint_impl(const mrt_problem* p, mrt_tape* t, const void* u0, const void* v0,
                  const void* control, const void* seed_u, double* gacc, hipStream_t s) {
  const mrt::ModelCoef<T> m = model_coef<T>(p);
  const mrt::CadjCoef<T> cc = mrt::host::cadj_coef<T>(p);
  const mrt::Geometry g = geometry(t);
  const int N = t->nsteps, K = t->K;
  const T* tu0 = static_cast<const T*>(u0);
  const T* tv0 = static_cast<const T*>(v0);
  const T* tc = static_cast<const T*>(control);
  const T* src = nullptr;
  for (int seg = t->nseg - 1; seg >= 0; --seg) {
    const int n0 = seg * K, n1 = std::min(N, n0 + K);
    if (t->rec_seg != seg) {
      const T* cs = seg == 0 ? nullptr : static_cast<const T*>(t->ckpt[seg]);
      const T* dummy = nullptr;
      t->rec_seg = -1;
      int rc = run_forward_steps<T>(t, m, g, n0, n1, cs, tu0, tv0, tc, true, false, 2, s,
                                    &dummy, true);
      if (rc) return rc;
      t->rec_seg = seg;
    }
    SpanGuard span(4, s);
    for (int n = n1 - 1; n >= n0; --n) {
      mrt::CadjLaunch<T> a;
      a.src = src;
      a.dst = static_cast<T*>(t->abuf[n & 1]);
      a.seed_u = static_cast<const T*>(seed_u);
      a.rec = slot<T>(t, n - n0);
      a.g = gacc;
      a.first = n == N - 1;
      mrt::launch_cadj_step<T>(g, m, cc, a, s);
      span.count();
      int rc = last_launch_error();
      if (rc) return rc;
      src = a.dst;
    }
  }
  return MRT_OK;
}

int read_result(mrt_tape* t, hipStream_t s, int n) {
  HIP_TRY(hipMemcpyAsync(t->host, t->result, sizeof(double) * n,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MRT_OK;
}

template <typename T>
int cost_impl(mrt_tape* t, double alpha, const void* uN, const void* ut,
              const void* ctrl, const double* gacc, void* seed, void* grad,
              mrt_scalars* out, hipStream_t s) {
  const mrt::Geometry g = geometry(t);
  mrt::launch_cost_grad<T>(g, static_cast<const T*>(uN),
                           static_cast<const T*>(ut),
                           static_cast<const T*>(ctrl), gacc,
                           static_cast<T*>(seed), static_cast<T*>(grad), alpha,
                           t->partials, t->result, s);
  int rc = last_launch_error();
  if (rc) return rc;
  rc = read_result(t, s, mrt::kRedSlots);
  if (rc) return rc;
  const double* h = t->host;
  mrt_scalars r{};
  r.J_track = h[0];
  r.J_reg = h[1];
  r.J = h[0] + h[1];
  r.grad_l2 = gacc ? std::sqrt(h[2]) : 0.0;
  r.grad_inf = gacc ? h[3] : 0.0;
  r.n_fluid = t->n_fluid;
  if (out) *out = r;
  if (h[4] != 0.0 || !std::isfinite(r.J) || !std::isfinite(r.grad_l2))
    return fail(MRT_ENONFINITE, "non-finite cost or gradient (%g values)", h[4]);
  return MRT_OK;
}

// Inner products <a_k, b_k> (k < n <= 4) over the fluid nodes, in one pass;
// out[k] for k < n.  Synchronises the stream.
int dots(const mrt_problem* p, mrt_tape* t, int n, const void* const* a, const void* const* b,
         double* out, hipStream_t s) {
  const mrt::Geometry g = geometry(t);
  if (p->grid.dtype == MRT_F64) {
    mrt::DotPairs<double> d{};
    for (int k = 0; k < n; ++k) {
      d.a[k] = static_cast<const double*>(a[k]);
      d.b[k] = static_cast<const double*>(b[k]);
    }
    d.n = n;
    mrt::launch_dots<double>(g, d, t->partials, t->result, s);
  } else {
    mrt::DotPairs<float> d{};
    for (int k = 0; k < n; ++k) {
      d.a[k] = static_cast<const float*>(a[k]);
      d.b[k] = static_cast<const float*>(b[k]);
    }
    d.n = n;
    mrt::launch_dots<float>(g, d, t->partials, t->result, s);
  }
  int rc = last_launch_error();
  if (rc) return rc;
  rc = read_result(t, s, mrt::kRedSlots);
  if (rc) return rc;
  if (t->host[3] != 0.0) return fail(MRT_ENONFINITE, "non-finite inner product");
  static const int slot[4] = {0, 1, 2, 4};
  for (int k = 0; k < n; ++k) out[k] = t->host[slot[k]];
  return MRT_OK;
}

void axpby_any(const mrt_problem* p, mrt_tape* t, const void* x, void* y, double a, double b,
               hipStream_t s) {
  const mrt::Geometry g = geometry(t);
  if (p->grid.dtype == MRT_F64)
    mrt::launch_axpby<double>(g, static_cast<const double*>(x), static_cast<double*>(y), a, b,
                              s);
  else
    mrt::launch_axpby<float>(g, static_cast<const float*>(x), static_cast<float*>(y), a, b, s);
}

// Products of the scalar formulas below are rounded before they are added
// (no fused multiply-add), as written.
double sum_of_products(double a, double x, double b, double y) {
#pragma clang fp contract(off)
  const double ax = a * x, by = b * y;
  return ax + by;
}

void free_tape(mrt_tape* t) {
  if (!t) return;
  for (void* a : t->allocs) (void)hipFree(a);
  if (t->host) (void)hipHostFree(t->host);
  delete t;
}

}  // namespace

extern "C" {

int mrt_validate(const mrt_problem* p) { return validate(p); }

int mrt_tape_bytes(const mrt_problem* p, int32_t ckpt_every, size_t* bytes) {
  int rc = validate(p);
  if (rc) return rc;
  if (!bytes) return fail(MRT_EINVAL, "bytes is NULL");
  *bytes = plan(p, ckpt_every).total;
  return MRT_OK;
}

int mrt_tape_create(const mrt_problem* p, int32_t ckpt_every,
                    size_t mem_budget, mrt_tape** out) {
  int rc = validate(p);
  if (rc) return rc;
  if (!out) return fail(MRT_EINVAL, "out is NULL");
  *out = nullptr;
  const Layout L = plan(p, ckpt_every);
  if (mem_budget > 0 && L.total > mem_budget)
    return fail(MRT_ENOMEM, "tape needs %zu bytes, budget %zu", L.total,
                mem_budget);
  mrt_tape* t = new mrt_tape();
  const mrt_grid& g = p->grid;
  t->nx = g.nx;
  t->ny = g.ny;
  t->pitch = g.pitch;
  t->nsteps = g.nsteps;
  t->dtype = g.dtype;
  t->periodic = g.periodic;
  t->masked = g.mask != nullptr ? 1 : 0;
  t->mode = L.mode;
  t->K = L.K;
  t->nseg = L.nseg;
  t->ns = p->nspecies == 3 ? 3 : 2;
  t->so2 = p->source_term == 2 ? 1 : 0;
  t->impl = p->source_term == 3 ? 1 : 0;
  t->plane = L.plane;
  t->elem = L.elem;
  t->state_bytes = L.state_bytes;
  t->rec_slot_bytes = L.rec_slot_bytes;
  t->total_bytes = L.total;
  auto alloc = [&](size_t bytes, void** ptr) -> int {
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(MRT_ENOMEM, "hipMalloc(%zu) failed: %s", bytes,
                  hipGetErrorString(e));
    }
    t->allocs.push_back(*ptr);
    return MRT_OK;
  };
  if (hipGetDevice(&t->device) != hipSuccess) {
    delete t;
    return fail(MRT_EHIP, "no HIP device");
  }
  rc = alloc(L.state_bytes, &t->buf[0]);
  if (!rc) rc = alloc(L.state_bytes, &t->buf[1]);
  if (!rc && t->so2) rc = alloc(L.lag_bytes, &t->lag);
  if (!rc && t->masked) rc = alloc(L.plane * sizeof(uint16_t), (void**)&t->link);
  if (!rc && t->masked)
    rc = alloc(size_t(g.ny) * ((g.nx + 63) / 64) * sizeof(uint32_t),
               (void**)&t->wflag);
  if (!rc)
    rc = alloc((size_t(mrt::kRedBlocks) * mrt::kRedSlots + 16) * sizeof(double),
               (void**)&t->partials);
  if (!rc && L.mode > 0) {
    rc = alloc(L.state_bytes, &t->abuf[0]);
    if (!rc) rc = alloc(L.state_bytes, &t->abuf[1]);
    t->ckpt.assign(L.nseg, nullptr);
    for (int k = 1; k < L.nseg && !rc; ++k) rc = alloc(L.state_bytes, &t->ckpt[k]);
    if (!rc && t->so2) rc = alloc(L.lag_bytes, &t->alag);
    if (!rc && t->impl) rc = alloc(L.tseed_bytes, &t->tseed);
    t->ckpt_lag.assign(L.nseg, nullptr);
    for (int k = 1; t->so2 && k < L.nseg && !rc; ++k) rc = alloc(L.lag_bytes, &t->ckpt_lag[k]);
    if (!rc) rc = alloc(size_t(L.K) * L.rec_slot_bytes, &t->rec);
  }
  if (!rc && hipHostMalloc((void**)&t->host, 16 * sizeof(double)) != hipSuccess)
    rc = fail(MRT_ENOMEM, "hipHostMalloc failed");
  if (rc) {
    free_tape(t);
    return rc;
  }
  t->result = t->partials + size_t(mrt::kRedBlocks) * mrt::kRedSlots;
  const mrt::Geometry geo = geometry(t);
  hipStream_t s = nullptr;
  if (t->masked)
    mrt::launch_build_link(geo, g.periodic, g.mask, t->link, t->wflag, s);
  mrt::launch_count_fluid(geo, t->partials, t->result, s);
  rc = last_launch_error();
  if (!rc) rc = read_result(t, s, 1);
  if (rc) {
    free_tape(t);
    return rc;
  }
  t->n_fluid = int64_t(t->host[0]);
  *out = t;
  return MRT_OK;
}

void mrt_tape_destroy(mrt_tape* t) {
  if (!t) return;
  (void)hipDeviceSynchronize();
  free_tape(t);
}

int mrt_tape_query(const mrt_tape* t, mrt_tape_info* info) {
  if (!t || !info) return fail(MRT_EINVAL, "NULL argument");
  info->mode = t->mode;
  info->ckpt_every = t->K;
  info->n_segments = t->nseg;
  info->reserved = 0;
  info->n_fluid = t->n_fluid;
  info->device_bytes = t->total_bytes;
  return MRT_OK;
}

int mrt_forward(const mrt_problem* p, mrt_tape* t, const void* u0,
                const void* v0, const void* control, void* state, void* uN,
                void* vN, void* stream) {
  int rc = validate(p);
  if (rc) return rc;
  rc = check_tape(p, t);
  if (rc) return rc;
  if (!u0 || !v0 || !control) return fail(MRT_EINVAL, "u0, v0, control required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return p->grid.dtype == MRT_F64
             ? forward_impl<double>(p, t, u0, v0, control, state, uN, vN, s)
             : forward_impl<float>(p, t, u0, v0, control, state, uN, vN, s);
}

int amrt_adjoint(const mrt_problem* p, mrt_tape* t, const void* u0,
                 const void* v0, const void* control, const void* seed_u,
                 const void* seed_v, double* grad_accum, void* adj_u0,
                 void* adj_v0, void* stream) {
  int rc = validate(p);
  if (rc) return rc;
  rc = check_tape(p, t);
  if (rc) return rc;
  if (t->mode == 0) return fail(MRT_ESTATE, "tape was created without adjoint record");
  if (!t->fwd_done) return fail(MRT_ESTATE, "no forward solve recorded on this tape");
  if (u0 != t->f_u0 || v0 != t->f_v0 || control != t->f_ctrl)
    return fail(MRT_ESTATE, "u0/v0/control differ from the recorded forward");
  if (!seed_u || !grad_accum) return fail(MRT_EINVAL, "seed_u and grad_accum required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return p->grid.dtype == MRT_F64
             ? adjoint_impl<double>(p, t, u0, v0, control, seed_u, seed_v,
                                    grad_accum, adj_u0, adj_v0, s)
             : adjoint_impl<float>(p, t, u0, v0, control, seed_u, seed_v,
                                   grad_accum, adj_u0, adj_v0, s);
}

int cost_gradient(const mrt_problem* p, mrt_tape* t, const void* uN,
                  const void* u_target, const void* control,
                  const double* grad_accum, void* seed_out, void* grad_out,
                  mrt_scalars* out, void* stream) {
  int rc = validate(p);
  if (rc) return rc;
  rc = check_tape(p, t);
  if (rc) return rc;
  if (!uN || !u_target || !control)
    return fail(MRT_EINVAL, "uN, u_target, control required");
  if (grad_accum && !grad_out)
    return fail(MRT_EINVAL, "grad_out required with grad_accum");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return p->grid.dtype == MRT_F64
             ? cost_impl<double>(t, p->alpha, uN, u_target, control,
                                 grad_accum, seed_out, grad_out, out, s)
             : cost_impl<float>(t, p->alpha, uN, u_target, control, grad_accum,
                                seed_out, grad_out, out, s);
}

int cost_gradient_noalloc(const mrt_problem* p, const void* uN, const void* u_target,
                          const void* control, const double* grad_accum, void* seed_out,
                          void* grad_out, mrt_scalars* out, void* stream) {
  int rc = validate(p);
  if (rc) return rc;
  if (!uN || !u_target || !control)
    return fail(MRT_EINVAL, "uN, u_target, control required");
  if (grad_accum && !grad_out)
    return fail(MRT_EINVAL, "grad_out required with grad_accum");
  const mrt_grid& gr = p->grid;
  const size_t nodes = size_t(gr.nx) * size_t(gr.ny);
  if (nodes > mrt::kNoallocMaxNodes)
    return fail(MRT_EINVAL,
                "cost_gradient_noalloc: %zu nodes exceed the maximum of %zu (2^30)", nodes,
                mrt::kNoallocMaxNodes);
  mrt::Geometry g{};
  g.nx = gr.nx;
  g.ny = gr.ny;
  g.pitch = gr.pitch;
  g.periodic = gr.periodic;
  g.masked = gr.mask != nullptr;
  g.plane = size_t(gr.ny) * size_t(gr.pitch);
  g.nsx = (gr.nx + 63) / 64;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double h[2 * mrt::kRedSlots];
  const hipError_t e =
      gr.dtype == MRT_F64
          ? mrt::launch_cost_grad_noalloc<double>(
                g, gr.mask, static_cast<const double*>(uN),
                static_cast<const double*>(u_target), static_cast<const double*>(control),
                grad_accum, static_cast<double*>(seed_out), static_cast<double*>(grad_out),
                p->alpha, h, s)
          : mrt::launch_cost_grad_noalloc<float>(
                g, gr.mask, static_cast<const float*>(uN),
                static_cast<const float*>(u_target), static_cast<const float*>(control),
                grad_accum, static_cast<float*>(seed_out), static_cast<float*>(grad_out),
                p->alpha, h, s);
  if (e != hipSuccess)
    return fail(MRT_EHIP, "cost_gradient_noalloc: %s", hipGetErrorString(e));
  mrt_scalars r{};
  r.J_track = h[0];
  r.J_reg = h[1];
  r.J = h[0] + h[1];
  r.grad_l2 = grad_accum ? std::sqrt(h[2]) : 0.0;
  r.grad_inf = grad_accum ? h[3] : 0.0;
  r.n_fluid = int64_t(h[mrt::kRedSlots]);
  if (out) *out = r;
  if (h[4] != 0.0 || !std::isfinite(r.J) || !std::isfinite(r.grad_l2))
    return fail(MRT_ENONFINITE, "non-finite cost or gradient (%g values)", h[4]);
  return MRT_OK;
}

int gd_step(const mrt_problem* p, mrt_tape* t, void* control, const void* grad,
            double zeta, double lo, double hi, double* zeta_used,
            void* stream) {
  int rc = validate(p);
  if (rc) return rc;
  rc = check_tape(p, t);
  if (rc) return rc;
  if (!control || !grad) return fail(MRT_EINVAL, "control and grad required");
  if (std::isnan(zeta) || std::isnan(lo) || std::isnan(hi) || lo > hi)
    return fail(MRT_EINVAL, "invalid zeta or bounds");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const mrt::Geometry g = geometry(t);
  if (p->grid.dtype == MRT_F64)
    mrt::launch_gd_step<double>(g, static_cast<double*>(control),
                                static_cast<const double*>(grad), zeta, lo, hi,
                                t->partials, t->result, s);
  else
    mrt::launch_gd_step<float>(g, static_cast<float*>(control),
                               static_cast<const float*>(grad), zeta, lo, hi,
                               t->partials, t->result, s);
  rc = last_launch_error();
  if (rc) return rc;
  if (zeta_used) {
    HIP_TRY(hipMemcpyAsync(t->host + mrt::kRedSlots, t->result + mrt::kRedSlots,
                           sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *zeta_used = t->host[mrt::kRedSlots];
    if (!std::isfinite(*zeta_used))
      return fail(MRT_ENONFINITE, "non-finite step (gradient not finite)");
  }
  return MRT_OK;
}

int mrt_tlm(const mrt_problem* p, mrt_tape* t, const void* u0, const void* v0,
            const void* control, const void* dc, const void* du0, const void* dv0,
            void* duN, void* dvN, void* stream) {
  int rc = validate(p);
  if (rc) return rc;
  rc = check_tape(p, t);
  if (rc) return rc;
  if (t->mode == 0) return fail(MRT_ESTATE, "tape was created without a record");
  if (!t->fwd_done) return fail(MRT_ESTATE, "no forward solve recorded on this tape");
  if (u0 != t->f_u0 || v0 != t->f_v0 || control != t->f_ctrl)
    return fail(MRT_ESTATE, "u0/v0/control differ from the recorded forward");
  if (!duN && !dvN) return fail(MRT_EINVAL, "duN or dvN required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return p->grid.dtype == MRT_F64
             ? tlm_impl<double>(p, t, u0, v0, control, dc, du0, dv0, duN, dvN, s)
             : tlm_impl<float>(p, t, u0, v0, control, dc, du0, dv0, duN, dvN, s);
}

int mrt_cadjoint(const mrt_problem* p, mrt_tape* t, const void* u0, const void* v0,
                 const void* control, const void* seed_u, double* grad_accum, void* stream) {
  int rc = validate(p);
  if (rc) return rc;
  rc = check_tape(p, t);
  if (rc) return rc;
  if (t->mode == 0) return fail(MRT_ESTATE, "tape was created without a record");
  if (!t->fwd_done) return fail(MRT_ESTATE, "no forward solve recorded on this tape");
  if (u0 != t->f_u0 || v0 != t->f_v0 || control != t->f_ctrl)
    return fail(MRT_ESTATE, "u0/v0/control differ from the recorded forward");
  if (!seed_u || !grad_accum) return fail(MRT_EINVAL, "seed_u and grad_accum required");
  if (t->ns == 3) return fail(MRT_EINVAL, "the continuous adjoint takes two species only");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return p->grid.dtype == MRT_F64
             ? cadjoint_impl<double>(p, t, u0, v0, control, seed_u, grad_accum, s)
             : cadjoint_impl<float>(p, t, u0, v0, control, seed_u, grad_accum, s);
}

int mrt_dot(const mrt_problem* p, mrt_tape* t, const void* x, const void* y, double* out,
            void* stream) {
  int rc = validate(p);
  if (rc) return rc;
  rc = check_tape(p, t);
  if (rc) return rc;
  if (!x || !y || !out) return fail(MRT_EINVAL, "x, y and out required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const mrt::Geometry g = geometry(t);
  if (p->grid.dtype == MRT_F64)
    mrt::launch_dot<double>(g, static_cast<const double*>(x), static_cast<const double*>(y),
                            t->partials, t->result, s);
  else
    mrt::launch_dot<float>(g, static_cast<const float*>(x), static_cast<const float*>(y),
                           t->partials, t->result, s);
  rc = last_launch_error();
  if (rc) return rc;
  rc = read_result(t, s, mrt::kRedSlots);
  if (rc) return rc;
  *out = t->host[0];
  if (t->host[4] != 0.0 || !std::isfinite(*out))
    return fail(MRT_ENONFINITE, "non-finite dot product");
  return MRT_OK;
}

int mrt_axpby(const mrt_problem* p, mrt_tape* t, const void* x, void* y, double a, double b,
              void* stream) {
  int rc = validate(p);
  if (rc) return rc;
  rc = check_tape(p, t);
  if (rc) return rc;
  if (!x || !y) return fail(MRT_EINVAL, "x and y required");
  if (!std::isfinite(a) || !std::isfinite(b)) return fail(MRT_EINVAL, "non-finite a or b");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const mrt::Geometry g = geometry(t);
  if (p->grid.dtype == MRT_F64)
    mrt::launch_axpby<double>(g, static_cast<const double*>(x), static_cast<double*>(y), a, b,
                              s);
  else
    mrt::launch_axpby<float>(g, static_cast<const float*>(x), static_cast<float*>(y), a, b, s);
  return last_launch_error();
}

int mrt_lma_step(const mrt_problem* p, mrt_tape* t, const void* control, const void* dir,
                 const void* resid, const void* P, double* zeta, void* stream) {
  int rc = validate(p);
  if (rc) return rc;
  rc = check_tape(p, t);
  if (rc) return rc;
  if (!control || !dir || !resid || !P || !zeta)
    return fail(MRT_EINVAL, "control, dir, resid, P and zeta required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const void* a[4] = {resid, control, P, dir};
  const void* b[4] = {P, dir, P, dir};
  double d[4];
  rc = dots(p, t, 4, a, b, d, s);
  if (rc) return rc;
  const double num = sum_of_products(1.0, d[0], p->alpha, d[1]);
  const double den = sum_of_products(1.0, d[2], p->alpha, d[3]);
  *zeta = den > 0.0 ? num / den : 0.0;
  if (!std::isfinite(*zeta)) return fail(MRT_ENONFINITE, "non-finite LMA step");
  return MRT_OK;
}

int mrt_cg_direction(const mrt_problem* p, mrt_tape* t, int32_t rule, int32_t first,
                     const void* G, const void* Gprev, void* D, double gg_old, double dg_old,
                     mrt_cg_info* out, void* stream) {
  int rc = validate(p);
  if (rc) return rc;
  rc = check_tape(p, t);
  if (rc) return rc;
  if (!G || !D || !out || (!first && !Gprev))
    return fail(MRT_EINVAL, "G, D, out (and Gprev after the first iteration) required");
  if (rule < MRT_CG_FR || rule > MRT_CG_DY) return fail(MRT_EINVAL, "unknown CG rule %d", rule);
  if (!first && (!(gg_old > 0.0) || !std::isfinite(dg_old)))
    return fail(MRT_EINVAL, "previous <G, G> must be positive and <D, G> finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  mrt_cg_info r{};
  if (first) {
    const void* a[1] = {G};
    rc = dots(p, t, 1, a, a, &r.gg, s);
    if (rc) return rc;
    axpby_any(p, t, G, D, -1.0, 0.0, s);
    r.restart = 1;
  } else {
    const void* a[3] = {G, G, D};
    const void* b[3] = {G, Gprev, G};
    double d[3];
    rc = dots(p, t, 3, a, b, d, s);
    if (rc) return rc;
    r.gg = d[0];
    const double g_go = d[1], d_g = d[2];
    const double y_g = r.gg - g_go;  // <G_k, G_k - G_{k-1}>
    const double d_y = d_g - dg_old; // <D_{k-1}, G_k - G_{k-1}>
    double beta = 0.0;
    switch (rule) {
      case MRT_CG_FR: beta = r.gg / gg_old; break;
      case MRT_CG_PR: beta = std::max(0.0, y_g / gg_old); break;
      case MRT_CG_HS: beta = d_y != 0.0 ? std::max(0.0, y_g / d_y) : 0.0; break;
      default: beta = d_y != 0.0 ? r.gg / d_y : 0.0; break;
    }
    r.beta = beta;
    // Powell: restart when consecutive gradients are far from orthogonal
    r.restart = std::fabs(g_go) >= 0.2 * r.gg ? 1 : 0;
    axpby_any(p, t, G, D, -1.0, r.restart ? 0.0 : beta, s);
  }
  const void* a[1] = {D};
  const void* b[1] = {G};
  rc = dots(p, t, 1, a, b, &r.dg, s);
  if (rc) return rc;
  if (!r.restart && r.dg >= 0.0) {  // not a descent direction: steepest descent
    axpby_any(p, t, G, D, -1.0, 0.0, s);
    r.restart = 1;
    rc = dots(p, t, 1, a, b, &r.dg, s);
    if (rc) return rc;
  }
  *out = r;
  return last_launch_error();
}

const char* mrt_last_error(void) { return g_err.c_str(); }

int mrt_timing_enable(int32_t on) {
  Timing& t = timing();
  std::lock_guard<std::mutex> lk(t.mu);
  t.on = on != 0;
  return MRT_OK;
}

int mrt_timing_reset(void) {
  Timing& t = timing();
  std::lock_guard<std::mutex> lk(t.mu);
  for (auto& sp : t.pending) {
    (void)hipEventSynchronize(sp.b);
    (void)hipEventDestroy(sp.a);
    (void)hipEventDestroy(sp.b);
  }
  t.pending.clear();
  for (int k = 0; k < 5; ++k) {
    t.ms[k] = 0.0;
    t.launches[k] = 0;
  }
  return MRT_OK;
}

int mrt_stream_probe(int32_t reads, int32_t writes, int32_t order, const float* in, float* out,
                     int64_t n, void* stream) {
  if (!in || !out || n < 0) return fail(MRT_EINVAL, "NULL buffer or negative size");
  if (order != 0 && order != 1) return fail(MRT_EINVAL, "order must be 0 or 1");
  if (!mrt::stream_probe_has_mix(reads, writes))
    return fail(MRT_EINVAL, "stream probe: mix (%d, %d) not built", int(reads), int(writes));
  if (n == 0) return MRT_OK;
  if (!mrt::launch_stream_probe(reads, writes, order == 1, in, out, size_t(n),
                                static_cast<hipStream_t>(stream)))
    return fail(MRT_EINVAL, "stream probe: n too large");
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRT_OK : fail(MRT_EHIP, "%s", hipGetErrorString(e));
}

int mrt_timing_read(int32_t kind, double* ms, int64_t* launches) {
  if (kind < 0 || kind > 4) return fail(MRT_EINVAL, "kind must be 0..4");
  Timing& t = timing();
  std::lock_guard<std::mutex> lk(t.mu);
  for (auto& sp : t.pending) {
    HIP_TRY(hipEventSynchronize(sp.b));
    float e = 0.f;
    HIP_TRY(hipEventElapsedTime(&e, sp.a, sp.b));
    t.ms[sp.kind] += e;
    t.launches[sp.kind] += sp.launches;
    (void)hipEventDestroy(sp.a);
    (void)hipEventDestroy(sp.b);
  }
  t.pending.clear();
  if (ms) *ms = t.ms[kind];
  if (launches) *launches = t.launches[kind];
  return MRT_OK;
}

}  // extern "C"
