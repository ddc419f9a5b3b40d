// C-ABI runtime of the D3Q19 hot path: parameter validation, the device
// workspace ("tape"), the forward / adjoint / tangent step loops with the
// checkpoint schedule, and the cost, gradient and update reductions (the
// D2Q9 reduction kernels applied to the 3-D fields as [nz*ny][pitch]).
// See include/mrt3.h for the contract of every entry point.
#include "mrt3.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mrt3_internal.h"
#include "mrt_host.h"
#include "mrt_internal.h"

using mrt::host::failf;

#define HIP_TRY3(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return failf(MRT_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

namespace {

constexpr double kCs2 = 1.0 / 3.0;
constexpr double kTau = 1.0;

bool finite_all(const double* a, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

bool inv3(const double* a, double* r) {
  const double c0 = a[4] * a[8] - a[5] * a[7];
  const double c1 = a[5] * a[6] - a[3] * a[8];
  const double c2 = a[3] * a[7] - a[4] * a[6];
  const double det = a[0] * c0 + a[1] * c1 + a[2] * c2;
  if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
  r[0] = c0 / det;
  r[1] = (a[2] * a[7] - a[1] * a[8]) / det;
  r[2] = (a[1] * a[5] - a[2] * a[4]) / det;
  r[3] = c1 / det;
  r[4] = (a[0] * a[8] - a[2] * a[6]) / det;
  r[5] = (a[2] * a[3] - a[0] * a[5]) / det;
  r[6] = c2 / det;
  r[7] = (a[1] * a[6] - a[0] * a[7]) / det;
  r[8] = (a[0] * a[4] - a[1] * a[3]) / det;
  return true;
}

void mul3(const double* a, const double* b, double* c) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}

// K = (D / (d Cs^2 tau) + I/2)^-1, from D = d Cs^2 tau (K^-1 - I/2).
bool k_block3(const mrt3_species& s, double K[9]) {
  double A[9];
  for (int k = 0; k < 9; ++k) A[k] = s.D[k] / (s.d * kCs2 * kTau) + (k % 4 == 0 ? 0.5 : 0.0);
  return inv3(A, K);
}

int check_species3(const mrt3_species& s, const char* name) {
  if (!finite_all(s.D, 9) || !std::isfinite(s.d) || !finite_all(s.s, 16))
    return failf(MRT_EINVAL, "species %s: non-finite coefficient", name);
  double scale = 1e-300;
  for (int k = 0; k < 9; ++k) scale = std::max(scale, std::fabs(s.D[k]));
  for (int a = 0; a < 3; ++a)
    for (int b = a + 1; b < 3; ++b)
      if (std::fabs(s.D[3 * a + b] - s.D[3 * b + a]) > 1e-12 * scale)
        return failf(MRT_EINVAL, "species %s: D must be symmetric", name);
  // Sylvester: leading principal minors positive
  const double m1 = s.D[0];
  const double m2 = s.D[0] * s.D[4] - s.D[1] * s.D[3];
  const double m3 = s.D[0] * (s.D[4] * s.D[8] - s.D[5] * s.D[7]) -
                    s.D[1] * (s.D[3] * s.D[8] - s.D[5] * s.D[6]) +
                    s.D[2] * (s.D[3] * s.D[7] - s.D[4] * s.D[6]);
  if (!(m1 > 0.0 && m2 > 0.0 && m3 > 0.0))
    return failf(MRT_EINVAL, "species %s: D must be positive definite", name);
  if (!(s.d > 0.0)) return failf(MRT_EINVAL, "species %s: d must be > 0", name);
  for (int j = 0; j < 16; ++j)
    if (!(s.s[j] > 0.0 && s.s[j] < 2.0))
      return failf(MRT_EINVAL, "species %s: rate s%d = %g outside (0, 2)", name, j, s.s[j]);
  // K = (D/(d Cs^2 tau) + I/2)^-1 then has its eigenvalues in (0, 2)
  double K[9];
  if (!k_block3(s, K)) return failf(MRT_EINVAL, "species %s: singular K", name);
  return MRT_OK;
}

int validate3(const mrt3_problem* p) {
  if (!p) return failf(MRT_EINVAL, "problem is NULL");
  const mrt3_grid& g = p->grid;
  if (g.nx < 1 || g.ny < 1 || g.nz < 1 || g.nx > 4096 || g.ny > 4096 || g.nz > 4096)
    return failf(MRT_EINVAL, "grid %d x %d x %d outside 1..4096", g.nx, g.ny, g.nz);
  if (g.pitch < g.nx) return failf(MRT_EINVAL, "pitch %d < nx %d", g.pitch, g.nx);
  if (double(g.nz) * double(g.ny) * double(g.pitch) >= 2147483648.0)
    return failf(MRT_EINVAL, "nz * ny * pitch must be < 2^31");
  if (mrt3::internal_plane(g.nx, g.ny, g.nz) >= (size_t(1) << 29))
    return failf(MRT_EINVAL, "lattice too large: (nz + 2)(ny + 2) * roundup(nx, 64) "
                             "must be < 2^29");
  if (g.nsteps < 1) return failf(MRT_EINVAL, "nsteps %d < 1", g.nsteps);
  if (g.dtype != MRT_F32 && g.dtype != MRT_F64)
    return failf(MRT_EINVAL, "unknown dtype %d", g.dtype);
  if (g.periodic != 0 && g.periodic != 1) return failf(MRT_EINVAL, "periodic must be 0 or 1");
  if (g.reserved != 0) return failf(MRT_EINVAL, "grid.reserved must be 0");
  int rc = check_species3(p->u, "u");
  if (rc) return rc;
  rc = check_species3(p->v, "v");
  if (rc) return rc;
  const double sc[4] = {p->chi, p->r_u, p->a_uv, p->b_v};
  if (!finite_all(sc, 4) || !finite_all(p->Cchi, 9) || !std::isfinite(p->alpha))
    return failf(MRT_EINVAL, "non-finite model coefficient");
  if (p->alpha < 0.0) return failf(MRT_EINVAL, "alpha < 0");
  return MRT_OK;
}

double row_norm2(int k) {
  double s = 0;
  for (int i = 0; i < mrt3::Q; ++i) s += double(mrt3::mrow(k, i)) * mrt3::mrow(k, i);
  return s;
}

template <typename T>
mrt3::Species3Coef<T> species_coef3(const mrt3_species& s) {
  mrt3::Species3Coef<T> c{};
  for (int k = 0; k < mrt3::Q; ++k) c.c[k] = T(0);
  for (int j = 1; j < 16; ++j) {
    const int k = mrt3::free_row(j);
    c.c[k] = T(s.s[j] / row_norm2(k));
  }
  double K[9];
  k_block3(s, K);
  for (int k = 0; k < 9; ++k) c.k[k] = T(K[k] / row_norm2(3));
  // (phieq) with zero flux and B = d Cs^2 Theta I:
  // w~_i = w_i (1 + (d - 1)(|e_i|^2 - 3 Cs^2) / (2 Cs^2))
  const double w[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
  double wt[3];
  for (int sh = 0; sh < 3; ++sh)
    wt[sh] = w[sh] * (1.0 + (s.d - 1.0) * (double(sh) - 3.0 * kCs2) / (2.0 * kCs2));
  double e_eq = 0, eps_eq = 0;
  for (int i = 0; i < mrt3::Q; ++i) {
    const double wi = wt[i == 0 ? 0 : (i <= 6 ? 1 : 2)];
    e_eq += mrt3::mrow(1, i) * wi;
    eps_eq += mrt3::mrow(2, i) * wi;
  }
  c.e_eq = T(e_eq);
  c.eps_eq = T(eps_eq);
  c.w_rest = T(wt[0]);
  c.w_axis = T(wt[1]);
  c.w_diag = T(wt[2]);
  return c;
}

template <typename T>
mrt3::Model3Coef<T> model_coef3(const mrt3_problem* p) {
  mrt3::Model3Coef<T> m{};
  m.u = species_coef3<T>(p->u);
  m.v = species_coef3<T>(p->v);
  // A_u1 grad v = (K_u chi u Cchi / tau)(-K_v j_v / (tau d_v Cs^2)) = u B j_v
  double Ku[9], Kv[9], KC[9], B[9];
  k_block3(p->u, Ku);
  k_block3(p->v, Kv);
  mul3(Ku, p->Cchi, KC);
  mul3(KC, Kv, B);
  const double f = -p->chi / (kTau * kTau * p->v.d * kCs2);
  for (int k = 0; k < 9; ++k) m.b[k] = T(f * B[k]);
  m.r_u = T(p->r_u);
  m.a_uv = T(p->a_uv);
  m.b_v = T(p->b_v);
  return m;
}

struct Layout3 {
  int mode, K, nseg;
  size_t plane, planeI, elem, state_bytes, rec_slot_bytes, total;
};

// Link words are in use with a mask and on every non-periodic lattice.
bool uses_links(const mrt3_grid& g) { return g.mask != nullptr || g.periodic == 0; }

Layout3 plan3(const mrt3_problem* p, int ckpt_every) {
  Layout3 L{};
  const mrt3_grid& g = p->grid;
  L.plane = size_t(g.nz) * size_t(g.ny) * size_t(g.pitch);
  L.planeI = mrt3::internal_plane(g.nx, g.ny, g.nz);
  L.elem = g.dtype == MRT_F64 ? 8 : 4;
  L.state_bytes = size_t(2 * mrt3::Q) * L.planeI * L.elem;
  L.rec_slot_bytes = 4 * L.plane * L.elem;
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
  size_t t = 2 * L.state_bytes;
  if (uses_links(g))
    t += L.plane * (sizeof(uint32_t) + sizeof(uint16_t)) +
         size_t(g.nz) * g.ny * ((g.nx + 63) / 64) * sizeof(uint32_t);
  t += (size_t(mrt::kRedBlocks) * mrt::kRedSlots + 16) * sizeof(double);
  if (L.mode > 0) {
    t += 2 * L.state_bytes;                            // adjoint ping-pong
    t += size_t(L.nseg - 1) * L.state_bytes;           // checkpoints
    t += size_t(L.K) * L.rec_slot_bytes;               // record slots
  }
  L.total = t;
  return L;
}

}  // namespace

struct mrt3_tape {
  int nx, ny, nz, pitch, nsteps, dtype, periodic, masked, device;
  int has_mask;              // a solid mask was given (masked: link words in use)
  int mode, K, nseg;
  size_t plane, planeI, elem, state_bytes, rec_slot_bytes, total_bytes;
  void* buf[2] = {nullptr, nullptr};
  void* abuf[2] = {nullptr, nullptr};
  std::vector<void*> ckpt;   // ckpt[s] (s >= 1): post-collision state of step sK-1
  void* rec = nullptr;       // record slots [K][4][plane]
  uint32_t* link = nullptr;
  uint32_t* wflag = nullptr;
  uint16_t* solid16 = nullptr;
  double* partials = nullptr;
  double* result = nullptr;
  double* host = nullptr;    // pinned
  int64_t n_fluid = 0;
  bool fwd_done = false;
  int rec_seg = -1;
  const void* f_u0 = nullptr;
  const void* f_v0 = nullptr;
  const void* f_ctrl = nullptr;
  std::vector<void*> allocs;
};

namespace {

int check_tape3(const mrt3_problem* p, const mrt3_tape* t) {
  if (!t) return failf(MRT_EINVAL, "tape is NULL");
  const mrt3_grid& g = p->grid;
  const int has_mask = g.mask != nullptr ? 1 : 0;
  if (g.nx != t->nx || g.ny != t->ny || g.nz != t->nz || g.pitch != t->pitch ||
      g.nsteps != t->nsteps || g.dtype != t->dtype || g.periodic != t->periodic ||
      has_mask != t->has_mask)
    return failf(MRT_ESTATE, "tape was created for another grid");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != t->device)
    return failf(MRT_ESTATE, "tape belongs to device %d, current is %d", t->device, dev);
  return MRT_OK;
}

mrt3::Geometry3 geometry3(const mrt3_tape* t) {
  mrt3::Geometry3 g{};
  g.nx = t->nx;
  g.ny = t->ny;
  g.nz = t->nz;
  g.pitch = t->pitch;
  g.periodic = t->periodic;
  g.masked = t->masked;
  g.plane = uint32_t(t->plane);
  g.pitchI = mrt3::internal_pitch(t->nx);
  g.planeI = uint32_t(t->planeI);
  g.link = t->masked ? t->link : nullptr;
  g.wflag = t->masked ? t->wflag : nullptr;
  g.nsx = (t->nx + 63) / 64;
  g.band = mrt3::band_of(t->nx, t->ny);
  return g;
}

// The fields as a 2-D lattice [nz*ny][pitch] for the reduction kernels.
mrt::Geometry flat_geometry(const mrt3_tape* t) {
  mrt::Geometry g{};
  g.nx = t->nx;
  g.ny = t->ny * t->nz;
  g.pitch = t->pitch;
  g.periodic = t->periodic;
  g.plane = t->plane;
  g.masked = t->has_mask;
  g.link = t->has_mask ? t->solid16 : nullptr;
  g.wflag = nullptr;
  g.nsx = (t->nx + 63) / 64;
  return g;
}

template <typename T>
T* slot(const mrt3_tape* t, int k) {
  return reinterpret_cast<T*>(static_cast<char*>(t->rec) + size_t(k) * t->rec_slot_bytes);
}

int last_launch_error() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return failf(MRT_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
  return MRT_OK;
}

struct Span {
  void* h;
  int64_t n = 0;
  Span(int kind, hipStream_t s) : h(mrt::host::span_begin(kind, s)) {}
  ~Span() { mrt::host::span_end(h, n); }
};

// Forward steps [n0, n1) from `src` (null = equilibrium of u0, v0); a step
// closing a segment writes its checkpoint (when write_ckpt).
template <typename T>
int run_forward3(mrt3_tape* t, const mrt3::Model3Coef<T>& m, const mrt3::Geometry3& g, int n0,
                 int n1, const T* src, const T* u0, const T* v0, const T* ctrl, bool record,
                 bool write_ckpt, int kind, hipStream_t s, const T** last) {
  Span span(kind, s);
  const int seg = n0 / t->K;
  for (int n = n0; n < n1; ++n) {
    mrt3::Fwd3Launch<T> a{};
    a.src = src;
    a.u0 = u0;
    a.v0 = v0;
    a.ctrl = ctrl;
    a.rec = record ? slot<T>(t, n - seg * t->K) : nullptr;
    T* dst = static_cast<T*>(t->buf[n & 1]);
    const bool closes = write_ckpt && t->mode == 2 && (n + 1) % t->K == 0 && n + 1 < t->nsteps;
    if (closes) dst = static_cast<T*>(t->ckpt[(n + 1) / t->K]);
    a.dst = dst;
    mrt3::launch_forward3<T>(g, m, a, s);
    ++span.n;
    int rc = last_launch_error();
    if (rc) return rc;
    src = dst;
  }
  *last = src;
  return MRT_OK;
}

template <typename T>
int forward3_impl(const mrt3_problem* p, mrt3_tape* t, const void* u0, const void* v0,
                  const void* control, void* state, void* uN, void* vN, hipStream_t s) {
  const mrt3::Model3Coef<T> m = model_coef3<T>(p);
  const mrt3::Geometry3 g = geometry3(t);
  const int N = t->nsteps;
  const bool adj = t->mode > 0;
  const int last_seg = t->nseg - 1;
  const T* cur = nullptr;
  const T* tu0 = static_cast<const T*>(u0);
  const T* tv0 = static_cast<const T*>(v0);
  const T* tc = static_cast<const T*>(control);
  t->fwd_done = false;
  int rc;
  const int rec_start = adj ? last_seg * t->K : N;
  if (rec_start > 0) {
    rc = run_forward3<T>(t, m, g, 0, rec_start, nullptr, tu0, tv0, tc, false, true, 0, s, &cur);
    if (rc) return rc;
  }
  if (rec_start < N) {
    rc = run_forward3<T>(t, m, g, rec_start, N, cur, tu0, tv0, tc, true, true, 0, s, &cur);
    if (rc) return rc;
  }
  mrt3::launch_finalize3<T>(g, cur, static_cast<T*>(state), static_cast<T*>(uN),
                            static_cast<T*>(vN), s);
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
int rerecord3(const mrt3_problem* p, mrt3_tape* t, const mrt3::Model3Coef<T>& m,
              const mrt3::Geometry3& g, int seg, const T* u0, const T* v0, const T* ctrl,
              hipStream_t s) {
  if (t->rec_seg == seg) return MRT_OK;
  const int n0 = seg * t->K, n1 = std::min(t->nsteps, n0 + t->K);
  const T* src = seg == 0 ? nullptr : static_cast<const T*>(t->ckpt[seg]);
  const T* dummy = nullptr;
  t->rec_seg = -1;
  int rc = run_forward3<T>(t, m, g, n0, n1, src, u0, v0, ctrl, true, false, 2, s, &dummy);
  if (rc) return rc;
  t->rec_seg = seg;
  (void)p;
  return MRT_OK;
}

template <typename T>
int adjoint3_impl(const mrt3_problem* p, mrt3_tape* t, const void* u0, const void* v0,
                  const void* control, const void* seed_u, const void* seed_v, double* gacc,
                  void* adj_u0, void* adj_v0, hipStream_t s) {
  const mrt3::Model3Coef<T> m = model_coef3<T>(p);
  const mrt3::Geometry3 g = geometry3(t);
  const int N = t->nsteps, K = t->K;
  const T* tu0 = static_cast<const T*>(u0);
  const T* tv0 = static_cast<const T*>(v0);
  const T* tc = static_cast<const T*>(control);
  const bool want0 = adj_u0 != nullptr || adj_v0 != nullptr;
  const T* asrc = nullptr;
  for (int seg = t->nseg - 1; seg >= 0; --seg) {
    const int n0 = seg * K, n1 = std::min(N, n0 + K);
    int rc = rerecord3<T>(p, t, m, g, seg, tu0, tv0, tc, s);
    if (rc) return rc;
    Span span(1, s);
    for (int n = n1 - 1; n >= n0; --n) {
      mrt3::Adj3Launch<T> a{};
      a.src = asrc;
      a.first = n == N - 1;
      a.last = (n == 0 && want0) ? 1 : 0;
      a.dst = n == 0 ? nullptr : static_cast<T*>(t->abuf[n & 1]);
      a.seed_u = static_cast<const T*>(seed_u);
      a.seed_v = static_cast<const T*>(seed_v);
      a.rec = slot<T>(t, n - n0);
      a.g = gacc;
      a.adj_u0 = static_cast<T*>(adj_u0);
      a.adj_v0 = static_cast<T*>(adj_v0);
      mrt3::launch_adjoint3<T>(g, m, a, s);
      ++span.n;
      rc = last_launch_error();
      if (rc) return rc;
      asrc = a.dst;
    }
  }
  return MRT_OK;
}

template <typename T>
int tlm3_impl(const mrt3_problem* p, mrt3_tape* t, const void* u0, const void* v0,
              const void* control, const void* dc, const void* du0, const void* dv0, void* duN,
              void* dvN, hipStream_t s) {
  const mrt3::Model3Coef<T> m = model_coef3<T>(p);
  const mrt3::Geometry3 g = geometry3(t);
  const int N = t->nsteps, K = t->K;
  const T* tu0 = static_cast<const T*>(u0);
  const T* tv0 = static_cast<const T*>(v0);
  const T* tc = static_cast<const T*>(control);
  const T* dsrc = nullptr;
  for (int seg = 0; seg < t->nseg; ++seg) {
    const int n0 = seg * K, n1 = std::min(N, n0 + K);
    int rc = rerecord3<T>(p, t, m, g, seg, tu0, tv0, tc, s);
    if (rc) return rc;
    Span span(3, s);
    for (int n = n0; n < n1; ++n) {
      mrt3::Tlm3Launch<T> a{};
      a.src = dsrc;
      a.dst = static_cast<T*>(t->abuf[n & 1]);
      a.du0 = static_cast<const T*>(du0);
      a.dv0 = static_cast<const T*>(dv0);
      a.dc = static_cast<const T*>(dc);
      a.rec = slot<T>(t, n - n0);
      mrt3::launch_tlm3<T>(g, m, a, s);
      ++span.n;
      rc = last_launch_error();
      if (rc) return rc;
      dsrc = a.dst;
    }
  }
  mrt3::launch_finalize3<T>(g, dsrc, nullptr, static_cast<T*>(duN), static_cast<T*>(dvN), s);
  return last_launch_error();
}

int read_result3(mrt3_tape* t, hipStream_t s, int n) {
  HIP_TRY3(hipMemcpyAsync(t->host, t->result, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  HIP_TRY3(hipStreamSynchronize(s));
  return MRT_OK;
}

template <typename T>
int cost3_impl(mrt3_tape* t, double alpha, const void* uN, const void* ut, const void* ctrl,
               const double* gacc, void* seed, void* grad, mrt_scalars* out, hipStream_t s) {
  const mrt::Geometry g = flat_geometry(t);
  mrt::launch_cost_grad<T>(g, static_cast<const T*>(uN), static_cast<const T*>(ut),
                           static_cast<const T*>(ctrl), gacc, static_cast<T*>(seed),
                           static_cast<T*>(grad), alpha, t->partials, t->result, s);
  int rc = last_launch_error();
  if (rc) return rc;
  rc = read_result3(t, s, mrt::kRedSlots);
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
    return failf(MRT_ENONFINITE, "non-finite cost or gradient (%g values)", h[4]);
  return MRT_OK;
}

void free_tape3(mrt3_tape* t) {
  if (!t) return;
  for (void* a : t->allocs) (void)hipFree(a);
  if (t->host) (void)hipHostFree(t->host);
  delete t;
}

int check_recorded(const mrt3_tape* t, const void* u0, const void* v0, const void* control) {
  if (t->mode == 0) return failf(MRT_ESTATE, "tape was created without adjoint record");
  if (!t->fwd_done) return failf(MRT_ESTATE, "no forward solve recorded on this tape");
  if (u0 != t->f_u0 || v0 != t->f_v0 || control != t->f_ctrl)
    return failf(MRT_ESTATE, "u0/v0/control differ from the recorded forward");
  return MRT_OK;
}

}  // namespace

extern "C" {

int mrt3_validate(const mrt3_problem* p) { return validate3(p); }

int mrt3_tape_bytes(const mrt3_problem* p, int32_t ckpt_every, size_t* bytes) {
  int rc = validate3(p);
  if (rc) return rc;
  if (!bytes) return failf(MRT_EINVAL, "bytes is NULL");
  *bytes = plan3(p, ckpt_every).total;
  return MRT_OK;
}

int mrt3_tape_create(const mrt3_problem* p, int32_t ckpt_every, size_t mem_budget,
                     mrt3_tape** out) {
  int rc = validate3(p);
  if (rc) return rc;
  if (!out) return failf(MRT_EINVAL, "out is NULL");
  *out = nullptr;
  const Layout3 L = plan3(p, ckpt_every);
  if (mem_budget > 0 && L.total > mem_budget)
    return failf(MRT_ENOMEM, "tape needs %zu bytes, budget %zu", L.total, mem_budget);
  mrt3_tape* t = new mrt3_tape();
  const mrt3_grid& g = p->grid;
  t->nx = g.nx;
  t->ny = g.ny;
  t->nz = g.nz;
  t->pitch = g.pitch;
  t->nsteps = g.nsteps;
  t->dtype = g.dtype;
  t->periodic = g.periodic;
  t->masked = uses_links(g) ? 1 : 0;
  t->has_mask = g.mask != nullptr ? 1 : 0;
  t->mode = L.mode;
  t->K = L.K;
  t->nseg = L.nseg;
  t->plane = L.plane;
  t->planeI = L.planeI;
  t->elem = L.elem;
  t->state_bytes = L.state_bytes;
  t->rec_slot_bytes = L.rec_slot_bytes;
  t->total_bytes = L.total;
  auto alloc = [&](size_t bytes, void** ptr) -> int {
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return failf(MRT_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    t->allocs.push_back(*ptr);
    return MRT_OK;
  };
  if (hipGetDevice(&t->device) != hipSuccess) {
    delete t;
    return failf(MRT_EHIP, "no HIP device");
  }
  const size_t nwf = size_t(g.nz) * g.ny * ((g.nx + 63) / 64);
  rc = alloc(L.state_bytes, &t->buf[0]);
  if (!rc) rc = alloc(L.state_bytes, &t->buf[1]);
  if (!rc && t->masked) rc = alloc(L.plane * sizeof(uint32_t), (void**)&t->link);
  if (!rc && t->masked) rc = alloc(L.plane * sizeof(uint16_t), (void**)&t->solid16);
  if (!rc && t->masked) rc = alloc(nwf * sizeof(uint32_t), (void**)&t->wflag);
  if (!rc)
    rc = alloc((size_t(mrt::kRedBlocks) * mrt::kRedSlots + 16) * sizeof(double),
               (void**)&t->partials);
  if (!rc && L.mode > 0) {
    rc = alloc(L.state_bytes, &t->abuf[0]);
    if (!rc) rc = alloc(L.state_bytes, &t->abuf[1]);
    t->ckpt.assign(L.nseg, nullptr);
    for (int k = 1; k < L.nseg && !rc; ++k) rc = alloc(L.state_bytes, &t->ckpt[k]);
    if (!rc) rc = alloc(size_t(L.K) * L.rec_slot_bytes, &t->rec);
  }
  if (!rc && hipHostMalloc((void**)&t->host, 16 * sizeof(double)) != hipSuccess)
    rc = failf(MRT_ENOMEM, "hipHostMalloc failed");
  if (rc) {
    free_tape3(t);
    return rc;
  }
  t->result = t->partials + size_t(mrt::kRedBlocks) * mrt::kRedSlots;
  hipStream_t s = nullptr;
  if (t->masked) {
    mrt3::launch_build_link3(geometry3(t), g.mask, t->link, t->wflag, t->solid16, s);
    rc = last_launch_error();
  }
  if (!rc) {
    mrt::launch_count_fluid(flat_geometry(t), t->partials, t->result, s);
    rc = last_launch_error();
  }
  if (!rc) rc = read_result3(t, s, 1);
  if (rc) {
    free_tape3(t);
    return rc;
  }
  t->n_fluid = int64_t(t->host[0]);
  *out = t;
  return MRT_OK;
}

void mrt3_tape_destroy(mrt3_tape* t) {
  if (!t) return;
  (void)hipDeviceSynchronize();
  free_tape3(t);
}

int mrt3_tape_query(const mrt3_tape* t, mrt_tape_info* info) {
  if (!t || !info) return failf(MRT_EINVAL, "NULL argument");
  info->mode = t->mode;
  info->ckpt_every = t->K;
  info->n_segments = t->nseg;
  info->reserved = 0;
  info->n_fluid = t->n_fluid;
  info->device_bytes = t->total_bytes;
  return MRT_OK;
}

int mrt3_forward(const mrt3_problem* p, mrt3_tape* t, const void* u0, const void* v0,
                 const void* control, void* state, void* uN, void* vN, void* stream) {
  int rc = validate3(p);
  if (rc) return rc;
  rc = check_tape3(p, t);
  if (rc) return rc;
  if (!u0 || !v0 || !control) return failf(MRT_EINVAL, "u0, v0, control required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return p->grid.dtype == MRT_F64
             ? forward3_impl<double>(p, t, u0, v0, control, state, uN, vN, s)
             : forward3_impl<float>(p, t, u0, v0, control, state, uN, vN, s);
}

int amrt3_adjoint(const mrt3_problem* p, mrt3_tape* t, const void* u0, const void* v0,
                  const void* control, const void* seed_u, const void* seed_v,
                  double* grad_accum, void* adj_u0, void* adj_v0, void* stream) {
  int rc = validate3(p);
  if (rc) return rc;
  rc = check_tape3(p, t);
  if (rc) return rc;
  rc = check_recorded(t, u0, v0, control);
  if (rc) return rc;
  if (!seed_u || !grad_accum) return failf(MRT_EINVAL, "seed_u and grad_accum required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return p->grid.dtype == MRT_F64
             ? adjoint3_impl<double>(p, t, u0, v0, control, seed_u, seed_v, grad_accum, adj_u0,
                                     adj_v0, s)
             : adjoint3_impl<float>(p, t, u0, v0, control, seed_u, seed_v, grad_accum, adj_u0,
                                    adj_v0, s);
}

int mrt3_tlm(const mrt3_problem* p, mrt3_tape* t, const void* u0, const void* v0,
             const void* control, const void* dc, const void* du0, const void* dv0, void* duN,
             void* dvN, void* stream) {
  int rc = validate3(p);
  if (rc) return rc;
  rc = check_tape3(p, t);
  if (rc) return rc;
  rc = check_recorded(t, u0, v0, control);
  if (rc) return rc;
  if (!duN && !dvN) return failf(MRT_EINVAL, "duN or dvN required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return p->grid.dtype == MRT_F64
             ? tlm3_impl<double>(p, t, u0, v0, control, dc, du0, dv0, duN, dvN, s)
             : tlm3_impl<float>(p, t, u0, v0, control, dc, du0, dv0, duN, dvN, s);
}

int mrt3_cost_gradient(const mrt3_problem* p, mrt3_tape* t, const void* uN,
                       const void* u_target, const void* control, const double* grad_accum,
                       void* seed_out, void* grad_out, mrt_scalars* out, void* stream) {
  int rc = validate3(p);
  if (rc) return rc;
  rc = check_tape3(p, t);
  if (rc) return rc;
  if (!uN || !u_target || !control) return failf(MRT_EINVAL, "uN, u_target, control required");
  if (grad_accum && !grad_out) return failf(MRT_EINVAL, "grad_out required with grad_accum");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return p->grid.dtype == MRT_F64
             ? cost3_impl<double>(t, p->alpha, uN, u_target, control, grad_accum, seed_out,
                                  grad_out, out, s)
             : cost3_impl<float>(t, p->alpha, uN, u_target, control, grad_accum, seed_out,
                                 grad_out, out, s);
}

int mrt3_gd_step(const mrt3_problem* p, mrt3_tape* t, void* control, const void* grad,
                 double zeta, double lo, double hi, double* zeta_used, void* stream) {
  int rc = validate3(p);
  if (rc) return rc;
  rc = check_tape3(p, t);
  if (rc) return rc;
  if (!control || !grad) return failf(MRT_EINVAL, "control and grad required");
  if (std::isnan(zeta) || std::isnan(lo) || std::isnan(hi) || lo > hi)
    return failf(MRT_EINVAL, "invalid zeta or bounds");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const mrt::Geometry g = flat_geometry(t);
  if (p->grid.dtype == MRT_F64)
    mrt::launch_gd_step<double>(g, static_cast<double*>(control),
                                static_cast<const double*>(grad), zeta, lo, hi, t->partials,
                                t->result, s);
  else
    mrt::launch_gd_step<float>(g, static_cast<float*>(control), static_cast<const float*>(grad),
                               zeta, lo, hi, t->partials, t->result, s);
  rc = last_launch_error();
  if (rc) return rc;
  if (zeta_used) {
    HIP_TRY3(hipMemcpyAsync(t->host + mrt::kRedSlots, t->result + mrt::kRedSlots,
                            sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY3(hipStreamSynchronize(s));
    *zeta_used = t->host[mrt::kRedSlots];
    if (!std::isfinite(*zeta_used))
      return failf(MRT_ENONFINITE, "non-finite step (gradient not finite)");
  }
  return MRT_OK;
}

}  // extern "C"
