// Runtime of the convolutional surrogate: parameter storage (FP32 masters,
// BF16 compute copies, Adam moments), the four-layer forward and backward
// sequence, the training step and input gradients.  See include/mrt.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "mrt.h"
#include "mrt_internal.h"
#include "srg_internal.h"

namespace {

constexpr int kC = 32;  // hidden channels

int err(int code, const std::string& m) { return mrt::host::set_error(code, m.c_str()); }

#define HIP_OK(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      return err(MRT_EHIP, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
  } while (0)

struct Layer {
  int cin = 0, cout = 0;
  float* w = nullptr;      // FP32 master [cout][cin][9]
  uint16_t* wb = nullptr;  // BF16 compute copy [cout][cin][9] (one-channel layers)
  uint16_t* wf = nullptr;  // MFMA fragments, forward and transposed (32 x 32 layers)
  uint16_t* wt = nullptr;
  float* b = nullptr;      // [cout]
  float* dw = nullptr;
  float* db = nullptr;
  float* mw = nullptr;
  float* vw = nullptr;
  float* mb = nullptr;
  float* vb = nullptr;
  int nw() const { return cin * cout * 9; }
};

}  // namespace

struct mrt_srg {
  int max_batch = 0, max_h = 0, max_w = 0;
  float s_in = 1.f, s_out = 1.f;
  Layer L[4];
  uint16_t* act[3] = {nullptr, nullptr, nullptr};  // BF16 [B][H][W][32]
  uint16_t* g[2] = {nullptr, nullptr};             // BF16 [B][H][W][32]
  float* wpart = nullptr;                          // weight-gradient partials
  double* tpart = nullptr;
  float* dout = nullptr;
  float* xbuf = nullptr;    // step candidates [n][H][W]
  float* wm = nullptr;      // warm start: Adam moments and input gradient,
  float* wv = nullptr;      // max_h * max_w each
  float* wg = nullptr;
  double* partials = nullptr;
  double* loss_dev = nullptr;
  double* obj_dev = nullptr;  // per-field objectives [kSrgMaxSteps]
  double* bbpart = nullptr;   // warm start: Barzilai-Borwein partials and state
  double* bbst = nullptr;
  double* host = nullptr;     // pinned [kSrgMaxSteps + 8]
  int64_t step = 0;
  std::vector<void*> allocs;
};

namespace {

int check_shape(const mrt_srg* s, int B, int H, int W) {
  // work buffers hold max_batch * max_h * max_w pixels
  if (B < 1 || H < 3 || W < 3 ||
      size_t(B) * H * W > size_t(s->max_batch) * s->max_h * s->max_w)
    return err(MRT_EINVAL, "batch or size outside what the surrogate was created for");
  // the convolution kernels address a row of 64-byte pixels with 32-bit offsets
  if (W > (1 << 24)) return err(MRT_EINVAL, "at most 2^24 pixels per row");
  return MRT_OK;
}

int launch_err() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MRT_OK
                         : err(MRT_EHIP, std::string("launch failed: ") + hipGetErrorString(e));
}

void forward(mrt_srg* s, const float* x, float* y, int B, int H, int W, hipStream_t st) {
  mrt::launch_srg_l0_fwd(x, s->L[0].wb, s->L[0].b, s->act[0], B, H, W, s->s_in, st);
  mrt::launch_srg_c32_fwd(s->act[0], s->L[1].wf, s->L[1].b, s->act[1], B, H, W, st);
  mrt::launch_srg_c32_fwd(s->act[1], s->L[2].wf, s->L[2].b, s->act[2], B, H, W, st);
  mrt::launch_srg_l3_fwd(s->act[2], s->L[3].wb, s->L[3].b, y, B, H, W, s->s_out, st);
}

// Backward through the layers of the last forward on x, from dy = dL/dy.
void backward(mrt_srg* s, const float* x, const float* dy, float* dx, bool wgrads, int B,
              int H, int W, hipStream_t st) {
  uint16_t* g0 = s->g[0];
  uint16_t* g1 = s->g[1];
  // layer 3 (32 -> 1): dz2 with the tanh of layer 2 folded in
  mrt::launch_srg_l3_bwd_data(dy, s->L[3].wb, s->act[2], g0, B, H, W, s->s_out, st);
  if (wgrads)
    mrt::launch_srg_thin_wgrad(s->act[2], dy, -1, s->tpart, B, H, W, s->s_out, s->s_out, 0,
                               s->L[3].dw, s->L[3].db, st);
  // layer 2 (32 -> 32)
  if (wgrads)
    mrt::launch_srg_c32_bwd_weight(g0, s->act[1], s->wpart, s->L[2].dw, s->L[2].db, B, H, W, st);
  mrt::launch_srg_c32_bwd_data(g0, s->L[2].wt, s->act[1], g1, B, H, W, st);
  // layer 1 (32 -> 32)
  if (wgrads)
    mrt::launch_srg_c32_bwd_weight(g1, s->act[0], s->wpart, s->L[1].dw, s->L[1].db, B, H, W, st);
  mrt::launch_srg_c32_bwd_data(g1, s->L[1].wt, s->act[0], g0, B, H, W, st);
  // layer 0 (1 -> 32)
  if (dx) mrt::launch_srg_l0_bwd_data(g0, s->L[0].wb, dx, B, H, W, s->s_in, st);
  if (wgrads)
    mrt::launch_srg_thin_wgrad(g0, x, 1, s->tpart, B, H, W, s->s_in, 1.f, 1, s->L[0].dw,
                               s->L[0].db, st);
}

// BF16 compute copies of the FP32 masters.
void refresh_weights(mrt_srg* s, hipStream_t st) {
  for (int l = 0; l < 4; ++l) {
    Layer& y = s->L[l];
    if (y.wf)
      mrt::launch_srg_pack(y.w, y.wf, y.wt, st);
    else
      mrt::launch_to_bf16(y.w, y.wb, y.nw(), st);
  }
}

// Surrogate cost of B fields x (and, when dx is given, its gradient
// S'(x)^T r + alpha x) into s->obj_dev[0..B).
void objective(mrt_srg* s, const float* x, const float* ub, const float* ut, float alpha,
               int B, int H, int W, float* dx, hipStream_t st) {
  float* y = s->dout;
  forward(s, x, y, B, H, W, st);
  mrt::launch_objective(y, ub, ut, x, s->partials, s->obj_dev, B, H, W, alpha, st);
  if (dx) {
    backward(s, x, y, dx, false, B, H, W, st);
    mrt::launch_axpy(dx, x, alpha, size_t(B) * H * W, st);
  }
}

int read_objectives(mrt_srg* s, int n, double* J, hipStream_t st) {
  HIP_OK(hipMemcpyAsync(s->host, s->obj_dev, size_t(n) * 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  for (int i = 0; i < n; ++i) {
    J[i] = s->host[i];
    if (!std::isfinite(J[i])) return err(MRT_ENONFINITE, "non-finite surrogate cost");
  }
  return MRT_OK;
}

void free_srg(mrt_srg* s) {
  if (!s) return;
  for (void* p : s->allocs) (void)hipFree(p);
  if (s->host) (void)hipHostFree(s->host);
  delete s;
}

}  // namespace

extern "C" {

int mrt_srg_create(int32_t channels, int32_t max_batch, int32_t max_h, int32_t max_w,
                   float in_scale, float out_scale, mrt_srg** out) {
  if (!out) return err(MRT_EINVAL, "out is NULL");
  *out = nullptr;
  if (channels != kC) return err(MRT_EINVAL, "the surrogate has 32 hidden channels");
  if (max_batch < 1 || max_h < 3 || max_w < 3) return err(MRT_EINVAL, "invalid sizes");
  if (size_t(max_batch) * size_t(max_h) * size_t(max_w) > (size_t(1) << 28))
    return err(MRT_EINVAL, "at most 2^28 pixels (batch x height x width)");
  if (!(std::isfinite(in_scale) && std::isfinite(out_scale)))
    return err(MRT_EINVAL, "non-finite scales");
  mrt_srg* s = new mrt_srg();
  s->max_batch = max_batch;
  s->max_h = max_h;
  s->max_w = max_w;
  s->s_in = in_scale;
  s->s_out = out_scale;
  const int cin[4] = {1, kC, kC, kC}, cout[4] = {kC, kC, kC, 1};
  int rc = MRT_OK;
  auto alloc = [&](size_t bytes, void** p) -> int {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return err(MRT_ENOMEM, "hipMalloc failed");
    }
    s->allocs.push_back(*p);
    return hipMemset(*p, 0, bytes) == hipSuccess ? MRT_OK : err(MRT_EHIP, "hipMemset failed");
  };
  for (int l = 0; l < 4 && !rc; ++l) {
    Layer& y = s->L[l];
    y.cin = cin[l];
    y.cout = cout[l];
    const size_t nw = size_t(y.nw()) * 4, nb = size_t(y.cout) * 4;
    rc = alloc(nw, (void**)&y.w);
    if (y.cin == kC && y.cout == kC) {
      if (!rc) rc = alloc(nw / 2, (void**)&y.wf);
      if (!rc) rc = alloc(nw / 2, (void**)&y.wt);
    } else if (!rc) {
      rc = alloc(nw / 2, (void**)&y.wb);
    }
    if (!rc) rc = alloc(nb, (void**)&y.b);
    if (!rc) rc = alloc(nw, (void**)&y.dw);
    if (!rc) rc = alloc(nb, (void**)&y.db);
    if (!rc) rc = alloc(nw, (void**)&y.mw);
    if (!rc) rc = alloc(nw, (void**)&y.vw);
    if (!rc) rc = alloc(nb, (void**)&y.mb);
    if (!rc) rc = alloc(nb, (void**)&y.vb);
  }
  const size_t hwb = size_t(max_batch) * max_h * max_w;
  for (int i = 0; i < 3 && !rc; ++i) rc = alloc(hwb * kC * 2, (void**)&s->act[i]);
  for (int i = 0; i < 2 && !rc; ++i) rc = alloc(hwb * kC * 2, (void**)&s->g[i]);
  if (!rc) rc = alloc(size_t(mrt::kSrgWBlocks) * mrt::kSrgWPart * 4, (void**)&s->wpart);
  if (!rc) rc = alloc(mrt::kSrgThinPartDoubles * 8, (void**)&s->tpart);
  if (!rc) rc = alloc(hwb * 4, (void**)&s->dout);
  if (!rc) rc = alloc(hwb * 4, (void**)&s->xbuf);
  const size_t hw1 = size_t(max_h) * max_w;
  if (!rc) rc = alloc(hw1 * 4, (void**)&s->wm);
  if (!rc) rc = alloc(hw1 * 4, (void**)&s->wv);
  if (!rc) rc = alloc(hw1 * 4, (void**)&s->wg);
  // MSE: one partial per 256 pixels; objectives: per field, rounded up
  if (!rc) rc = alloc((size_t(mrt::mse_partials_needed(max_batch, max_h, max_w)) +
                       mrt::kSrgMaxSteps + 8) * 8,
                      (void**)&s->partials);
  if (!rc) rc = alloc(64, (void**)&s->loss_dev);
  if (!rc) rc = alloc(mrt::kSrgMaxSteps * 8, (void**)&s->obj_dev);
  if (!rc) rc = alloc(size_t(mrt::kSrgBBBlocks) * 3 * 8, (void**)&s->bbpart);
  if (!rc) rc = alloc(8 * 8, (void**)&s->bbst);
  if (!rc && hipHostMalloc((void**)&s->host, (mrt::kSrgMaxSteps + 8) * 8) != hipSuccess)
    rc = err(MRT_ENOMEM, "pinned");
  if (rc) {
    free_srg(s);
    return rc;
  }
  *out = s;
  return MRT_OK;
}

void mrt_srg_destroy(mrt_srg* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  free_srg(s);
}

int mrt_srg_param(mrt_srg* s, int32_t layer, int32_t kind, void** ptr, int64_t* count) {
  if (!s || !ptr || layer < 0 || layer > 3 || kind < 0 || kind > 3)
    return err(MRT_EINVAL, "invalid parameter query");
  Layer& y = s->L[layer];
  float* p[4] = {y.w, y.b, y.dw, y.db};
  const int64_t n[4] = {y.nw(), y.cout, y.nw(), y.cout};
  *ptr = p[kind];
  if (count) *count = n[kind];
  return MRT_OK;
}

int mrt_srg_copy_param(mrt_srg* s, int32_t layer, int32_t kind, int32_t to_srg,
                       void* data, void* stream) {
  void* p = nullptr;
  int64_t n = 0;
  int rc = mrt_srg_param(s, layer, kind, &p, &n);
  if (rc) return rc;
  if (!data) return err(MRT_EINVAL, "data is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (to_srg)
    HIP_OK(hipMemcpyAsync(p, data, size_t(n) * 4, hipMemcpyDeviceToDevice, st));
  else
    HIP_OK(hipMemcpyAsync(data, p, size_t(n) * 4, hipMemcpyDeviceToDevice, st));
  return MRT_OK;
}

int mrt_srg_sync(mrt_srg* s, void* stream) {
  if (!s) return err(MRT_EINVAL, "surrogate is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  refresh_weights(s, st);
  for (int l = 0; l < 4; ++l) {
    Layer& y = s->L[l];
    HIP_OK(hipMemsetAsync(y.mw, 0, size_t(y.nw()) * 4, st));
    HIP_OK(hipMemsetAsync(y.vw, 0, size_t(y.nw()) * 4, st));
    HIP_OK(hipMemsetAsync(y.mb, 0, size_t(y.cout) * 4, st));
    HIP_OK(hipMemsetAsync(y.vb, 0, size_t(y.cout) * 4, st));
  }
  s->step = 0;
  return launch_err();
}

int mrt_srg_forward(mrt_srg* s, const float* x, float* y, int32_t B, int32_t H, int32_t W,
                    void* stream) {
  if (!s || !x || !y) return err(MRT_EINVAL, "NULL argument");
  int rc = check_shape(s, B, H, W);
  if (rc) return rc;
  forward(s, x, y, B, H, W, static_cast<hipStream_t>(stream));
  return launch_err();
}

int mrt_srg_backward(mrt_srg* s, const float* x, const float* dy, float* dx,
                     int32_t weight_grads, int32_t B, int32_t H, int32_t W, void* stream) {
  if (!s || !x || !dy) return err(MRT_EINVAL, "NULL argument");
  int rc = check_shape(s, B, H, W);
  if (rc) return rc;
  backward(s, x, dy, dx, weight_grads != 0, B, H, W, static_cast<hipStream_t>(stream));
  return launch_err();
}

int mrt_srg_loss(mrt_srg* s, const float* x, const float* target, int32_t B, int32_t H,
                 int32_t W, int32_t border, double* loss, void* stream) {
  if (!s || !x || !target || !loss) return err(MRT_EINVAL, "NULL argument");
  int rc = check_shape(s, B, H, W);
  if (rc) return rc;
  if (border < 0 || 2 * border >= H || 2 * border >= W) return err(MRT_EINVAL, "bad border");
  hipStream_t st = static_cast<hipStream_t>(stream);
  forward(s, x, s->dout, B, H, W, st);
  mrt::launch_mse(s->dout, target, nullptr, s->partials, s->loss_dev, B, H, W, border, st);
  rc = launch_err();
  if (rc) return rc;
  HIP_OK(hipMemcpyAsync(s->host, s->loss_dev, 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  *loss = s->host[0];
  return std::isfinite(*loss) ? MRT_OK : err(MRT_ENONFINITE, "non-finite loss");
}

int mrt_srg_train_step(mrt_srg* s, const float* x, const float* target, int32_t B,
                       int32_t H, int32_t W, int32_t border, float lr, double* loss,
                       void* stream) {
  if (!s || !x || !target) return err(MRT_EINVAL, "NULL argument");
  int rc = check_shape(s, B, H, W);
  if (rc) return rc;
  if (border < 0 || 2 * border >= H || 2 * border >= W) return err(MRT_EINVAL, "bad border");
  if (!(lr > 0.f)) return err(MRT_EINVAL, "lr must be > 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* pred = s->dout;  // prediction, then overwritten by dL/dpred
  forward(s, x, pred, B, H, W, st);
  mrt::launch_mse(pred, target, pred, s->partials, s->loss_dev, B, H, W, border, st);
  backward(s, x, pred, nullptr, true, B, H, W, st);
  s->step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - std::pow(b1, float(s->step)), c2 = 1.f - std::pow(b2, float(s->step));
  mrt::SrgAdamTable tab{};
  for (int l = 0; l < 4; ++l) {
    Layer& y = s->L[l];
    tab.g[tab.n++] = {y.w, y.dw, y.mw, y.vw, y.wb, y.wf, y.wt, y.nw()};
    tab.g[tab.n++] = {y.b, y.db, y.mb, y.vb, nullptr, nullptr, nullptr, y.cout};
  }
  mrt::launch_adam_all(tab, lr, b1, b2, eps, c1, c2, st);
  rc = launch_err();
  if (rc) return rc;
  if (loss) {
    HIP_OK(hipMemcpyAsync(s->host, s->loss_dev, 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    *loss = s->host[0];
    if (!std::isfinite(*loss)) return err(MRT_ENONFINITE, "non-finite loss");
  }
  return MRT_OK;
}

int mrt_srg_gather(const float* src, int32_t L, const int32_t* idx, const int32_t* oy,
                   const int32_t* ox, const float* sub, float* out, int32_t n, int32_t h,
                   int32_t w, void* stream) {
  if (!src || !idx || !oy || !ox || !out || L < 1 || n < 1 || h < 1 || w < 1 || h > L || w > L)
    return err(MRT_EINVAL, "invalid crop request");
  mrt::launch_gather_crops(src, L, idx, oy, ox, sub, out, n, h, w,
                           static_cast<hipStream_t>(stream));
  return launch_err();
}

int mrt_srg_objective(mrt_srg* s, const float* x, const float* u_base, const float* u_target,
                      double alpha, int32_t B, int32_t H, int32_t W, double* J, float* dx,
                      void* stream) {
  if (!s || !x || !u_base || !u_target) return err(MRT_EINVAL, "NULL argument");
  int rc = check_shape(s, B, H, W);
  if (rc) return rc;
  if (B > mrt::kSrgMaxSteps) return err(MRT_EINVAL, "at most 32 fields per objective call");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return err(MRT_EINVAL, "alpha must be >= 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  objective(s, x, u_base, u_target, float(alpha), B, H, W, dx, st);
  rc = launch_err();
  if (rc || !J) return rc;
  return read_objectives(s, B, J, st);
}

int mrt_srg_score_steps(mrt_srg* s, const float* c, const float* E, const double* lambdas,
                        int32_t n, const float* u_base, const float* u_target, double alpha,
                        int32_t H, int32_t W, double* J, void* stream) {
  if (!s || !c || !E || !lambdas || !u_base || !u_target || !J)
    return err(MRT_EINVAL, "NULL argument");
  if (n < 1 || n > mrt::kSrgMaxSteps) return err(MRT_EINVAL, "1..32 step candidates");
  int rc = check_shape(s, n, H, W);
  if (rc) return rc;
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return err(MRT_EINVAL, "alpha must be >= 0");
  mrt::SrgSteps lam{};
  for (int k = 0; k < n; ++k) {
    if (!std::isfinite(lambdas[k])) return err(MRT_EINVAL, "non-finite step size");
    lam.v[k] = float(lambdas[k]);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t hw = size_t(H) * W;
  mrt::launch_candidates(c, E, lam, n, hw, s->xbuf, st);
  objective(s, s->xbuf, u_base, u_target, float(alpha), n, H, W, nullptr, st);
  rc = launch_err();
  if (rc) return rc;
  return read_objectives(s, n, J, st);
}

int mrt_srg_warm_start(mrt_srg* s, const float* u_base, const float* u_target, double alpha,
                       int32_t H, int32_t W, int32_t iters, float lr, float* c,
                       void* stream) {
  if (!s || !u_base || !u_target || !c) return err(MRT_EINVAL, "NULL argument");
  int rc = check_shape(s, 1, H, W);
  if (rc) return rc;
  if (size_t(H) * W > size_t(s->max_h) * s->max_w)
    return err(MRT_EINVAL, "warm start field larger than max_h x max_w");
  if (iters < 0 || !(lr > 0.f)) return err(MRT_EINVAL, "iters >= 0 and lr > 0 required");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return err(MRT_EINVAL, "alpha must be >= 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t hw = size_t(H) * W;
  HIP_OK(hipMemsetAsync(s->wm, 0, hw * 4, st));
  HIP_OK(hipMemsetAsync(s->wv, 0, hw * 4, st));
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int k = 1; k <= iters; ++k) {
    objective(s, c, u_base, u_target, float(alpha), 1, H, W, s->wg, st);
    const float c1 = 1.f - std::pow(b1, float(k)), c2 = 1.f - std::pow(b2, float(k));
    mrt::launch_adam(c, nullptr, s->wg, s->wm, s->wv, int(hw), lr, b1, b2, eps, c1, c2, st);
  }
  return launch_err();
}

int mrt_srg_warm_start_bb(mrt_srg* s, const float* u_base, const float* u_target,
                          double alpha, int32_t H, int32_t W, int32_t iters, float step0,
                          float* c, void* stream) {
  if (!s || !u_base || !u_target || !c) return err(MRT_EINVAL, "NULL argument");
  int rc = check_shape(s, 1, H, W);
  if (rc) return rc;
  if (size_t(H) * W > size_t(s->max_h) * s->max_w)
    return err(MRT_EINVAL, "warm start field larger than max_h x max_w");
  if (iters < 0 || !(step0 > 0.f) || !std::isfinite(step0))
    return err(MRT_EINVAL, "iters >= 0 and a finite step0 > 0 required");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return err(MRT_EINVAL, "alpha must be >= 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t hw = size_t(H) * W;
  float *cp = s->wm, *gp = s->wv, *g = s->wg, *best = s->xbuf;
  for (int k = 0; k < iters; ++k) {
    objective(s, c, u_base, u_target, float(alpha), 1, H, W, g, st);
    mrt::launch_bb_step(c, cp, g, gp, hw, s->bbpart, step0, k == 0 ? 1 : 0, s->obj_dev, s->bbst,
                        st);
    mrt::launch_bb_update(c, cp, g, gp, best, s->bbst, hw, st);
  }
  if (iters > 0) {
    objective(s, c, u_base, u_target, float(alpha), 1, H, W, nullptr, st);
    mrt::launch_bb_final(c, best, s->bbst, s->obj_dev, hw, st);
  }
  return launch_err();
}

}  // extern "C"
