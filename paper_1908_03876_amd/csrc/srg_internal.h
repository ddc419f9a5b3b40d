// Internal interface of the surrogate kernels (srg_kernels.hip) and their
// runtime (mrt_srg.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mrt {

template <int CIN, int COUT>
void launch_conv_fwd(const float* x, const uint16_t* w, const float* b, float* y,
                     int B, int H, int W, float iscale, float oscale, bool act,
                     hipStream_t s);
template <int CIN, int COUT>
void launch_conv_bwd(const float* dz, const float* x, const uint16_t* w, float* dx,
                     float* dw, float* db, int B, int H, int W, float iscale,
                     float oscale, hipStream_t s);
void launch_tanh_bwd(const float* y, const float* dy, float* dz, size_t n, hipStream_t s);
void launch_mse(const float* pred, const float* t, float* dpred, double* partials,
                double* out, int B, int H, int W, int border, hipStream_t s);
int mse_partials_needed(int B, int H, int W);
void launch_adam(float* w, uint16_t* wb, const float* g, float* m, float* v, int n,
                 float lr, float b1, float b2, float eps, float c1, float c2,
                 hipStream_t s);
void launch_to_bf16(const float* w, uint16_t* wb, int n, hipStream_t s);
void launch_gather_crops(const float* src, int L, const int* idx, const int* oy,
                         const int* ox, const float* sub, float* out, int n, int h, int w,
                         hipStream_t s);

// Step sizes of the candidate controls c - lambda_k E (kernel argument).
constexpr int kSrgMaxSteps = 32;
struct SrgSteps {
  float v[kSrgMaxSteps];
};

// Per-field surrogate cost J_b = 1/2 |u_base + y_b - u_target|^2 +
// alpha/2 |x_b|^2 into out[b] (double); y is overwritten by the residual.
void launch_objective(float* y, const float* ub, const float* ut, const float* x,
                      double* partials, double* out, int B, int H, int W, float alpha,
                      hipStream_t s);
int objective_partials_needed(int B, int H, int W);
void launch_axpy(float* dx, const float* x, float alpha, size_t n, hipStream_t s);
void launch_candidates(const float* c, const float* E, const SrgSteps& lam, int n, size_t hw,
                       float* X, hipStream_t s);

}  // namespace mrt
