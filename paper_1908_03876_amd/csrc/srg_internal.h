// Internal interface of the surrogate kernels (srg_kernels.hip) and their
// runtime (mrt_srg.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mrt {

// Sizes of the reduction scratch of the weight gradients.
constexpr int kSrgWPart = 32 * 32 * 9 + 32;  // one block partial: dW, db
constexpr int kSrgWBlocks = 256;             // max blocks of the MFMA weight gradient
constexpr int kSrgThinBlocks = 1024;         // max blocks of the thin ones
constexpr size_t kSrgThinPartDoubles = size_t(11) * kSrgThinBlocks * 32 + kSrgThinBlocks;

// Hidden activations and gradients are BF16 channels-last [B][H][W][32].
void launch_srg_l0_fwd(const float* x, const uint16_t* w, const float* b, uint16_t* out, int B,
                       int H, int W, float iscale, hipStream_t s);
void launch_srg_l0_bwd_data(const uint16_t* dz, const uint16_t* w, float* dx, int B, int H,
                            int W, float iscale, hipStream_t s);
void launch_srg_l3_fwd(const uint16_t* a, const uint16_t* w, const float* b, float* y, int B,
                       int H, int W, float oscale, hipStream_t s);
void launch_srg_l3_bwd_data(const float* dy, const uint16_t* w, const uint16_t* a, uint16_t* dz,
                            int B, int H, int W, float oscale, hipStream_t s);
// dw[c][t] = scale sum_p F[p][c] S[p + sgn off(t)]; db per channel
// (bscale sum F) or single (bscale sum S).
void launch_srg_thin_wgrad(const uint16_t* F, const float* S, int sgn, double* part, int B,
                           int H, int W, float scale, float bscale, int bias_per_channel,
                           float* dw, float* db, hipStream_t s);
// MFMA weight fragments (forward and transposed) of a 32 x 32 layer.
void launch_srg_pack(const float* w, uint16_t* fwd, uint16_t* bwd, hipStream_t s);
void launch_srg_c32_fwd(const uint16_t* in, const uint16_t* wf, const float* b, uint16_t* out,
                        int B, int H, int W, hipStream_t s);
void launch_srg_c32_bwd_data(const uint16_t* dz, const uint16_t* wt, const uint16_t* aprev,
                             uint16_t* dzprev, int B, int H, int W, hipStream_t s);
// part: kSrgWBlocks * kSrgWPart floats
void launch_srg_c32_bwd_weight(const uint16_t* dz, const uint16_t* a, float* part, float* dw,
                               float* db, int B, int H, int W, hipStream_t s);
void launch_mse(const float* pred, const float* t, float* dpred, double* partials,
                double* out, int B, int H, int W, int border, hipStream_t s);
int mse_partials_needed(int B, int H, int W);
void launch_adam(float* w, uint16_t* wb, const float* g, float* m, float* v, int n,
                 float lr, float b1, float b2, float eps, float c1, float c2,
                 hipStream_t s);
void launch_to_bf16(const float* w, uint16_t* wb, int n, hipStream_t s);
// Adam on every parameter group in one launch, with the compute copies
// (BF16 weights of the one-channel layers, MFMA fragments of the 32 x 32
// layers) written from the updated masters.
struct SrgAdamGroup {
  float* w;
  const float* grad;
  float* m;
  float* v;
  uint16_t* wb;  // BF16 copy [n], or null
  uint16_t* wf;  // MFMA fragments of a 32 x 32 layer (n = 32 * 32 * 9), or null
  uint16_t* wt;
  int n;
};
struct SrgAdamTable {
  SrgAdamGroup g[8];
  int n;
};
void launch_adam_all(const SrgAdamTable& tab, float lr, float b1, float b2, float eps, float c1,
                     float c2, hipStream_t s);
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

// Barzilai-Borwein warm start: the step of an iteration into st[0] (from
// the iterate c, its gradient g and the previous ones cp, gp; eta0 / RMS(g)
// when first), with the best cost seen (st[2], J[0] being the cost at c)
// and its flag (st[1]); then the update (best, cp, gp, c), and at the end
// c <- best if that is better.  part: kSrgBBBlocks * 3 doubles.
constexpr int kSrgBBBlocks = 512;
void launch_bb_step(const float* c, const float* cp, const float* g, const float* gp, size_t n,
                    double* part, float eta0, int first, const double* J, double* st,
                    hipStream_t s);
void launch_bb_update(float* c, float* cp, const float* g, float* gp, float* best,
                      const double* st, size_t n, hipStream_t s);
void launch_bb_final(float* c, const float* best, const double* st, const double* J, size_t n,
                     hipStream_t s);

}  // namespace mrt
