// Kernels of the convolutional surrogate of the control-to-state map
// c -> u(T): four periodic 3x3 convolution layers (1 -> C -> C -> C -> 1
// channels), tanh between layers, BF16 weights with FP32 accumulation, MSE
// loss and Adam.  The surrogate only proposes warm starts and step sizes;
// the MRT solve still decides whether each proposed step is accepted.
//
// Layout: activations NCHW float [B][C][H][W], weights [Cout][Cin][3][3]
// (BF16 compute copy of an FP32 master), periodic padding.  A layer
// computes z = oscale * (W * (iscale * x) + b).
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include "srg_internal.h"

namespace mrt {
namespace {

constexpr int kB = 256;

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(uint32_t(h) << 16);
}

// round to nearest even
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t(u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

__device__ __forceinline__ int wrap(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Forward: one thread per output pixel, all COUT channels in registers;
// the layer's weights are staged once per block in LDS as FP32.
template <int CIN, int COUT, bool TANH>
__global__ __launch_bounds__(kB) void conv_fwd_kernel(
    const float* __restrict__ x, const uint16_t* __restrict__ w,
    const float* __restrict__ bias, float* __restrict__ y, int B, int H, int W,
    float iscale, float oscale) {
  __shared__ float sw[COUT * CIN * 9];
  for (int i = threadIdx.x; i < COUT * CIN * 9; i += kB) sw[i] = bf16_to_f32(w[i]);
  __syncthreads();
  const size_t hw = size_t(H) * W;
  const size_t p = size_t(blockIdx.x) * kB + threadIdx.x;
  if (p >= size_t(B) * hw) return;
  const int b = int(p / hw);
  const int r = int(p % hw);
  const int py = r / W, px = r % W;
  float acc[COUT];
#pragma unroll
  for (int co = 0; co < COUT; ++co) acc[co] = bias[co];
  const float* xb = x + size_t(b) * CIN * hw;
  for (int ci = 0; ci < CIN; ++ci) {
    const float* xc = xb + size_t(ci) * hw;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int yy = wrap(py + t / 3 - 1, H), xx = wrap(px + t % 3 - 1, W);
      const float v = iscale * xc[size_t(yy) * W + xx];
#pragma unroll
      for (int co = 0; co < COUT; ++co) acc[co] += sw[(co * CIN + ci) * 9 + t] * v;
    }
  }
  float* yb = y + size_t(b) * COUT * hw + r;
#pragma unroll
  for (int co = 0; co < COUT; ++co) {
    float z = oscale * acc[co];
    if (TANH) z = tanhf(z);
    yb[size_t(co) * hw] = z;
  }
}

// dz = dy * (1 - y^2) for a tanh output y (in place on dy allowed).
__global__ __launch_bounds__(kB) void tanh_bwd_kernel(const float* __restrict__ y,
                                                     const float* dy, float* dz,
                                                     size_t n) {
  const size_t i = size_t(blockIdx.x) * kB + threadIdx.x;
  if (i >= n) return;
  const float t = y[i];
  dz[i] = dy[i] * (1.0f - t * t);
}

// Backward data: dx[b][ci][p] = iscale * oscale *
//   sum_co sum_t W[co][ci][t] dz[b][co][p - off(t)].
template <int CIN, int COUT>
__global__ __launch_bounds__(kB) void conv_bwd_data_kernel(
    const float* __restrict__ dz, const uint16_t* __restrict__ w,
    float* __restrict__ dx, int B, int H, int W, float iscale, float oscale) {
  __shared__ float sw[COUT * CIN * 9];
  for (int i = threadIdx.x; i < COUT * CIN * 9; i += kB) sw[i] = bf16_to_f32(w[i]);
  __syncthreads();
  const size_t hw = size_t(H) * W;
  const size_t p = size_t(blockIdx.x) * kB + threadIdx.x;
  if (p >= size_t(B) * hw) return;
  const int b = int(p / hw);
  const int r = int(p % hw);
  const int py = r / W, px = r % W;
  float acc[CIN];
#pragma unroll
  for (int ci = 0; ci < CIN; ++ci) acc[ci] = 0.f;
  const float* db = dz + size_t(b) * COUT * hw;
  for (int co = 0; co < COUT; ++co) {
    const float* dc = db + size_t(co) * hw;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      // output pixel q = p - off(t) used input pixel p through tap t
      const int yy = wrap(py - (t / 3 - 1), H), xx = wrap(px - (t % 3 - 1), W);
      const float g = dc[size_t(yy) * W + xx];
#pragma unroll
      for (int ci = 0; ci < CIN; ++ci) acc[ci] += sw[(co * CIN + ci) * 9 + t] * g;
    }
  }
  float* xb = dx + size_t(b) * CIN * hw + r;
  const float s = iscale * oscale;
#pragma unroll
  for (int ci = 0; ci < CIN; ++ci) xb[size_t(ci) * hw] = s * acc[ci];
}

__device__ __forceinline__ float block_sum(float v) {
  __shared__ float part[kB / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = 0.f;
  if (threadIdx.x == 0)
    for (int i = 0; i < kB / 64; ++i) r += part[i];
  __syncthreads();
  return r;  // valid in thread 0
}

// Backward weights: block (co, ci) sums over all pixels in fixed order:
// dW[co][ci][t] = oscale * iscale * sum_p dz[b][co][p] x[b][ci][p + off(t)],
// and for ci == 0 also db[co] = oscale * sum_p dz[b][co][p].
template <int CIN, int COUT>
__global__ __launch_bounds__(kB) void conv_bwd_weight_kernel(
    const float* __restrict__ dz, const float* __restrict__ x,
    float* __restrict__ dw, float* __restrict__ dbias, int B, int H, int W,
    float iscale, float oscale) {
  const int co = blockIdx.x / CIN, ci = blockIdx.x % CIN;
  const size_t hw = size_t(H) * W;
  float acc[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) acc[t] = 0.f;
  for (size_t p = threadIdx.x; p < size_t(B) * hw; p += kB) {
    const int b = int(p / hw);
    const int r = int(p % hw);
    const int py = r / W, px = r % W;
    const float g = dz[(size_t(b) * COUT + co) * hw + r];
    const float* xc = x + (size_t(b) * CIN + ci) * hw;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int yy = wrap(py + t / 3 - 1, H), xx = wrap(px + t % 3 - 1, W);
      acc[t] += g * xc[size_t(yy) * W + xx];
    }
    acc[9] += g;
  }
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const float s = block_sum(acc[t]);
    if (threadIdx.x == 0) dw[(co * CIN + ci) * 9 + t] = oscale * iscale * s;
  }
  const float s = block_sum(acc[9]);
  if (threadIdx.x == 0 && ci == 0) dbias[co] = oscale * s;
}

// MSE over the interior (a border of `border` pixels excluded):
// per-block partial sums of (pred - t)^2 / count and the gradient
// dpred = 2 (pred - t) / count on the interior, 0 elsewhere.
// pred and dpred may be the same buffer (each thread reads then writes its
// own element), so they are not restrict-qualified.
__global__ __launch_bounds__(kB) void mse_kernel(const float* pred,
                                                 const float* __restrict__ t,
                                                 float* dpred,
                                                 double* __restrict__ partials,
                                                 int B, int H, int W, int border,
                                                 float inv_count) {
  const size_t hw = size_t(H) * W;
  const size_t p = size_t(blockIdx.x) * kB + threadIdx.x;
  float e2 = 0.f;
  if (p < size_t(B) * hw) {
    const int r = int(p % hw);
    const int py = r / W, px = r % W;
    const bool in = py >= border && py < H - border && px >= border && px < W - border;
    const float d = in ? pred[p] - t[p] : 0.f;
    e2 = d * d * inv_count;
    if (dpred) dpred[p] = 2.f * d * inv_count;
  }
  const float s = block_sum(e2);
  if (threadIdx.x == 0) partials[blockIdx.x] = double(s);
}

__global__ __launch_bounds__(kB) void sum_partials_kernel(const double* __restrict__ in,
                                                          int n, double* __restrict__ out) {
  __shared__ double part[kB];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) s += in[i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int i = 0; i < kB; ++i) r += part[i];
    out[0] = r;
  }
}

// Adam on FP32 masters, refreshing the BF16 compute copy when there is one
// (weights; biases stay FP32).
__global__ __launch_bounds__(kB) void adam_kernel(float* __restrict__ w, uint16_t* __restrict__ wb,
                                                  const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v,
                                                  int n, float lr, float b1, float b2,
                                                  float eps, float c1, float c2) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  if (wb) wb[i] = f32_to_bf16(wi);
}

__global__ __launch_bounds__(kB) void to_bf16_kernel(const float* __restrict__ w,
                                                     uint16_t* __restrict__ wb, int n) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i < n) wb[i] = f32_to_bf16(w[i]);
}

// Periodic crops: out[i] = src[idx[i]] shifted by (oy[i], ox[i]), size h x w,
// minus the same window of the L x L field `sub` when given.
__global__ __launch_bounds__(kB) void gather_crops_kernel(
    const float* __restrict__ src, int L, const int* __restrict__ idx,
    const int* __restrict__ oy, const int* __restrict__ ox,
    const float* __restrict__ sub, float* __restrict__ out, int n, int h, int w) {
  const size_t p = size_t(blockIdx.x) * kB + threadIdx.x;
  const size_t hw = size_t(h) * w;
  if (p >= size_t(n) * hw) return;
  const int i = int(p / hw);
  const int r = int(p % hw);
  const int y = (r / w + oy[i]) % L, x = (r % w + ox[i]) % L;
  const size_t q = size_t(y) * L + x;
  float v = src[size_t(idx[i]) * L * L + q];
  if (sub) v -= sub[q];
  out[p] = v;
}

__device__ __forceinline__ double block_sum_d(double v) {
  __shared__ double part[kB / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kB / 64; ++i) r += part[i];
  __syncthreads();
  return r;  // valid in thread 0
}

// Surrogate cost of B candidate controls x_b (one field each):
//   r_b = u_base + y_b - u_target   (written over y, same index)
//   J_b = 1/2 sum r_b^2 + alpha/2 sum x_b^2
// Block (blockIdx.x, b) writes its FP64 partial to partials[b][blockIdx.x].
__global__ __launch_bounds__(kB) void objective_kernel(float* y, const float* __restrict__ ub,
                                                       const float* __restrict__ ut,
                                                       const float* __restrict__ x,
                                                       double* __restrict__ partials, int hw,
                                                       float alpha) {
  const int b = blockIdx.y;
  const int p = blockIdx.x * kB + threadIdx.x;
  double acc = 0.0;
  if (p < hw) {
    const size_t q = size_t(b) * hw + p;
    const float d = ub[p] + y[q] - ut[p];
    y[q] = d;
    const float xv = x[q];
    acc = 0.5 * double(d) * double(d) + 0.5 * double(alpha) * double(xv) * double(xv);
  }
  const double s = block_sum_d(acc);
  if (threadIdx.x == 0) partials[size_t(b) * gridDim.x + blockIdx.x] = s;
}

// out[b] = sum of row b of partials [B][n], fixed order.
__global__ __launch_bounds__(kB) void rows_sum_kernel(const double* __restrict__ partials,
                                                      int n, double* __restrict__ out) {
  const double* row = partials + size_t(blockIdx.x) * n;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kB) s += row[i];
  s = block_sum_d(s);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// dx += alpha * x
__global__ __launch_bounds__(kB) void axpy_kernel(float* __restrict__ dx,
                                                  const float* __restrict__ x, float alpha,
                                                  size_t n) {
  const size_t i = size_t(blockIdx.x) * kB + threadIdx.x;
  if (i < n) dx[i] += alpha * x[i];
}

// Step candidates X_k = c - lambda_k E (k < n).
__global__ __launch_bounds__(kB) void candidates_kernel(const float* __restrict__ c,
                                                        const float* __restrict__ E,
                                                        SrgSteps lam, int n, size_t hw,
                                                        float* __restrict__ X) {
  const size_t p = size_t(blockIdx.x) * kB + threadIdx.x;
  if (p >= size_t(n) * hw) return;
  const int k = int(p / hw);
  const size_t q = p % hw;
  X[p] = c[q] - lam.v[k] * E[q];
}

int blocks_for(size_t n) { return int((n + kB - 1) / kB); }

}  // namespace

template <int CIN, int COUT>
void launch_conv_fwd(const float* x, const uint16_t* w, const float* b, float* y,
                     int B, int H, int W, float is, float os, bool act, hipStream_t s) {
  const int nb = blocks_for(size_t(B) * H * W);
  if (act)
    hipLaunchKernelGGL((conv_fwd_kernel<CIN, COUT, true>), dim3(nb), dim3(kB), 0, s, x, w, b,
                       y, B, H, W, is, os);
  else
    hipLaunchKernelGGL((conv_fwd_kernel<CIN, COUT, false>), dim3(nb), dim3(kB), 0, s, x, w, b,
                       y, B, H, W, is, os);
}

template <int CIN, int COUT>
void launch_conv_bwd(const float* dz, const float* x, const uint16_t* w, float* dx, float* dw,
                     float* db, int B, int H, int W, float is, float os, hipStream_t s) {
  if (dw)
    hipLaunchKernelGGL((conv_bwd_weight_kernel<CIN, COUT>), dim3(CIN * COUT), dim3(kB), 0, s,
                       dz, x, dw, db, B, H, W, is, os);
  if (dx)
    hipLaunchKernelGGL((conv_bwd_data_kernel<CIN, COUT>), dim3(blocks_for(size_t(B) * H * W)),
                       dim3(kB), 0, s, dz, w, dx, B, H, W, is, os);
}

void launch_tanh_bwd(const float* y, const float* dy, float* dz, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(tanh_bwd_kernel, dim3(blocks_for(n)), dim3(kB), 0, s, y, dy, dz, n);
}

void launch_mse(const float* pred, const float* t, float* dpred, double* partials,
                double* out, int B, int H, int W, int border, hipStream_t s) {
  const int nb = blocks_for(size_t(B) * H * W);
  const double count = double(B) * double(H - 2 * border) * double(W - 2 * border);
  hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(kB), 0, s, pred, t, dpred, partials, B, H, W,
                     border, float(1.0 / count));
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kB), 0, s, partials, nb, out);
}

int mse_partials_needed(int B, int H, int W) { return blocks_for(size_t(B) * H * W); }

void launch_adam(float* w, uint16_t* wb, const float* g, float* m, float* v, int n, float lr,
                 float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(kB), 0, s, w, wb, g, m, v, n, lr,
                     b1, b2, eps, c1, c2);
}

void launch_to_bf16(const float* w, uint16_t* wb, int n, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(n)), dim3(kB), 0, s, w, wb, n);
}

void launch_gather_crops(const float* src, int L, const int* idx, const int* oy, const int* ox,
                         const float* sub, float* out, int n, int h, int w, hipStream_t s) {
  hipLaunchKernelGGL(gather_crops_kernel, dim3(blocks_for(size_t(n) * h * w)), dim3(kB), 0, s,
                     src, L, idx, oy, ox, sub, out, n, h, w);
}

int objective_partials_needed(int B, int H, int W) { return B * blocks_for(size_t(H) * W); }

void launch_objective(float* y, const float* ub, const float* ut, const float* x,
                      double* partials, double* out, int B, int H, int W, float alpha,
                      hipStream_t s) {
  const int hw = H * W;
  const int nb = blocks_for(size_t(hw));
  hipLaunchKernelGGL(objective_kernel, dim3(nb, B), dim3(kB), 0, s, y, ub, ut, x, partials, hw,
                     alpha);
  hipLaunchKernelGGL(rows_sum_kernel, dim3(B), dim3(kB), 0, s, partials, nb, out);
}

void launch_axpy(float* dx, const float* x, float alpha, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel, dim3(blocks_for(n)), dim3(kB), 0, s, dx, x, alpha, n);
}

void launch_candidates(const float* c, const float* E, const SrgSteps& lam, int n, size_t hw,
                       float* X, hipStream_t s) {
  hipLaunchKernelGGL(candidates_kernel, dim3(blocks_for(size_t(n) * hw)), dim3(kB), 0, s, c, E,
                     lam, n, hw, X);
}

#define MRT_SRG_INST(CI, CO)                                                            \
  template void launch_conv_fwd<CI, CO>(const float*, const uint16_t*, const float*,   \
                                        float*, int, int, int, float, float, bool,     \
                                        hipStream_t);                                  \
  template void launch_conv_bwd<CI, CO>(const float*, const float*, const uint16_t*,   \
                                        float*, float*, float*, int, int, int, float,  \
                                        float, hipStream_t);
MRT_SRG_INST(1, 32)
MRT_SRG_INST(32, 32)
MRT_SRG_INST(32, 1)
#undef MRT_SRG_INST

}  // namespace mrt
