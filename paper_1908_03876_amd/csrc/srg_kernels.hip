// Kernels of the convolutional surrogate of the control-to-state map
// c -> u(T): four periodic 3x3 convolution layers (1 -> C -> C -> C -> 1
// channels, C = 32), tanh between layers, BF16 weights with FP32
// accumulation, MSE loss and Adam.  The surrogate only proposes warm starts
// and step sizes; the MRT solve still decides whether each proposed step is
// accepted.
//
// Layout: the input x and the output y are float [B][H][W]; the hidden
// activations and the gradients with respect to the hidden pre-activations
// are BF16 channels-last [B][H][W][32] (64 bytes per pixel), rounded to
// nearest even after the tanh (forward) or after the factor 1 - a^2
// (backward).  Master weights are FP32 [Cout][Cin][3][3]; compute copies
// are BF16.  Periodic padding.  A layer computes
// z = oscale * (W * (iscale * x) + b).
//
// The two 32 -> 32 layers are implicit GEMMs on the matrix cores
// (v_mfma_f32_16x16x32_bf16): per tap t the 32 x 32 weight matrix W_t
// multiplies the 32 channels of the 16 pixels of a tile, giving an output
// of channels x pixels.  In the forward the rows of the two channel blocks
// are interleaved so that a lane holds 8 consecutive channels of one pixel
// and the 4 lanes of a pixel write its 64 bytes with one 16-byte store each:
// a store instruction that leaves part of a 64-byte chunk to another one
// costs a read-modify-write in memory.  A block keeps the 18 weight fragments
// (9 taps x 2 channel blocks) in LDS, read per MFMA, and walks many tiles;
// the forward stages its input patches in LDS as well.
// The one-channel first layer runs its 9-tap products on the FP32 matrix
// cores (v_mfma_f32_16x16x4_f32) and its tanh on the vector ALU, and so
// does the input gradient of the last layer (the same 1 -> 32 product with
// the taps mirrored); the last layer's forward and the first layer's input
// gradient (32 -> 1) are BF16 pair dot products on the vector ALU.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "srg_internal.h"

namespace mrt {
namespace {

constexpr int kB = 256;
constexpr int kC = 32;
constexpr int kWaves = kB / 64;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

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

// Two floats rounded to nearest even and packed (low half = a): the
// hardware conversion.
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

// Hyperbolic tangent in five instructions: tanh x = 1 - 2 / (e^{2x} + 1),
// from the hardware base-2 exponential and reciprocal.  The absolute error
// stays within about 3e-7 for every x (an ulp or two of the terms near 1),
// 0 and the limits +-1 come out exact, and non-finite inputs give +-1 or
// NaN.  Near zero the form cancels, so the error is absolute, not relative:
// below the BF16 spacing of every stored activation with |a| > 1e-4, and a
// few units of 1e-7 on the smaller ones.
__device__ __forceinline__ float tanh_fast(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // 2 log2(e)
  return 1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f);
}

// Row m of output channel block mb of an MFMA product (channels x pixels)
// is channel 8 (m / 4) + 4 mb + m % 4, so that the accumulator lanes
// (q, pixel) of blocks 0 and 1 hold channels 8q..8q+3 and 8q+4..8q+7: the 8
// consecutive channels, 16 bytes, of one pixel.
__device__ __forceinline__ int frag_row(int mb, int m) { return 8 * (m >> 2) + 4 * mb + (m & 3); }

__device__ __forceinline__ int wrap(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

__device__ __forceinline__ size_t pix(int bh, int W, int x) { return size_t(bh) * W + x; }

// A staged coordinate i in [-2, n + k) to [0, n): periodic for -n <= i < 2n
// (every coordinate a patch's outputs depend on), clamped beyond (halo
// coordinates past a ragged edge, whose results are not used).
__device__ __forceinline__ int wrap_any(int i, int n) {
  i = i < 0 ? i + n : (i >= n ? i - n : i);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// 8 channels (16 bytes) of a channels-last BF16 field as an MFMA fragment.
__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
}

// unpack 2 BF16 of a 32-bit word
__device__ __forceinline__ float lo16(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi16(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

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

// ------------------------------------------------ first layer (1 -> 32)

// a0 = bf16(tanh(b + W0 * (s_in x))), 32 channels.  A wavefront takes 64
// consecutive pixels of one row as four tiles of 16.  Per tile the 32 x 9
// weight matrix times the 9 x 16 window matrix is six
// v_mfma_f32_16x16x4_f32 (FP32 operands and accumulation), which takes the
// 288 multiply-adds per pixel off the vector ALU; the tanh stays there.
// K-step ks takes the window row y + ks - 1, and its slot q < 3 the column
// x + q - 1 (slot 3 is zero padding), so a k-step reads one wave-uniform
// row and a tile's three k-steps share their column offsets.  Lane
// (q, pixel) ends with channels 8q..8q+7 of its pixel and writes them with
// one 16-byte store.
__global__ __launch_bounds__(kB) void l0_fwd_kernel(const float* __restrict__ x,
                                                    const uint16_t* __restrict__ w,
                                                    const float* __restrict__ bias,
                                                    uint16_t* __restrict__ out, int B, int H,
                                                    int W, float iscale) {
  const int lane = threadIdx.x & 63, n = lane & 15, q = lane >> 4;
  // (row, segment) units fit 32 bits: fields hold at most 2^28 pixels
  const unsigned nseg = unsigned(W + 63) >> 6;
  const unsigned unit = blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (unit >= unsigned(B) * unsigned(H) * nseg) return;  // the whole wavefront
  const int seg = int(unit % nseg);
  const unsigned row = unit / nseg;  // image b, row y: b H + y
  const int y = int(row % unsigned(H));
  const float* xr[3];  // the three window rows, periodic
#pragma unroll
  for (int ks = 0; ks < 3; ++ks)
    xr[ks] = x + size_t(row - y + wrap(y + ks - 1, H)) * W;
  float wa[2][3];  // A operands: W0[frag_row(mb, n)][3 ks + q], zero for q = 3
#pragma unroll
  for (int ks = 0; ks < 3; ++ks)
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      const float wv = bf16_to_f32(w[frag_row(mb, n) * 9 + 3 * ks + (q < 3 ? q : 2)]);
      wa[mb][ks] = q < 3 ? wv : 0.f;
    }
  f32x4 b0, b1;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    b0[i] = bias[8 * q + i];
    b1[i] = bias[8 * q + 4 + i];
  }
  // the window values of all four tiles, loaded together; every address
  // is in the row (lanes past a ragged row end and the padding slot read a
  // valid pixel and use zero)
  float v[4][3];
#pragma unroll
  for (int tile = 0; tile < 4; ++tile) {
    const int px = seg * 64 + tile * 16 + n;
    const bool use = px < W && q < 3;
    const int col = px < W ? wrap(px + (q < 3 ? q : 1) - 1, W) : 0;
#pragma unroll
    for (int ks = 0; ks < 3; ++ks) {
      const float xv = xr[ks][col];
      v[tile][ks] = use ? iscale * xv : 0.f;
    }
  }
  uint16_t* orow = out + size_t(row) * W * kC + 8 * q;
#pragma unroll
  for (int tile = 0; tile < 4; ++tile) {
    const int px = seg * 64 + tile * 16 + n;
    f32x4 a0 = b0, a1 = b1;
#pragma unroll
    for (int ks = 0; ks < 3; ++ks) {
      a0 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[0][ks], v[tile][ks], a0, 0, 0, 0);
      a1 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[1][ks], v[tile][ks], a1, 0, 0, 0);
    }
    if (px < W)
      __builtin_nontemporal_store(u32x4{pack_bf16(tanh_fast(a0[0]), tanh_fast(a0[1])),
                                        pack_bf16(tanh_fast(a0[2]), tanh_fast(a0[3])),
                                        pack_bf16(tanh_fast(a1[0]), tanh_fast(a1[1])),
                                        pack_bf16(tanh_fast(a1[2]), tanh_fast(a1[3]))},
                                  reinterpret_cast<u32x4*>(orow + size_t(px) * kC));
  }
}

// dx[p] = s_in * sum_t sum_co W0[co][t] dz0[p - off(t)][co]: one thread per
// pixel, the 32 channels of each mirrored tap summed as 16 two-channel dot
// products of BF16 pairs (exact products, FP32 sums), the weight pairs read
// as LDS broadcasts.
__global__ __launch_bounds__(kB) void l0_bwd_data_kernel(const uint16_t* __restrict__ dz,
                                                         const uint16_t* __restrict__ w,
                                                         float* __restrict__ dx, int B, int H,
                                                         int W, float iscale) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  // (W0[2j][t], W0[2j+1][t]) as BF16 pairs, [t][j]
  __shared__ __attribute__((aligned(16))) uint32_t wp[9 * 16];
  for (int i = threadIdx.x; i < 9 * 16; i += kB) {
    const int t = i / 16, j = i - 16 * t;
    wp[i] = uint32_t(w[(2 * j) * 9 + t]) | (uint32_t(w[(2 * j + 1) * 9 + t]) << 16);
  }
  __syncthreads();
  const size_t hw = size_t(H) * W;
  const size_t p = size_t(blockIdx.x) * kB + threadIdx.x;
  if (p >= size_t(B) * hw) return;
  const int b = int(p / hw), r = int(p % hw), py = r / W, px = r % W;
  float acc = 0.f;
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int yy = wrap(py - (t / 3 - 1), H), xx = wrap(px - (t % 3 - 1), W);
    const u32x4* g = reinterpret_cast<const u32x4*>(dz + (size_t(b) * hw + size_t(yy) * W + xx) * kC);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const u32x4 q = g[k];
      const u32x4 wq = *reinterpret_cast<const u32x4*>(&wp[t * 16 + 4 * k]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // through scalars: a bit cast of a vector element itself reads element 0
        const uint32_t qe = q[e], we = wq[e];
        acc = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, qe),
                                              __builtin_bit_cast(bf16x2, we), acc, false);
      }
    }
  }
  dx[p] = iscale * acc;
}

// ------------------------------------------------- last layer (32 -> 1)

// Patches of kPR rows x 64 pixels, staged in LDS with their one-pixel halo
// ((kPR + 2) rows x 66 pixels of 64 bytes, periodic wrap) so that every
// input pixel crosses the vector memory unit once per patch instead of
// once per tap.  The 16-byte quarter `part` of staged pixel px sits in slot
// (part + px / 2) % 4 of the pixel, so that eight consecutive pixels read
// at the same quarter fall on distinct banks.
constexpr int kPR = 4;                      // output rows per patch
constexpr int kSW = 66;                     // staged pixels per row
constexpr int kStage = (kPR + 2) * kSW * 4; // 16-byte chunks staged
static_assert(kPR == 4, "the 32 -> 1 layer maps one wavefront to two patch rows, two per block");

__device__ __forceinline__ uint32_t stage_off(int r, int px, int part) {
  return uint32_t((r * kSW + px) * 64 + (((part + (px >> 1)) & 3) << 4));
}

// Stage the patch's chunks this thread owns into registers (the caller
// writes them to LDS once the previous patch is done).
template <int NCH, int NT = kB>
__device__ __forceinline__ void fetch_patch(const uint16_t* __restrict__ in, int patch, int pr,
                                            int pc, int H, int W, u32x4 (&pre)[NCH]) {
  const int b = patch / (pr * pc), rem = patch - b * (pr * pc);
  const int y0 = (rem / pc) * kPR, x0 = (rem - (rem / pc) * pc) * 64;
#pragma unroll
  for (int k = 0; k < NCH; ++k) {
    const int c = int(threadIdx.x) + k * NT;
    if (c < kStage) {
      const int r = c / (kSW * 4), rr = c - r * (kSW * 4), px = rr >> 2, part = rr & 3;
      int yy = y0 - 1 + r;
      yy = yy < 0 ? yy + H : (yy >= H ? yy - H : yy);
      int xx = x0 - 1 + px;
      // x = -1 and x = W wrap; staged pixels further out feed no output
      xx = xx < 0 ? xx + W : (xx >= W ? (xx - W < W ? xx - W : W - 1) : xx);
      pre[k] = *reinterpret_cast<const u32x4*>(in + pix(b * H + yy, W, xx) * kC + 8 * part);
    }
  }
}

template <int NCH, int NT = kB>
__device__ __forceinline__ void store_patch(unsigned char* st, const u32x4 (&pre)[NCH]) {
#pragma unroll
  for (int k = 0; k < NCH; ++k) {
    const int c = int(threadIdx.x) + k * NT;
    if (c < kStage) {
      const int r = c / (kSW * 4), rr = c - r * (kSW * 4), px = rr >> 2, part = rr & 3;
      *reinterpret_cast<u32x4*>(st + stage_off(r, px, part)) = pre[k];
    }
  }
}

constexpr int kChunks = (kStage + kB - 1) / kB;

constexpr int kB3 = 128;  // threads of a 32 -> 1 block: two wavefronts
constexpr int kChunks3 = (kStage + kB3 - 1) / kB3;

// y[p] = s_out * (b + sum_t sum_ci W3[ci][t] a2[p + off(t)][ci]) over a
// staged patch: wavefront w takes patch rows 2w and 2w + 1, a lane the two
// pixels of its column.  The 32 channels of a tap are summed as 16
// two-channel dot products of BF16 pairs (exact products, FP32 sums).  Per
// column offset dx and channel quarter the lane reads the weight quarters
// of the three taps (dy, dx) once and the four staged rows its two pixels
// share once each, 84 LDS reads for two pixels where one pixel at a time
// took 72; LDS bandwidth bounds this layer.
__global__ __launch_bounds__(kB3, 3) void l3_fwd_kernel(const uint16_t* __restrict__ a,
                                                     const uint16_t* __restrict__ w,
                                                     const float* __restrict__ bias,
                                                     float* __restrict__ y, int B, int H, int W,
                                                     float oscale) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  // (W3[2j][t], W3[2j+1][t]) as BF16 pairs, [t][j]
  __shared__ __attribute__((aligned(16))) uint32_t wp[9 * 16];
  __shared__ __attribute__((aligned(16))) unsigned char st[kStage * 16];
  for (int i = threadIdx.x; i < 9 * 16; i += kB3) {
    const int t = i / 16, j = i - 16 * t;
    wp[i] = uint32_t(w[(2 * j) * 9 + t]) | (uint32_t(w[(2 * j + 1) * 9 + t]) << 16);
  }
  const float b0 = bias[0];
  const int pr = (H + kPR - 1) / kPR, pc = (W + 63) >> 6;
  const int npatch = B * pr * pc;
  const int r0 = 2 * __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6), col = threadIdx.x & 63;
  // byte offsets of this lane's three x taps (each quarter) in a staged
  // row, and of the matching weight pairs.  Lane group g = col / 16 takes
  // the quarters in the order g, g + 1, ... (mod 4), so that the four groups
  // read different quarters at once, the access of the 32 -> 32 layers for
  // which the staging rotates the quarters (all 64 lanes on one quarter
  // conflicted in LDS)
  uint32_t colo[3][4], wo[4];
#pragma unroll
  for (int part = 0; part < 4; ++part) {
    const int pq = (part + (col >> 4)) & 3;
    wo[part] = uint32_t(4 * pq);
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) colo[dx][part] = stage_off(0, col + dx, pq);
  }
  const uint32_t rowo = uint32_t(r0 * kSW * 64);
  u32x4 pre[kChunks3];
  if (int(blockIdx.x) < npatch) fetch_patch<kChunks3, kB3>(a, blockIdx.x, pr, pc, H, W, pre);
  for (int patch = blockIdx.x; patch < npatch; patch += gridDim.x) {
    const int b = patch / (pr * pc), rem = patch - b * (pr * pc);
    const int y0 = (rem / pc) * kPR, x0 = (rem - (rem / pc) * pc) * 64;
    __syncthreads();  // the previous patch's reads of st are done (and wp is written)
    store_patch<kChunks3, kB3>(st, pre);
    __syncthreads();
    if (patch + int(gridDim.x) < npatch)
      fetch_patch<kChunks3, kB3>(a, patch + gridDim.x, pr, pc, H, W, pre);
    float acc0 = 0.f, acc1 = 0.f;  // patch rows r0 and r0 + 1
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
#pragma unroll
      for (int part = 0; part < 4; ++part) {
        u32x4 wq[3];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
          wq[dy] = *reinterpret_cast<const u32x4*>(&wp[(3 * dy + dx) * 16 + wo[part]]);
#pragma unroll
        for (int sr = 0; sr < 4; ++sr) {  // staged row r0 + sr
          const u32x4 v = *reinterpret_cast<const u32x4*>(st + rowo + colo[dx][part] +
                                                          uint32_t(sr * kSW * 64));
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            // through scalars: a bit cast of a vector element itself reads element 0
            const uint32_t ve = v[e];
            if (sr < 3) {
              const uint32_t we = wq[sr][e];
              acc0 = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, ve),
                                                     __builtin_bit_cast(bf16x2, we), acc0, false);
            }
            if (sr > 0) {
              const uint32_t we = wq[sr - 1][e];
              acc1 = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, ve),
                                                     __builtin_bit_cast(bf16x2, we), acc1, false);
            }
          }
        }
      }
    }
    // both sums complete here: left to the conditional stores below, the
    // compiler sinks the dot products into them and keeps all 84 LDS reads
    // live across the branch (spilling)
    asm volatile("" : "+v"(acc0), "+v"(acc1));
    const int yo = y0 + r0, xo = x0 + col;
    if (xo < W) {
      if (yo < H) y[pix(b * H + yo, W, xo)] = oscale * (b0 + acc0);
      if (yo + 1 < H) y[pix(b * H + yo + 1, W, xo)] = oscale * (b0 + acc1);
    }
  }
}

// dz2[p][ci] = bf16((s_out sum_t W3[ci][t] dy[p - off(t)]) (1 - a2[p][ci]^2)):
// the 1 -> 32 product of the first layer's forward with the taps mirrored,
// on the same FP32 MFMA tiles (a wavefront per 64 pixels of a row, k-step
// ks on the row y - ks + 1, slot q < 3 on the column x - q + 1), and the
// tanh derivative of the stored activations in the epilogue.
__global__ __launch_bounds__(kB) void l3_bwd_data_kernel(const float* __restrict__ dy,
                                                         const uint16_t* __restrict__ w,
                                                         const uint16_t* __restrict__ a,
                                                         uint16_t* __restrict__ dz, int B, int H,
                                                         int W, float oscale) {
  const int lane = threadIdx.x & 63, n = lane & 15, q = lane >> 4;
  // (row, segment) units fit 32 bits: fields hold at most 2^28 pixels
  const unsigned nseg = unsigned(W + 63) >> 6;
  const unsigned unit = blockIdx.x * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (unit >= unsigned(B) * unsigned(H) * nseg) return;  // the whole wavefront
  const int seg = int(unit % nseg);
  const unsigned row = unit / nseg;  // image b, row y: b H + y
  const int y = int(row % unsigned(H));
  const float* gr[3];  // the three mirrored window rows, periodic
#pragma unroll
  for (int ks = 0; ks < 3; ++ks)
    gr[ks] = dy + size_t(row - y + wrap(y + 1 - ks, H)) * W;
  float wa[2][3];  // A operands: W3[frag_row(mb, n)][3 ks + q], zero for q = 3
#pragma unroll
  for (int ks = 0; ks < 3; ++ks)
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      const float wv = bf16_to_f32(w[frag_row(mb, n) * 9 + 3 * ks + (q < 3 ? q : 2)]);
      wa[mb][ks] = q < 3 ? wv : 0.f;
    }
  float v[4][3];
#pragma unroll
  for (int tile = 0; tile < 4; ++tile) {
    const int px = seg * 64 + tile * 16 + n;
    const bool use = px < W && q < 3;
    const int col = px < W ? wrap(px + 1 - (q < 3 ? q : 1), W) : 0;
#pragma unroll
    for (int ks = 0; ks < 3; ++ks) {
      const float gv = gr[ks][col];
      v[tile][ks] = use ? oscale * gv : 0.f;
    }
  }
  const size_t rowp = size_t(row) * W;
#pragma unroll
  for (int tile = 0; tile < 4; ++tile) {
    const int px = seg * 64 + tile * 16 + n;
    f32x4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 3; ++ks) {
      s0 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[0][ks], v[tile][ks], s0, 0, 0, 0);
      s1 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[1][ks], v[tile][ks], s1, 0, 0, 0);
    }
    if (px < W) {
      // channels 8q..8q+7 of the pixel: s0 holds 8q..8q+3, s1 8q+4..8q+7
      const size_t off = (rowp + size_t(px)) * kC + 8 * q;
      const u32x4 av = *reinterpret_cast<const u32x4*>(a + off);
      u32x4 r;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float a0 = lo16(av[e]), a1 = hi16(av[e]);
        const float z0 = e < 2 ? s0[2 * e] : s1[2 * e - 4];
        const float z1 = e < 2 ? s0[2 * e + 1] : s1[2 * e - 3];
        r[e] = pack_bf16(z0 * (1.f - a0 * a0), z1 * (1.f - a1 * a1));
      }
      *reinterpret_cast<u32x4*>(dz + off) = r;
    }
  }
}

// Weight gradients of a one-channel layer from a 32-channel field F and a
// one-channel field S:  out[c][t] = sum_p F[p][c] S[p + sgn off(t)], all nine
// taps in one pass over F.  Lane = (pixel pp = lane / 8 of the wavefront's 8
// pixels, channel quad cq = lane % 8); each lane keeps 9 x 4 products, the 4
// channel sums and (cq = 0) the sum of S.  A lane's (image, row, column)
// advances by the grid stride with carries, and its nine S offsets come
// from three wrapped rows and three wrapped columns.  Block partials:
// [9][nblk][32] products, [nblk][32] channel sums of F (slot 9), [nblk]
// sums of S.
__global__ __launch_bounds__(kB) void thin_wgrad_kernel(const uint16_t* __restrict__ F,
                                                        const float* __restrict__ S, int sgn,
                                                        double* __restrict__ part, int B, int H,
                                                        int W) {
  const int nblk = gridDim.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int pp = lane >> 3, cq = lane & 7;
  const size_t hw = size_t(H) * W, n = size_t(B) * hw;
  float acc[9][4], fs[4] = {0.f, 0.f, 0.f, 0.f}, ss = 0.f;
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[t][j] = 0.f;
  // four pixels per lane per pass, all their loads issued before the sums;
  // the lane's (image, row, column) advances by the grid stride with
  // carries instead of a division per pixel
  constexpr int kU = 4;
  const size_t stride = size_t(nblk) * kWaves * 8;
  const int sb = int(stride / hw), srem = int(stride % hw), sy = srem / W, sx = srem % W;
  size_t p0 = (size_t(blockIdx.x) * kWaves + wv) * 8 + pp;
  int b = int(p0 / hw), py, px;
  {
    const int r = int(p0 % hw);
    py = r / W;
    px = r % W;
  }
  for (; p0 < n; p0 += kU * stride) {
    u32x2 qv[kU];
    float sv[kU][9];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const size_t p = p0 + u * stride;
      qv[u] = u32x2{0u, 0u};
#pragma unroll
      for (int t = 0; t < 9; ++t) sv[u][t] = 0.f;
      if (p < n) {
        qv[u] = *reinterpret_cast<const u32x2*>(F + p * kC + 4 * cq);
        const float* Sb = S + size_t(b) * hw;
        int ro[3], co[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          ro[d] = wrap(py + sgn * (d - 1), H) * W;
          co[d] = wrap(px + sgn * (d - 1), W);
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) sv[u][t] = Sb[ro[t / 3] + co[t % 3]];
      }
      px += sx;
      if (px >= W) { px -= W; ++py; }
      py += sy;
      if (py >= H) { py -= H; ++b; }
      b += sb;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const float f[4] = {lo16(qv[u][0]), hi16(qv[u][0]), lo16(qv[u][1]), hi16(qv[u][1])};
#pragma unroll
      for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[t][j] += f[j] * sv[u][t];
      if (cq == 0) ss += sv[u][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) fs[j] += f[j];
    }
  }
  // lanes of one channel quad: xor 8, 16, 32; then the waves in LDS
  constexpr int kV = 9 * 4 + 4 + 1;
  __shared__ float red[kWaves][8][kV];
#pragma unroll
  for (int k = 0; k < kV; ++k) {
    float v = k < 36 ? acc[k / 4][k % 4] : (k < 40 ? fs[k - 36] : ss);
    v += __shfl_xor(v, 8, 64);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (pp == 0) red[wv][cq][k] = v;
  }
  __syncthreads();
  // 9 x 32 products, 32 channel sums, 1 sum of S
  for (int i = threadIdx.x; i < 9 * kC + kC + 1; i += kB) {
    double v = 0.0;
    if (i < 9 * kC) {
      const int t = i / kC, c = i % kC;
      for (int k = 0; k < kWaves; ++k) v += double(red[k][c / 4][t * 4 + c % 4]);
      part[(size_t(t) * nblk + blockIdx.x) * kC + c] = v;
    } else if (i < 10 * kC) {
      const int c = i - 9 * kC;
      for (int k = 0; k < kWaves; ++k) v += double(red[k][c / 4][36 + c % 4]);
      part[(size_t(9) * nblk + blockIdx.x) * kC + c] = v;
    } else {
      for (int k = 0; k < kWaves; ++k) v += double(red[k][0][40]);
      part[size_t(10) * nblk * kC + blockIdx.x] = v;
    }
  }
}

// Finish of thin_wgrad, one block per output: dw[c * 9 + t] = scale *
// sum_blk part[t][blk][c] (master layout [Cout][Cin][9] with one of them 1),
// then either 32 per-channel bias gradients (bscale * sum of F) or one
// (bscale * sum of S).  Fixed summation order.
__global__ __launch_bounds__(kB) void thin_wgrad_finish_kernel(const double* __restrict__ part,
                                                               int nblk, float scale,
                                                               float bscale, int bias_per_channel,
                                                               float* __restrict__ dw,
                                                               float* __restrict__ db) {
  const int o = blockIdx.x;
  const double* src;
  size_t stride;
  if (o < 9 * kC) {
    const int c = o / 9, t = o % 9;
    src = part + size_t(t) * nblk * kC + c;
    stride = kC;
  } else if (bias_per_channel) {
    src = part + size_t(9) * nblk * kC + (o - 9 * kC);
    stride = kC;
  } else {
    src = part + size_t(10) * nblk * kC;
    stride = 1;
  }
  double v = 0.0;
  for (int k = threadIdx.x; k < nblk; k += kB) v += src[size_t(k) * stride];
  v = block_sum_d(v);
  if (threadIdx.x == 0) {
    if (o < 9 * kC)
      dw[o] = float(scale * v);
    else
      db[o - 9 * kC] = float(bscale * v);
  }
}

// ------------------------------------------- 32 -> 32 layers on MFMA

// Weight fragments for the matrix cores, from the FP32 masters [32][32][9]:
//   fwd[t][mb][lane][j] = W[co = frag_row(mb, lane % 16)][ci = 8 (lane / 16) + j][t]
//   bwd[t][mb][lane][j] = W[co = 8 (lane / 16) + j][ci = frag_row(mb, lane % 16)][t]
// (A operands of D = W_t X and D = W_t^T G), with the rows interleaved by
// frag_row.

__global__ __launch_bounds__(kB) void pack_weights_kernel(const float* __restrict__ w,
                                                          uint16_t* __restrict__ fwd,
                                                          uint16_t* __restrict__ bwd) {
  const int i = blockIdx.x * kB + threadIdx.x;  // over 9 * 2 * 64 * 8
  if (i >= 9 * 2 * 64 * 8) return;
  const int j = i & 7, lane = (i >> 3) & 63, mb = (i >> 9) & 1, t = i >> 10;
  const int a = frag_row(mb, lane & 15), b = 8 * (lane >> 4) + j;
  fwd[i] = f32_to_bf16(w[(a * kC + b) * 9 + t]);
  bwd[i] = f32_to_bf16(w[(b * kC + a) * 9 + t]);
}

// The 18 MFMAs per tile of a staged patch for the kPR rows of wavefront
// column wv: tap t = 3 dy + dx reads the staged pixel at p + sgn off(t).
template <int SGN>
__device__ __forceinline__ void staged_taps(const unsigned char* st, const bf16x8* wl,
                                            const uint32_t (&colo)[3], int lane,
                                            f32x4 (&acc)[kPR][2]) {
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int dy = SGN > 0 ? t / 3 : 2 - t / 3, dx = SGN > 0 ? t % 3 : 2 - t % 3;
    const bf16x8 w0 = wl[(t * 2) * 64 + lane], w1 = wl[(t * 2 + 1) * 64 + lane];
#pragma unroll
    for (int j = 0; j < kPR; ++j) {
      const bf16x8 v = *reinterpret_cast<const bf16x8*>(
          st + colo[dx] + uint32_t((j + dy) * kSW * 64));
      acc[j][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w0, v, acc[j][0], 0, 0, 0);
      acc[j][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1, v, acc[j][1], 0, 0, 0);
    }
  }
}

// Forward of a hidden layer: out = bf16(tanh(b + sum_t W_t in[p + off(t)])).
// A block walks staged patches (above), loading the next patch into
// registers while the current one computes; wavefront w computes the
// 16-pixel column w of all kPR rows, lane = (channel group q, pixel c16),
// reading each weight fragment once per tap for the kPR rows.  The
// accumulators start at the bias.
__global__ __launch_bounds__(kB, 3) void c32_fwd_kernel(const uint16_t* __restrict__ in,
                                                     const uint16_t* __restrict__ wf,
                                                     const float* __restrict__ bias,
                                                     uint16_t* __restrict__ out, int B, int H,
                                                     int W) {
  __shared__ bf16x8 wl[18 * 64];
  __shared__ __attribute__((aligned(16))) unsigned char st[kStage * 16];
  const int lane = threadIdx.x & 63, q = lane >> 4, c16 = lane & 15;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  for (int k = threadIdx.x; k < 18 * 64; k += kB) wl[k] = load8(wf + size_t(k) * 8);
  f32x4 bv[2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[mb][j] = bias[8 * q + 4 * mb + j];
  const int pr = (H + kPR - 1) / kPR, pc = (W + 63) >> 6;
  const int npatch = B * pr * pc;
  // column offsets (bytes) of this lane's three x taps in a staged row
  uint32_t colo[3];
#pragma unroll
  for (int dx = 0; dx < 3; ++dx) colo[dx] = stage_off(0, 16 * wv + c16 + dx, q);
  // the next patch's chunks are loaded into registers while the current
  // one computes
  // A block takes a contiguous run of patches in column-major order (down
  // a 64-pixel column, row block after row block), so that the two halo
  // rows it stages for the next patch are rows it fetched for this one
  // and are still in L2.
  const int rows = B * pr;  // row blocks over all fields
  const int per = (npatch + int(gridDim.x) - 1) / int(gridDim.x);
  const int s0 = int(blockIdx.x) * per, s1 = min(s0 + per, npatch);
  auto patch_of = [&](int sq) {
    const int cb = sq / rows;
    return (sq - cb * rows) * pc + cb;
  };
  u32x4 pre[kChunks];
  if (s0 < s1) fetch_patch(in, patch_of(s0), pr, pc, H, W, pre);
  for (int sq = s0; sq < s1; ++sq) {
    const int patch = patch_of(sq);
    const int b = patch / (pr * pc), rem = patch - b * (pr * pc);
    const int y0 = (rem / pc) * kPR, x0 = (rem - (rem / pc) * pc) * 64;
    __syncthreads();  // the previous patch's reads of st are done (and wl is written)
    store_patch(st, pre);
    __syncthreads();
    if (sq + 1 < s1) fetch_patch(in, patch_of(sq + 1), pr, pc, H, W, pre);
    f32x4 acc[kPR][2];
#pragma unroll
    for (int j = 0; j < kPR; ++j) {
      acc[j][0] = bv[0];
      acc[j][1] = bv[1];
    }
    staged_taps<1>(st, wl, colo, lane, acc);
    const int px = x0 + 16 * wv + c16;
#pragma unroll
    for (int j = 0; j < kPR; ++j) {
      const int y = y0 + j;
      if (y < H && px < W) {
        // channels 8q..8q+7 of the pixel
        uint16_t* o = out + pix(b * H + y, W, px) * kC + 8 * q;
        u32x4 r;
        r[0] = pack_bf16(tanh_fast(acc[j][0][0]), tanh_fast(acc[j][0][1]));
        r[1] = pack_bf16(tanh_fast(acc[j][0][2]), tanh_fast(acc[j][0][3]));
        r[2] = pack_bf16(tanh_fast(acc[j][1][0]), tanh_fast(acc[j][1][1]));
        r[3] = pack_bf16(tanh_fast(acc[j][1][2]), tanh_fast(acc[j][1][3]));
        __builtin_nontemporal_store(r, reinterpret_cast<u32x4*>(o));
      }
    }
  }
}

// Backward data of a hidden layer with the previous tanh folded in:
// dz_prev[p][ci] = bf16((sum_t W_t^T dz[p - off(t)])[ci] (1 - a_prev[p][ci]^2)),
// on the staged, prefetched patches of the forward with the transposed
// weight fragments in LDS.
__global__ __launch_bounds__(kB, 3) void c32_bwd_data_kernel(const uint16_t* __restrict__ dz,
                                                             const uint16_t* __restrict__ wt,
                                                             const uint16_t* __restrict__ aprev,
                                                             uint16_t* __restrict__ dzprev,
                                                             int B, int H, int W) {
  __shared__ bf16x8 wl[18 * 64];
  __shared__ __attribute__((aligned(16))) unsigned char st[kStage * 16];
  const int lane = threadIdx.x & 63, q = lane >> 4, c16 = lane & 15;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  for (int k = threadIdx.x; k < 18 * 64; k += kB) wl[k] = load8(wt + size_t(k) * 8);
  const int pr = (H + kPR - 1) / kPR, pc = (W + 63) >> 6;
  const int npatch = B * pr * pc;
  uint32_t colo[3];
#pragma unroll
  for (int dx = 0; dx < 3; ++dx) colo[dx] = stage_off(0, 16 * wv + c16 + dx, q);
  u32x4 pre[kChunks];
  if (int(blockIdx.x) < npatch) fetch_patch(dz, blockIdx.x, pr, pc, H, W, pre);
  for (int patch = blockIdx.x; patch < npatch; patch += gridDim.x) {
    const int b = patch / (pr * pc), rem = patch - b * (pr * pc);
    const int y0 = (rem / pc) * kPR, x0 = (rem - (rem / pc) * pc) * 64;
    __syncthreads();  // the previous patch's reads of st are done (and wl is written)
    store_patch(st, pre);
    __syncthreads();
    if (patch + int(gridDim.x) < npatch) fetch_patch(dz, patch + gridDim.x, pr, pc, H, W, pre);
    f32x4 acc[kPR][2];
#pragma unroll
    for (int j = 0; j < kPR; ++j) {
      acc[j][0] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc[j][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    staged_taps<-1>(st, wl, colo, lane, acc);
    const int px = x0 + 16 * wv + c16;
#pragma unroll
    for (int j = 0; j < kPR; ++j) {
      const int y = y0 + j;
      if (y < H && px < W) {
        // channels 8q..8q+7 of the pixel (blocks 0 and 1 of the accumulator)
        const size_t o = pix(b * H + y, W, px) * kC + 8 * q;
        const u32x4 pa = *reinterpret_cast<const u32x4*>(aprev + o);
        const float av[2][4] = {{lo16(pa[0]), hi16(pa[0]), lo16(pa[1]), hi16(pa[1])},
                                {lo16(pa[2]), hi16(pa[2]), lo16(pa[3]), hi16(pa[3])}};
        u32x4 r;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const float g0 = acc[j][mb][2 * h] * (1.f - av[mb][2 * h] * av[mb][2 * h]);
            const float g1 = acc[j][mb][2 * h + 1] * (1.f - av[mb][2 * h + 1] * av[mb][2 * h + 1]);
            r[2 * mb + h] = pack_bf16(g0, g1);
          }
        __builtin_nontemporal_store(r, reinterpret_cast<u32x4*>(dzprev + o));
      }
    }
  }
}

// Weight gradients of a hidden layer on the matrix cores:
//   dW[co][ci][t] = sum_p dz[p][co] a[p + off(t)][ci],  db[co] = sum_p dz[p][co]
// The MFMA's K dimension is pixels, so an operand is 8 consecutive pixels
// of one channel: a block walks the staged patches of the forward (kPR rows
// x 64 pixels) and stages dz and a (with its one-pixel halo) in LDS
// transposed, channel-major with the pixels contiguous.  A thread stages 8
// pixels x 8 channels: eight 16-byte loads, a transpose in registers and
// eight 16-byte LDS writes.  The channel strides (kCSa, kCSd) are 4 dwords
// modulo 32 (and 36 or 4 modulo 64), so the 16-byte fragment reads of 8
// or 16 lanes on consecutive channels fall on distinct banks.  For each row
// of taps a lane reads 8 + 2 staged pixels once: the taps dx = 0, 1, 2 are
// that window at offsets 0, 1 (realigned with alignbit) and 2.  Wavefront
// w takes the 32-pixel chunk column w % 2 of rows 2 (w / 2) and
// 2 (w / 2) + 1 and accumulates all 9 x 2 x 2 output fragments over its
// chunks.  The block's wavefronts are summed in a fixed order, and the block
// writes one partial [kSrgWPart] in fragment order: the weights as
// [t][mb][nb][lane][4] (co = 16 mb + 4 (lane / 16) + j, ci = 16 nb +
// lane % 16), then the 32 bias sums.
constexpr int kTW = 72;                          // staged pixels per row of a
constexpr int kCSa = (kPR + 2) * kTW + 24;       // channel stride of a (228 dwords)
constexpr int kCSd = kPR * 64 + 8;               // channel stride of dz (132 dwords)
constexpr int kWShared = kC * kCSa + kC * kCSd;  // uint16 elements of the stage
constexpr int kAItems = (kPR + 2) * (kTW / 8) * 4;  // (row, 8-pixel group, channel octet)
constexpr int kDItems = kPR * 8 * 4;
static_assert((kCSa / 2) % 32 == 4 && (kCSd / 2) % 32 == 4, "conflict-free channel strides");
// after the last patch the stage holds the four wavefronts' sums
constexpr int kWLds = kWShared > 2 * kWaves * kSrgWPart ? kWShared : 2 * kWaves * kSrgWPart;

// Transpose 8 pixels x 8 BF16 channels: v[j] holds channels 0..7 of pixel
// j; o[c] receives pixels 0..7 of channel c.
__device__ __forceinline__ void transpose8(const u32x4 (&v)[8], u32x4 (&o)[8]) {
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // low halves (even channel) or high halves (odd channel) of pixels 2k, 2k + 1
      const uint32_t lo = v[2 * k][c >> 1], hi = v[2 * k + 1][c >> 1];
      o[c][k] = (c & 1) ? __builtin_amdgcn_perm(hi, lo, 0x07060302u)
                        : __builtin_amdgcn_perm(hi, lo, 0x05040100u);
    }
}

// Staging item `it` of a patch: its 8 x 16-byte loads (issued, not waited
// for), and where its 8 channel rows go in the stage.
constexpr int kWItems = (kAItems + kDItems + kB - 1) / kB;  // items per thread
static_assert(kWItems == 2, "two staging items per thread");

__device__ __forceinline__ void wgrad_fetch(const uint16_t* __restrict__ dz,
                                            const uint16_t* __restrict__ a, int it, int b,
                                            int y0, int x0, int H, int W, u32x4 (&v)[8]) {
  if (it < kAItems) {
    // a: group g (pixels 8g .. 8g + 7 of the staged row) fastest
    const int g = it % (kTW / 8), rest = it / (kTW / 8), prt = rest & 3, r = rest >> 2;
    const size_t row = size_t(b * H + wrap_any(y0 - 1 + r, H)) * W;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      v[j] = *reinterpret_cast<const u32x4*>(a + (row + wrap_any(x0 - 1 + 8 * g + j, W)) * kC +
                                             8 * prt);
  } else if (it < kAItems + kDItems) {
    const int k = it - kAItems, g = k & 7, prt = (k >> 3) & 3, r = k >> 5;
    const int yy = y0 + r;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int xx = x0 + 8 * g + j;
      v[j] = (yy < H && xx < W)
                 ? *reinterpret_cast<const u32x4*>(dz + pix(b * H + yy, W, xx) * kC + 8 * prt)
                 : u32x4{0u, 0u, 0u, 0u};
    }
  }
}

__device__ __forceinline__ void wgrad_stage(uint16_t* aT, uint16_t* dT, int it,
                                            const u32x4 (&v)[8]) {
  uint16_t* dst;
  int cs;
  if (it < kAItems) {
    const int g = it % (kTW / 8), rest = it / (kTW / 8), prt = rest & 3, r = rest >> 2;
    dst = aT + 8 * prt * kCSa + r * kTW + 8 * g;
    cs = kCSa;
  } else if (it < kAItems + kDItems) {
    const int k = it - kAItems, g = k & 7, prt = (k >> 3) & 3, r = k >> 5;
    dst = dT + 8 * prt * kCSd + r * 64 + 8 * g;
    cs = kCSd;
  } else {
    return;
  }
  u32x4 o[8];
  transpose8(v, o);
#pragma unroll
  for (int c = 0; c < 8; ++c) *reinterpret_cast<u32x4*>(dst + c * cs) = o[c];
}

// One block per CU: the next patch's loads are in flight while the MFMAs of
// the current one run.
__global__ __launch_bounds__(kB, 1) void c32_bwd_weight_kernel(const uint16_t* __restrict__ dz,
                                                               const uint16_t* __restrict__ a,
                                                               float* __restrict__ part, int B,
                                                               int H, int W) {
  __shared__ __attribute__((aligned(16))) uint16_t sm[kWLds];
  uint16_t* aT = sm;             // [ci][r][p]: a at row y0 - 1 + r, column x0 - 1 + p
  uint16_t* dT = sm + kC * kCSa; // [co][r][p]: dz at row y0 + r, column x0 + p
  const int lane = threadIdx.x & 63, q = lane >> 4, c16 = lane & 15;
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int cw = wv & 1, rh = wv >> 1;
  f32x4 acc[9][2][2];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int n = 0; n < 2; ++n) acc[t][m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  float dbs[2] = {0.f, 0.f};
  const int pr = (H + kPR - 1) / kPR, pc = (W + 63) >> 6;
  const int npatch = B * pr * pc;
  const int it0 = threadIdx.x, it1 = threadIdx.x + kB;
  u32x4 v0[8], v1[8];
  auto fetch = [&](int patch) {
    const int b = patch / (pr * pc), rem = patch - b * (pr * pc);
    const int y0 = (rem / pc) * kPR, x0 = (rem - (rem / pc) * pc) * 64;
    wgrad_fetch(dz, a, it0, b, y0, x0, H, W, v0);
    wgrad_fetch(dz, a, it1, b, y0, x0, H, W, v1);
  };
  if (int(blockIdx.x) < npatch) fetch(blockIdx.x);
  for (int patch = blockIdx.x; patch < npatch; patch += gridDim.x) {
    __syncthreads();  // the previous patch's reads are done
    wgrad_stage(aT, dT, it0, v0);
    wgrad_stage(aT, dT, it1, v1);
    __syncthreads();
    if (patch + int(gridDim.x) < npatch) fetch(patch + gridDim.x);
#pragma unroll
    for (int jr = 0; jr < 2; ++jr) {
      const int row = 2 * rh + jr;
      const int p0 = 32 * cw + 8 * q;  // first pixel of this lane's K slice
      // A[m = co][k = pixel]: dz of the lane's 8 pixels for co = 16 mb + c16
      bf16x8 af[2];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        af[mb] = *reinterpret_cast<const bf16x8*>(dT + (16 * mb + c16) * kCSd + row * 64 + p0);
#pragma unroll
        for (int j = 0; j < 8; ++j) dbs[mb] += float(af[mb][j]);
      }
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        // B[k = pixel][n = ci]: a of the lane's 8 pixels shifted by the tap,
        // ci = 16 nb + c16; staged pixels p0 .. p0 + 9 serve dx = 0, 1, 2
        bf16x8 bf[3][2];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          const uint16_t* src = aT + (16 * nb + c16) * kCSa + (row + dy) * kTW + p0;
          const u32x4 d = *reinterpret_cast<const u32x4*>(src);
          const uint32_t d4 = *reinterpret_cast<const uint32_t*>(src + 8);
          const uint32_t d0 = d[0], d1 = d[1], d2 = d[2], d3 = d[3];
          bf[0][nb] = __builtin_bit_cast(bf16x8, d);
          bf[1][nb] = __builtin_bit_cast(
              bf16x8, u32x4{__builtin_amdgcn_alignbit(d1, d0, 16), __builtin_amdgcn_alignbit(d2, d1, 16),
                            __builtin_amdgcn_alignbit(d3, d2, 16), __builtin_amdgcn_alignbit(d4, d3, 16)});
          bf[2][nb] = __builtin_bit_cast(bf16x8, u32x4{d1, d2, d3, d4});
        }
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
          for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
              acc[3 * dy + dx][mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  af[mb], bf[dx][nb], acc[3 * dy + dx][mb][nb], 0, 0, 0);
      }
    }
  }
  __syncthreads();  // the stage becomes four regions, one per wavefront
  float* reg = reinterpret_cast<float*>(sm);
  float db2[2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    float v = dbs[mb];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    db2[mb] = v;
  }
  float* mine = reg + wv * kSrgWPart;
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
        *reinterpret_cast<f32x4*>(mine + (((t * 2 + mb) * 2 + nb) * 64 + lane) * 4) =
            acc[t][mb][nb];
  if (q == 0) {
    mine[kC * kC * 9 + c16] = db2[0];
    mine[kC * kC * 9 + 16 + c16] = db2[1];
  }
  __syncthreads();
  // the block's partial in fragment order (wavefronts summed in a fixed order)
  float* P = part + size_t(blockIdx.x) * kSrgWPart;
  for (int i = threadIdx.x; i < kSrgWPart; i += kB)
    P[i] = ((reg[i] + reg[kSrgWPart + i]) + reg[2 * kSrgWPart + i]) + reg[3 * kSrgWPart + i];
}

// dw, db = sums over the np block partials of c32_bwd_weight_kernel: 32
// partial entries per block, eight slices of the partials per entry (each
// in a fixed order), combined in a fixed order.
__global__ __launch_bounds__(kB) void wpart_sum_kernel(const float* __restrict__ part, int np,
                                                       float* __restrict__ dw,
                                                       float* __restrict__ db) {
  constexpr int kO = 32, kSl = kB / kO;
  const int o = threadIdx.x % kO, sl = threadIdx.x / kO;
  const int i = blockIdx.x * kO + o;
  __shared__ double red[kSl][kO];
  double s0 = 0.0, s1 = 0.0;
  if (i < kSrgWPart) {
    int k = sl;
    for (; k + kSl < np; k += 2 * kSl) {
      s0 += part[size_t(k) * kSrgWPart + i];
      s1 += part[size_t(k + kSl) * kSrgWPart + i];
    }
    if (k < np) s0 += part[size_t(k) * kSrgWPart + i];
  }
  red[sl][o] = s0 + s1;
  __syncthreads();
  if (sl == 0 && i < kSrgWPart) {
    double s = 0.0;
    for (int k = 0; k < kSl; ++k) s += red[k][o];
    if (i < kC * kC * 9) {
      // fragment order [t][mb][nb][lane][j] to the master layout [co][ci][t]
      const int j = i & 3, lane = (i >> 2) & 63, slot = i >> 8;
      const int t = slot >> 2, mb = (slot >> 1) & 1, nb = slot & 1;
      const int co = 16 * mb + 4 * (lane >> 4) + j, ci = 16 * nb + (lane & 15);
      dw[(co * kC + ci) * 9 + t] = float(s);
    } else {
      db[i - kC * kC * 9] = float(s);
    }
  }
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

// One Adam step for every parameter of the network in one launch: thread i
// finds its group in the table and updates the FP32 master, its moments and
// its compute copy -- the BF16 weight of a one-channel layer, or, for a
// 32 x 32 layer, its two MFMA fragment slots (forward: co = frag_row(mb,
// lane % 16), ci = 8 (lane / 16) + j; transposed: ci = frag_row(mb, lane %
// 16), co = 8 (lane / 16) + j; each master weight occupies one slot of each).
__global__ __launch_bounds__(kB) void adam_all_kernel(SrgAdamTable tab, float lr, float b1,
                                                      float b2, float eps, float c1, float c2) {
  int i = blockIdx.x * kB + threadIdx.x;
  int g = 0;
  while (g < tab.n && i >= tab.g[g].n) {
    i -= tab.g[g].n;
    ++g;
  }
  if (g >= tab.n) return;
  const SrgAdamGroup& G = tab.g[g];
  const float gi = G.grad[i];
  const float mi = b1 * G.m[i] + (1.f - b1) * gi;
  const float vi = b2 * G.v[i] + (1.f - b2) * gi * gi;
  G.m[i] = mi;
  G.v[i] = vi;
  const float wi = G.w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  G.w[i] = wi;
  const uint16_t hb = f32_to_bf16(wi);
  if (G.wb) G.wb[i] = hb;
  if (G.wf) {  // master layout [co][ci][9], 32 x 32
    const int t = i % 9, ci = (i / 9) % kC, co = i / (9 * kC);
    // inverse of frag_row: c = 8 (m / 4) + 4 mb + m % 4
    const int mf = (co >> 2) & 1, rf = 4 * (co >> 3) + (co & 3);
    const int mt = (ci >> 2) & 1, rt = 4 * (ci >> 3) + (ci & 3);
    G.wf[((t * 2 + mf) * 64 + rf + 16 * (ci / 8)) * 8 + ci % 8] = hb;
    G.wt[((t * 2 + mt) * 64 + rt + 16 * (co / 8)) * 8 + co % 8] = hb;
  }
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

// Barzilai-Borwein steepest descent on the surrogate cost (warm start).
// With s = c_k - c_{k-1} and y = g_k - g_{k-1}: block partials of <s, s>,
// <s, y> and <g_k, g_k>, [blk][3].
__global__ __launch_bounds__(kB) void bb_dots_kernel(const float* __restrict__ c,
                                                     const float* __restrict__ cp,
                                                     const float* __restrict__ g,
                                                     const float* __restrict__ gp, size_t n,
                                                     double* __restrict__ part) {
  double a[3] = {0.0, 0.0, 0.0};
  for (size_t i = size_t(blockIdx.x) * kB + threadIdx.x; i < n; i += size_t(gridDim.x) * kB) {
    const double gi = double(g[i]);
    const double sv = double(c[i]) - double(cp[i]), yv = gi - double(gp[i]);
    a[0] += sv * sv;
    a[1] += sv * yv;
    a[2] += gi * gi;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double t = block_sum_d(a[k]);
    if (threadIdx.x == 0) part[size_t(blockIdx.x) * 3 + k] = t;
  }
}

// One block: sums the partials in a fixed order and sets the step of this
// iteration, st[0] = <s, s>/<s, y> when that is positive and finite (else the
// previous step), or eta0 / RMS(g) at the first iteration.  It also keeps
// the best surrogate cost seen, st[2], and flags st[1] = 1 when the current
// iterate (cost J[0]) improves on it, so that the update copies it.
__global__ __launch_bounds__(kB) void bb_step_kernel(const double* __restrict__ part, int nblk,
                                                     double n, float eta0, int first,
                                                     const double* __restrict__ J,
                                                     double* __restrict__ st) {
  double a[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += kB)
#pragma unroll
    for (int k = 0; k < 3; ++k) a[k] += part[size_t(b) * 3 + k];
  double r[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) r[k] = block_sum_d(a[k]);
  if (threadIdx.x == 0) {
    if (first) {
      st[0] = r[2] > 0.0 ? double(eta0) / sqrt(r[2] / n) : 0.0;
      st[2] = INFINITY;
    } else if (r[1] > 0.0 && isfinite(r[0] / r[1])) {
      st[0] = r[0] / r[1];
    }
    const bool better = J[0] < st[2];
    st[1] = better ? 1.0 : 0.0;
    if (better) st[2] = J[0];
  }
}

// best <- c (when flagged), cp <- c, gp <- g, c <- c - eta g.
__global__ __launch_bounds__(kB) void bb_update_kernel(float* __restrict__ c,
                                                       float* __restrict__ cp,
                                                       const float* __restrict__ g,
                                                       float* __restrict__ gp,
                                                       float* __restrict__ best,
                                                       const double* __restrict__ st, size_t n) {
  const size_t i = size_t(blockIdx.x) * kB + threadIdx.x;
  if (i >= n) return;
  const float ci = c[i], gi = g[i];
  if (st[1] != 0.0) best[i] = ci;
  cp[i] = ci;
  gp[i] = gi;
  c[i] = float(double(ci) - st[0] * double(gi));
}

// c <- best when the best cost seen (st[2]) is below that of c (J[0]).
__global__ __launch_bounds__(kB) void bb_final_kernel(float* __restrict__ c,
                                                      const float* __restrict__ best,
                                                      const double* __restrict__ st,
                                                      const double* __restrict__ J, size_t n) {
  const size_t i = size_t(blockIdx.x) * kB + threadIdx.x;
  if (i < n && st[2] < J[0]) c[i] = best[i];
}

int blocks_for(size_t n) { return int((n + kB - 1) / kB); }


int blocks_for_pixels(int B, int H, int W) { return blocks_for(size_t(B) * H * W); }


}  // namespace

void launch_srg_l0_fwd(const float* x, const uint16_t* w, const float* b, uint16_t* out, int B,
                       int H, int W, float iscale, hipStream_t s) {
  // one wavefront per 64-pixel segment of a row
  const size_t units = size_t(B) * H * ((W + 63) / 64);
  const int nb = int((units + kWaves - 1) / kWaves);
  hipLaunchKernelGGL(l0_fwd_kernel, dim3(nb > 0 ? nb : 1), dim3(kB), 0, s, x, w, b, out, B, H,
                     W, iscale);
}

void launch_srg_l0_bwd_data(const uint16_t* dz, const uint16_t* w, float* dx, int B, int H,
                            int W, float iscale, hipStream_t s) {
  hipLaunchKernelGGL(l0_bwd_data_kernel, dim3(blocks_for_pixels(B, H, W)), dim3(kB), 0, s, dz,
                     w, dx, B, H, W, iscale);
}

void launch_srg_l3_fwd(const uint16_t* a, const uint16_t* w, const float* b, float* y, int B,
                       int H, int W, float oscale, hipStream_t s) {
  // patches of kPR rows x 64 pixels; six two-wavefront blocks per CU (six
  // 26 KB stages fit in 160 KB; the kernel is built for three wavefronts
  // per SIMD)
  const int np = B * ((H + kPR - 1) / kPR) * ((W + 63) / 64);
  const int nb = np < 1536 ? (np > 0 ? np : 1) : 1536;
  hipLaunchKernelGGL(l3_fwd_kernel, dim3(nb), dim3(kB3), 0, s, a, w, b,
                     y, B, H, W, oscale);
}

void launch_srg_l3_bwd_data(const float* dy, const uint16_t* w, const uint16_t* a, uint16_t* dz,
                            int B, int H, int W, float oscale, hipStream_t s) {
  // one wavefront per 64-pixel segment of a row
  const size_t units = size_t(B) * H * ((W + 63) / 64);
  const int nb = int((units + kWaves - 1) / kWaves);
  hipLaunchKernelGGL(l3_bwd_data_kernel, dim3(nb > 0 ? nb : 1), dim3(kB), 0, s, dy, w, a, dz, B,
                     H, W, oscale);
}

void launch_srg_thin_wgrad(const uint16_t* F, const float* S, int sgn, double* part, int B,
                           int H, int W, float scale, float bscale, int bias_per_channel,
                           float* dw, float* db, hipStream_t s) {
  const size_t n = size_t(B) * H * W;
  size_t want = (n + kWaves * 8 - 1) / (kWaves * 8);
  const int nblk = int(want < size_t(kSrgThinBlocks) ? want : size_t(kSrgThinBlocks));
  hipLaunchKernelGGL(thin_wgrad_kernel, dim3(nblk), dim3(kB), 0, s, F, S, sgn, part, B, H, W);
  const int nout = 9 * kC + (bias_per_channel ? kC : 1);
  hipLaunchKernelGGL(thin_wgrad_finish_kernel, dim3(nout), dim3(kB), 0, s, part, nblk, scale,
                     bscale, bias_per_channel, dw, db);
}

void launch_srg_pack(const float* w, uint16_t* fwd, uint16_t* bwd, hipStream_t s) {
  hipLaunchKernelGGL(pack_weights_kernel, dim3((9 * 2 * 64 * 8 + kB - 1) / kB), dim3(kB), 0, s,
                     w, fwd, bwd);
}

void launch_srg_c32_fwd(const uint16_t* in, const uint16_t* wf, const float* b, uint16_t* out,
                        int B, int H, int W, hipStream_t s) {
  // patches of kPR rows x 64 pixels; as many blocks as the LDS of the 256
  // CUs holds (160 KB each)
  const int np = B * ((H + kPR - 1) / kPR) * ((W + 63) / 64);
  const int lds = 18 * 64 * 16 + kStage * 16;
  const int most = 256 * (160 * 1024 / lds);
  const int nb = np < most ? (np > 0 ? np : 1) : most;
  hipLaunchKernelGGL(c32_fwd_kernel, dim3(nb), dim3(kB), 0, s, in, wf, b, out, B, H, W);
}

void launch_srg_c32_bwd_data(const uint16_t* dz, const uint16_t* wt, const uint16_t* aprev,
                             uint16_t* dzprev, int B, int H, int W, hipStream_t s) {
  // staged patches as in the forward, three blocks per CU
  const int np = B * ((H + kPR - 1) / kPR) * ((W + 63) / 64);
  const int nb = np < 768 ? (np > 0 ? np : 1) : 768;
  hipLaunchKernelGGL(c32_bwd_data_kernel, dim3(nb), dim3(kB), 0, s, dz, wt, aprev, dzprev, B, H,
                     W);
}

void launch_srg_c32_bwd_weight(const uint16_t* dz, const uint16_t* a, float* part, float* dw,
                               float* db, int B, int H, int W, hipStream_t s) {
  const int np = B * ((H + kPR - 1) / kPR) * ((W + 63) / 64);
  const int nb = np < kSrgWBlocks ? (np > 0 ? np : 1) : kSrgWBlocks;
  hipLaunchKernelGGL(c32_bwd_weight_kernel, dim3(nb), dim3(kB), 0, s, dz, a, part, B, H, W);
  hipLaunchKernelGGL(wpart_sum_kernel, dim3((kSrgWPart + 31) / 32), dim3(kB), 0, s, part, nb,
                     dw, db);
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

void launch_adam_all(const SrgAdamTable& tab, float lr, float b1, float b2, float eps, float c1,
                     float c2, hipStream_t s) {
  int n = 0;
  for (int g = 0; g < tab.n; ++g) n += tab.g[g].n;
  hipLaunchKernelGGL(adam_all_kernel, dim3(blocks_for(size_t(n))), dim3(kB), 0, s, tab, lr, b1,
                     b2, eps, c1, c2);
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

void launch_bb_step(const float* c, const float* cp, const float* g, const float* gp, size_t n,
                    double* part, float eta0, int first, const double* J, double* st,
                    hipStream_t s) {
  const int nb = std::min(kSrgBBBlocks, blocks_for(n));
  hipLaunchKernelGGL(bb_dots_kernel, dim3(nb), dim3(kB), 0, s, c, cp, g, gp, n, part);
  hipLaunchKernelGGL(bb_step_kernel, dim3(1), dim3(kB), 0, s, part, nb, double(n), eta0, first,
                     J, st);
}

void launch_bb_update(float* c, float* cp, const float* g, float* gp, float* best,
                      const double* st, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(bb_update_kernel, dim3(blocks_for(n)), dim3(kB), 0, s, c, cp, g, gp, best,
                     st, n);
}

void launch_bb_final(float* c, const float* best, const double* st, const double* J, size_t n,
                     hipStream_t s) {
  hipLaunchKernelGGL(bb_final_kernel, dim3(blocks_for(n)), dim3(kB), 0, s, c, best, st, J, n);
}

void launch_candidates(const float* c, const float* E, const SrgSteps& lam, int n, size_t hw,
                       float* X, hipStream_t s) {
  hipLaunchKernelGGL(candidates_kernel, dim3(blocks_for(size_t(n) * hw)), dim3(kB), 0, s, c, E,
                     lam, n, hw, X);
}


}  // namespace mrt
