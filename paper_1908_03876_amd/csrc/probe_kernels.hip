// Streaming probe for measurement: `R` read planes and `W` write planes of
// n floats, one element of each per thread, with the non-temporal loads
// and stores of the step kernels, in one of two work-group orders over the
// 256-element tiles: launch order, or XCD-banded as in the single-lattice
// step kernels (XCD k takes a contiguous range of tiles).  Which order
// streams a mix faster depends on its plane count and size (banded is
// about 10% faster for the 43 planes of 2048^2, launch order faster for
// the 84 planes of 256^3), so the ceiling is the better of the two.  The
// probe has the HBM access mix of a step kernel and none of its
// arithmetic: its bandwidth is what the memory system gives that mix, the
// practical ceiling the step kernels are compared with.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstddef>

#include "mrt_device.h"
#include "probe_internal.h"

namespace mrt {
namespace {

constexpr int kProbeBlock = 256;

template <int R, int W, bool BANDED>
__global__ __launch_bounds__(kProbeBlock) void stream_probe_kernel(const float* __restrict__ in,
                                                                   float* __restrict__ out,
                                                                   size_t n) {
  const int ntiles = int((n + kProbeBlock - 1) / kProbeBlock);
  const int t = BANDED ? dev::xcd_tile(int(blockIdx.x), ntiles) : int(blockIdx.x);
  const size_t i = size_t(t) * kProbeBlock + threadIdx.x;
  if (i >= n) return;
  float v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = __builtin_nontemporal_load(&in[size_t(r) * n + i]);
  float sum = 0.f;
#pragma unroll
  for (int r = 0; r < R; ++r) sum += v[r];
#pragma unroll
  for (int w = 0; w < W; ++w) __builtin_nontemporal_store(sum + float(w), &out[size_t(w) * n + i]);
}

}  // namespace

bool stream_probe_has_mix(int reads, int writes) {
  return (reads == 19 && (writes == 18 || writes == 21)) || (reads == 23 && writes == 20) ||
         (reads == 39 && writes == 42) || (reads == 44 && writes == 40);
}

bool launch_stream_probe(int reads, int writes, bool banded, const float* in, float* out,
                         size_t n, hipStream_t s) {
  if ((n + kProbeBlock - 1) / kProbeBlock > size_t(INT_MAX)) return false;
  const unsigned nb = unsigned((n + kProbeBlock - 1) / kProbeBlock);
#define MRT_PROBE(R, W)                                                              \
  if (reads == R && writes == W) {                                                   \
    if (banded)                                                                      \
      hipLaunchKernelGGL((stream_probe_kernel<R, W, true>), dim3(nb), dim3(kProbeBlock), \
                         0, s, in, out, n);                                          \
    else                                                                             \
      hipLaunchKernelGGL((stream_probe_kernel<R, W, false>), dim3(nb),               \
                         dim3(kProbeBlock), 0, s, in, out, n);                       \
    return true;                                                                     \
  }
  MRT_PROBE(19, 18)  // D2Q9 forward without record (148 B per node)
  MRT_PROBE(19, 21)  // D2Q9 forward with record (160 B)
  MRT_PROBE(23, 20)  // D2Q9 adjoint (172 B)
  MRT_PROBE(39, 42)  // D3Q19 forward with record (324 B)
  MRT_PROBE(44, 40)  // D3Q19 adjoint (336 B)
#undef MRT_PROBE
  return false;
}

}  // namespace mrt
