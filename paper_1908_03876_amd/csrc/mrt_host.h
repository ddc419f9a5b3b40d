// Host services of the C-ABI runtime (error text and kernel timing, defined
// in mrt_abi.cpp) shared with the D3Q19 runtime.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mrt {
namespace host {
// Records a printf-style message for mrt_last_error(); returns code.
int failf(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
// Timed span of a step loop for mrt_timing_read (kind 0 forward, 1
// adjoint, 2 recomputation, 3 tangent, 4 continuous adjoint): span_begin
// returns null when timing is off; span_end records `launches` kernels.
void* span_begin(int kind, hipStream_t s);
void span_end(void* span, int64_t launches);
}  // namespace host
}  // namespace mrt
