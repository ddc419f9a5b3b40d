// Streaming probe of the step kernels' access mixes (probe_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace mrt {
// Whether the mix (reads, writes) is built.
bool stream_probe_has_mix(int reads, int writes);
// `reads` + `writes` planes of n floats, in launch order or XCD-banded;
// false for a mix that is not built (see mrt_stream_probe in include/mrt.h).
bool launch_stream_probe(int reads, int writes, bool banded, const float* in, float* out,
                         size_t n, hipStream_t s);
}  // namespace mrt
