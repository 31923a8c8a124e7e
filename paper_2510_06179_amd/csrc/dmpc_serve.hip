// Device side of the serving runtime: scatter of request inputs into the
// session stores and gather of results into the staging buffer.
#include <hip/hip_runtime.h>

#include "dmpc_internal.h"

namespace dmpc {

// One workgroup per segment (grid-stride over segments), 32-bit words,
// consecutive threads on consecutive words.
__global__ __launch_bounds__(256) void seg_copy_kernel(const Seg* segs, int n) {
  for (int s = blockIdx.x; s < n; s += gridDim.x) {
    const uint32_t* src = segs[s].src;
    uint32_t* dst = segs[s].dst;
    const int64_t len = segs[s].len;
    for (int64_t i = threadIdx.x; i < len; i += blockDim.x) dst[i] = src[i];
  }
}

int launch_seg_copy(const Seg* segs, int n, void* stream) {
  if (n <= 0) return 0;
  const int grid = n < 4096 ? n : 4096;
  hipLaunchKernelGGL(seg_copy_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, segs, n);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace dmpc
