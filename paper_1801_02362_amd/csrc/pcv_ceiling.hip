// Streaming-read ceiling: a device buffer read once, 16 bytes per lane per
// load, non-temporal, two sets of loads in flight per wave (the landmark
// engines' load path without their arithmetic or synchronisation).  Each
// workgroup reads one contiguous chunk and writes the FP64 sum of its
// floats, so the loads cannot be elided and the result can be checked.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pcv.h"
#include "pcv_internal.h"

namespace pcv {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kCeilWG = 512;   // eight waves
constexpr int kDepth = 8;      // 16-byte loads per lane per set

__global__ __launch_bounds__(kCeilWG) void stream_read_kernel(const f4v* __restrict__ a, size_t n4,
                                                              double* __restrict__ wg_sums) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t per = (n4 + gridDim.x - 1) / gridDim.x;
  size_t b = (size_t)blockIdx.x * per;
  const size_t e = b + per < n4 ? b + per : n4;
  if (b > e) b = e;
  constexpr size_t stride = (size_t)kCeilWG * kDepth;   // float4 per workgroup round
  const size_t off = (size_t)wave * 64 * kDepth + lane;
  f4v acc = {0.f, 0.f, 0.f, 0.f};
  auto ld = [&](f4v (&v)[kDepth], size_t base) {
#pragma unroll
    for (int d = 0; d < kDepth; ++d) v[d] = ldg_nt(a + base + off + (size_t)d * 64);
  };
  // Full rounds only: every index base + off + 64 d < base + stride <= e.
  if (b + stride <= e) {
    f4v cur[kDepth];
    ld(cur, b);
    for (;;) {
      const size_t nb = b + stride;
      if (nb + stride <= e) {
        f4v nxt[kDepth];
        ld(nxt, nb);
#pragma unroll
        for (int d = 0; d < kDepth; ++d) acc += cur[d];
#pragma unroll
        for (int d = 0; d < kDepth; ++d) cur[d] = nxt[d];
        b = nb;
      } else {
#pragma unroll
        for (int d = 0; d < kDepth; ++d) acc += cur[d];
        b = nb;
        break;
      }
    }
  }
  for (size_t j = b + threadIdx.x; j < e; j += kCeilWG) acc += ldg(a + j);
  double v = (double)acc.x + (double)acc.y + (double)acc.z + (double)acc.w;
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  __shared__ double sh[kCeilWG / 64];
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kCeilWG / 64; ++w) t += sh[w];
    wg_sums[blockIdx.x] = t;
  }
}

}  // namespace

}  // namespace pcv

extern "C" pcv_status pcv_stream_read(const void* src, size_t bytes, double* wg_sums, int grid, void* stream) {
  if (!src || !wg_sums || bytes == 0 || bytes % 16 != 0 || grid < 1 || grid > 65536) return PCV_EINVAL;
  if (((uintptr_t)src & 15) != 0) return PCV_EINVAL;
  hipLaunchKernelGGL(pcv::stream_read_kernel, dim3(grid), dim3(pcv::kCeilWG), 0, (hipStream_t)stream,
                     (const pcv::f4v*)src, bytes / 16, wg_sums);
  return hipGetLastError() == hipSuccess ? PCV_OK : PCV_EHIP;
}
