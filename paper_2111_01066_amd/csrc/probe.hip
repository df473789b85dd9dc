// Measurement probes of the machine ceilings that the kernels are compared
// against: an MFMA issue loop per data type (no memory traffic) and a
// streaming device copy with 16-byte accesses.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace tnrcs {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kProbeBlocks = 2048;
constexpr int kProbeChains = 4;  // independent accumulators per wave

// Each wave keeps kProbeChains 32x32 accumulators and issues `iters` rounds
// of one MFMA per accumulator; the operands depend on the thread id so the
// compiler cannot fold them, and the sum of the results is stored so it
// cannot drop them.
template <int KIND>
__global__ __launch_bounds__(256) void k_mfma_peak(int64_t iters, float* out) {
  floatx16 acc[kProbeChains];
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c) acc[c] = floatx16{};
  const float x = 1.0f + 1e-7f * (float)(threadIdx.x & 7);
  if constexpr (KIND == 0) {
    const float a = x, b = 1.0f / 1024.f;
    for (int64_t i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < kProbeChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[c], 0, 0, 0);
  } else if constexpr (KIND == 1) {
    half8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      a[j] = (_Float16)x;
      b[j] = (_Float16)(1.0f / 1024.f);
    }
    for (int64_t i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < kProbeChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[c], 0, 0, 0);
  } else {
    bf16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      a[j] = (__bf16)x;
      b[j] = (__bf16)(1.0f / 1024.f);
    }
    for (int64_t i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < kProbeChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kProbeChains; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[c][r];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

hipError_t launch_mfma_peak(int kind, int64_t iters, float* out, double* flops, hipStream_t s) {
  // per wave and MFMA: 32*32*K multiply-adds, K = 2 (FP32) or 16 (FP16/BF16)
  const double per = 2.0 * 32 * 32 * (kind == 0 ? 2 : 16);
  *flops = per * kProbeChains * (double)iters * (kProbeBlocks * 256 / 64);
  const dim3 g(kProbeBlocks), b(256);
  if (kind == 0)
    hipLaunchKernelGGL(k_mfma_peak<0>, g, b, 0, s, iters, out);
  else if (kind == 1)
    hipLaunchKernelGGL(k_mfma_peak<1>, g, b, 0, s, iters, out);
  else
    hipLaunchKernelGGL(k_mfma_peak<2>, g, b, 0, s, iters, out);
  return hipGetLastError();
}

int64_t mfma_peak_out_floats() { return (int64_t)kProbeBlocks * 256; }

// Streaming copy: grid-stride over 16-byte words, eight nontemporal loads in
// flight per thread before their eight nontemporal stores, 16384 blocks of
// 256 threads (64 per CU).  Of the forms timed on a 4 GiB copy (1024 to
// 65536 blocks; 4, 8 or 16 words per thread; grid-stride or one contiguous
// chunk per block; plain or nontemporal loads and stores) this is among the
// fastest, level with the runtime's device-to-device copy.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyUnroll = 8;

__global__ __launch_bounds__(256) void k_stream_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                    int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (kCopyUnroll - 1) * stride < n; i += kCopyUnroll * stride) {
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) v[u] = __builtin_nontemporal_load(&src[i + u * stride]);
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) __builtin_nontemporal_store(v[u], &dst[i + u * stride]);
  }
  for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

hipError_t launch_stream_copy(const void* src, void* dst, int64_t n16, hipStream_t s) {
  if (n16 <= 0) return hipSuccess;
  const int64_t grid = std::min<int64_t>((n16 + 255) / 256, 16384);
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)grid), dim3(256), 0, s, (const u32x4*)src, (u32x4*)dst, n16);
  return hipGetLastError();
}

}  // namespace tnrcs
