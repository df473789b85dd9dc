// Device element types of the tnrcs kernels and their FP32 views (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tnrcs {

// Complex storage formats: complex64 (re, im FP32), and FP16 / BF16 pairs
// that hold a value times 2^-e for a per-tensor exponent e.
struct alignas(4) cf16 {
  _Float16 re, im;
};
struct alignas(4) cbf16 {
  __bf16 re, im;
};

__device__ __forceinline__ float2 to_f2(float2 v) { return v; }
__device__ __forceinline__ float2 to_f2(cf16 v) { return make_float2((float)v.re, (float)v.im); }
__device__ __forceinline__ float2 to_f2(cbf16 v) { return make_float2((float)v.re, (float)v.im); }

template <typename E>
__device__ __forceinline__ E from_f2(float re, float im);
template <>
__device__ __forceinline__ float2 from_f2<float2>(float re, float im) {
  return make_float2(re, im);
}
template <>
__device__ __forceinline__ cf16 from_f2<cf16>(float re, float im) {
  cf16 v;
  v.re = (_Float16)re;
  v.im = (_Float16)im;
  return v;
}
template <>
__device__ __forceinline__ cbf16 from_f2<cbf16>(float re, float im) {
  cbf16 v;
  v.re = (__bf16)re;
  v.im = (__bf16)im;
  return v;
}

__device__ __forceinline__ uint64_t dep(uint64_t x, const Runs& r) {
  uint64_t o = 0;
  for (int i = 0; i < r.n; ++i) o |= ((x >> r.src[i]) & ((1ull << r.len[i]) - 1ull)) << r.dst[i];
  return o;
}

// The same with the first N runs unrolled: their fields are read at fixed
// offsets of the kernel argument (scalar loads) instead of at a run index
// (a vector load per field), for maps evaluated once per output tile.
template <int N>
__device__ __forceinline__ uint64_t dep_u(uint64_t x, const Runs& r) {
  uint64_t o = 0;
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (i < r.n) o |= ((x >> r.src[i]) & ((1ull << r.len[i]) - 1ull)) << r.dst[i];
  for (int i = N; i < r.n; ++i) o |= ((x >> r.src[i]) & ((1ull << r.len[i]) - 1ull)) << r.dst[i];
  return o;
}

// Running maximum of |re|, |im| for the range check of scaled storage; a
// NaN counts as +inf (it comes from an overflow earlier in the same sum).
__device__ __forceinline__ float mag_max(float m, float re, float im) {
  const float t = fmaxf(m, fmaxf(fabsf(re), fabsf(im)));
  return (re != re || im != im) ? INFINITY : t;  // a select, not a branch
}

// Largest |component| over a workgroup, folded into *slot (non-negative
// floats order like their bit patterns).  One atomic per workgroup at most,
// and none once the record already holds a larger value.  Every thread of
// the workgroup must call it.
__device__ __forceinline__ void record_max_in(float* slot, float v, float* wmax) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) wmax[w] = v;
  __syncthreads();
  if (threadIdx.x == 0 && slot) {
    float m = wmax[0];
    for (int i = 1; i < nw; ++i) m = fmaxf(m, wmax[i]);
    unsigned int* u = reinterpret_cast<unsigned int*>(slot);
    const unsigned int bits = __float_as_uint(m);
    if (bits > __atomic_load_n(u, __ATOMIC_RELAXED)) atomicMax(u, bits);
  }
}

__device__ __forceinline__ void record_max(float* slot, float v) {
  __shared__ float wmax[16];
  record_max_in(slot, v, wmax);
}

// Workgroups are dealt to the 8 XCDs round-robin by id.  This maps a
// workgroup id to (tile_m, tile_n, z) so that every XCD receives one
// contiguous range of logical tiles, walked in groups of up to 8 tile-rows:
// the workgroups running together on one XCD share A and B panels in its L2.
__device__ __forceinline__ void xcd_tile(int64_t L, int64_t Mt, int64_t Nt, int64_t G, int64_t& tm, int64_t& tn,
                                         int64_t& z) {
  int64_t t = L;
  if ((G & 7) == 0) t = (L & 7) * (G >> 3) + (L >> 3);
  const int64_t per_z = Mt * Nt;
  z = t / per_z;
  t -= z * per_z;
  const int64_t gm = Mt < 8 ? Mt : 8;
  const int64_t base = (t / (gm * Nt)) * gm;  // first tile-row of this group
  const int64_t gh = Mt - base < gm ? Mt - base : gm;  // rows in this (possibly last, partial) group
  const int64_t r = t - base * Nt;
  tm = base + r % gh;
  tn = r / gh;
}

}  // namespace tnrcs
