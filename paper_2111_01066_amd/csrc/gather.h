// Address-ordered gathers of a 128-row x 16-k (or 32-k) chunk of an
// operand stored in an arbitrary bit layout (internal): shared by the skewed
// matrix-core kernels and the complex GEMMs that read their large operand in
// place.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tnrcs {

constexpr int kSkewMaxV = 12;  // index bits of one chunk: 7 row bits + up to 5 k bits

// Address order of one chunk: chunk element e (0 .. 2^v) has its bit i at
// A position pos[i], and is row bit mb[i] (or -1) / k bit kb[i] (or -1) of
// the chunk; the bits are sorted by A position.  Row m, k of the chunk sits
// in LDS at k * (row stride) + (m ^ h), h = XOR of hk[i] over the set k bits
// i and of hm[j] over the set row bits 5 + j: a swizzle that keeps the 32
// rows a matrix-core operand reads at one k in 32 distinct banks, and gives
// the 32 entries that one half-wave stores (consecutive in address order)
// distinct banks too.  All-zero hk and hm: no swizzle.
struct SkewMap {
  int32_t v;
  int8_t pos[kSkewMaxV];
  int8_t mb[kSkewMaxV];
  int8_t kb[kSkewMaxV];
  int8_t hk[5];
  int8_t hm[2];
};

__device__ __forceinline__ int skew_h(const SkewMap& mp, int m, int k) {
  int h = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i)
    if ((k >> i) & 1) h ^= mp.hk[i];
#pragma unroll
  for (int j = 0; j < 2; ++j)
    if ((m >> (5 + j)) & 1) h ^= mp.hm[j];
  return h;
}

// Chunk element e -> its offset from the chunk's first entry, its row m and
// its k within the chunk.  Unrolled over the largest map, so that the map's
// fields are read at fixed offsets of the kernel argument (scalar loads): the
// GEMMs that read A in place evaluate it in every workgroup, one per tile.
__device__ __forceinline__ void skew_split(const SkewMap& mp, int e, uint64_t& off, int& m, int& k) {
  off = 0;
  m = 0;
  k = 0;
#pragma unroll
  for (int i = 0; i < kSkewMaxV; ++i) {
    if (i < mp.v) {
      const int b = (e >> i) & 1;
      off |= (uint64_t)b << mp.pos[i];
      if (mp.mb[i] >= 0) m |= b << mp.mb[i];
      if (mp.kb[i] >= 0) k |= b << mp.kb[i];
    }
  }
}

// Host: the chunk map of rows 0..127 (op.aM bits 0..6) and k bits
// 0..kcb-1 (op.aK), with the bank swizzle for stores that cover chunk bits
// lv .. lv+4.  False when a bit has no position.
bool skew_map(const IndexOp& op, int kcb, int lv, SkewMap* mp);

}  // namespace tnrcs
