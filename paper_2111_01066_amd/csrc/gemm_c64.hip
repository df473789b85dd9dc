// Complex GEMM on FP32 matrix cores for complex64 storage (the matrix product
// of Supplement Eq. (matmul)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "elem.h"
#include "gather.h"
#include "kernels.h"

namespace tnrcs {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// ------------------------------------------------------------------- GEMM --
// C[M][N] = sum_k A[M][K] B[N][K], complex64 in and out, FP32 accumulation on
// v_mfma_f32_32x32x2_f32.  4M form: Cr += ArBr + (-Ai)Bi, Ci += ArBi + AiBr
// (four real products).  3M form: T1 = ArBr, T2 = AiBi,
// T3 = (Ar+Ai)(Br+Bi); Cr = T1 - T2, Ci = T3 - T1 - T2 (three products).
// Workgroup tile 64x64, four waves of 32x32, K staged through LDS in steps of
// 16 with re/im split into planar arrays.

constexpr int GBM = 64, GBN = 64, GBK = 16;

// blockIdx.z selects a batch entry or a split-K slab through the strides sA,
// sB, sC; each sums k_len terms of rows that are K long.
template <int FORM>
__global__ __launch_bounds__(256) void k_cgemm(const float2* __restrict__ A, const float2* __restrict__ B,
                                              float2* __restrict__ C, int64_t N, int64_t K, int64_t k_len,
                                              int64_t sA, int64_t sB, int64_t sC, int chunk) {
  __shared__ float As[2][GBK][GBM + 4];
  __shared__ float Bs[2][GBK][GBN + 4];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t bm = (int64_t)blockIdx.x * GBM, bn = (int64_t)blockIdx.y * GBN;
  const int64_t z = blockIdx.z;
  A += z * sA;
  B += z * sB;
  C += z * sC;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  floatx16 c0 = {}, c1 = {}, c2 = {};
  const int lrow = tid >> 2, lk = (tid & 3) * 4;
  const float2* Ap = A + (bm + lrow) * K + lk;
  const float2* Bp = B + (bn + lrow) * K + lk;
  const int j = lane & 31;
  // adds (ADD false: stores) the running FP32 sums to C and restarts them
  auto flush = [&](auto add) {
    constexpr bool ADD = decltype(add)::value;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      float2 v;
      if (FORM == TN_GEMM_3M) {
        v.x = c0[r] - c1[r];
        v.y = c2[r] - c0[r] - c1[r];
      } else {
        v.x = c0[r];
        v.y = c1[r];
      }
      float2* p = C + (bm + wm + i) * N + bn + wn + j;
      if constexpr (ADD) {
        const float2 o = *p;
        v.x += o.x;
        v.y += o.y;
      }
      *p = v;
    }
    c0 = floatx16{};
    c1 = floatx16{};
    c2 = floatx16{};
  };
  bool first = true;
  int it = 0;
  for (int64_t k0 = 0; k0 < k_len; k0 += GBK, ++it) {
    if (chunk > 0 && it > 0 && it % chunk == 0) {
      if (first)
        flush(std::false_type{});
      else
        flush(std::true_type{});
      first = false;
    }
    const float4 a01 = *reinterpret_cast<const float4*>(Ap + k0);
    const float4 a23 = *reinterpret_cast<const float4*>(Ap + k0 + 2);
    const float4 b01 = *reinterpret_cast<const float4*>(Bp + k0);
    const float4 b23 = *reinterpret_cast<const float4*>(Bp + k0 + 2);
    As[0][lk + 0][lrow] = a01.x;
    As[1][lk + 0][lrow] = a01.y;
    As[0][lk + 1][lrow] = a01.z;
    As[1][lk + 1][lrow] = a01.w;
    As[0][lk + 2][lrow] = a23.x;
    As[1][lk + 2][lrow] = a23.y;
    As[0][lk + 3][lrow] = a23.z;
    As[1][lk + 3][lrow] = a23.w;
    Bs[0][lk + 0][lrow] = b01.x;
    Bs[1][lk + 0][lrow] = b01.y;
    Bs[0][lk + 1][lrow] = b01.z;
    Bs[1][lk + 1][lrow] = b01.w;
    Bs[0][lk + 2][lrow] = b23.x;
    Bs[1][lk + 2][lrow] = b23.y;
    Bs[0][lk + 3][lrow] = b23.z;
    Bs[1][lk + 3][lrow] = b23.w;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 2) {
      const int kr = kk + (lane >> 5);
      const float ar = As[0][kr][wm + (lane & 31)];
      const float ai = As[1][kr][wm + (lane & 31)];
      const float br = Bs[0][kr][wn + (lane & 31)];
      const float bi = Bs[1][kr][wn + (lane & 31)];
      if (FORM == TN_GEMM_3M) {
        c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, bi, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar + ai, br + bi, c2, 0, 0, 0);
      } else {
        c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, c0, 0, 0, 0);
        c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai, bi, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi, c1, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, br, c1, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  if (first)
    flush(std::false_type{});
  else
    flush(std::true_type{});
}

// A read in place (GA = 1): the large operand's rows and contracted bits
// sit anywhere in its stored layout (row bit i at the position of aM bit i,
// k bit i at that of aK bit i, the k bits above 3 in increasing positions),
// so no permute runs before the product.  Each 128 x 16 chunk is gathered in
// A's address order (the chunk map) in 16-byte loads of two entries: A's
// lowest index bit is the lowest row or k bit, so it belongs to the chunk.
// The chunk's K offset moves by a carrying add restricted to the K bits
// (valid because they are in increasing positions).
struct GatherA {
  SkewMap mp;
  Runs aM;
  uint64_t maskK = 0, incK = 0;
};

// 128x128 workgroup tile, four waves of 64x64 (2x2 blocks of 32x32 MFMA
// tiles), K staged through LDS 16 at a time; the next K tile is loaded into
// registers while the current one is multiplied.  Planar LDS: re, im; the
// 3M operand sums re+im are formed in registers after the LDS reads, which
// keeps the kernel within 256 registers per lane (two waves per SIMD).
// blockIdx.z selects a batch entry or a split-K slab through the strides sA,
// sB, sC (GA = 0 only).
template <int FORM, int GA>
__global__ __launch_bounds__(256, 2) void k_cgemm128(const float2* __restrict__ A, const float2* __restrict__ B,
                                                 float2* __restrict__ C, int64_t N, int64_t K, int64_t k_len,
                                                 int64_t sA, int64_t sB, int64_t sC, int64_t Mt, int64_t Nt,
                                                 int chunk, const GatherA g) {
  constexpr int P = (FORM == TN_GEMM_3M) ? 3 : 2;
  constexpr int BM = 128, BN = 128, BK = 16, LD = BM + 2;
  constexpr int LPT = 4;  // gathered A: 16-byte loads per thread per chunk
  __shared__ float As[2][BK][LD];
  __shared__ float Bs[2][BK][LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t tm, tn, z;
  xcd_tile(blockIdx.x, Mt, Nt, gridDim.x, tm, tn, z);
  const int64_t bm = tm * BM, bn = tn * BN;
  A += z * sA;
  B += z * sB;
  C += z * sC;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  floatx16 acc[P][2][2];
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[p][i][j] = floatx16{};
  const int lrow = tid >> 1, lk = (tid & 1) * 8;
  const float2* Ap = A + (bm + lrow) * K + lk;
  const float2* Bp = B + (bn + lrow) * K + lk;
  float4 ra[4], rb[4];
  // gathered A: this thread's two entries per load (offset of the first
  // from the chunk's first entry; LDS indices k * LD + m of both, packed in
  // 16 bits each), the tile's row offset and the chunk's K offset
  uint32_t eoff[GA ? LPT : 1], eidx[GA ? LPT : 1];
  uint64_t abase = 0, kofs = 0;
  float4 rg[GA ? LPT : 1];
  if constexpr (GA != 0) {
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
      uint64_t off, off1;
      int m0, k0, m1, k1;
      skew_split(g.mp, (j * 256 + tid) * 2, off, m0, k0);
      skew_split(g.mp, (j * 256 + tid) * 2 + 1, off1, m1, k1);
      eoff[j] = (uint32_t)off;
      eidx[j] = (uint32_t)(k0 * LD + m0) | ((uint32_t)(k1 * LD + m1) << 16);
    }
    abase = dep_u<12>((uint64_t)bm, g.aM);
  }
  auto load_a = [&]() {
    if constexpr (GA != 0) {
      const float2* base = A + (abase + kofs);
#pragma unroll
      for (int j = 0; j < LPT; ++j) rg[j] = *reinterpret_cast<const float4*>(base + eoff[j]);
    }
  };
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if constexpr (GA == 0) ra[j] = *reinterpret_cast<const float4*>(Ap + 2 * j);
    rb[j] = *reinterpret_cast<const float4*>(Bp + 2 * j);
  }
  load_a();
  const int c = lane & 31, kh = lane >> 5;
  // Adds (ADD false: stores) the running FP32 sums to C and restarts them.
  // Called every `chunk` K stages, where the staged operands have just been
  // written to LDS and the prefetch registers are free, so one FP32
  // accumulation chain covers at most chunk * BK terms.
  auto flush = [&](auto add) {
    constexpr bool ADD = decltype(add)::value;
    // the row stride is made opaque here so that the compiler does not keep
    // the 64 output addresses live across the K loop
    int64_t ld = N;
    asm volatile("" : "+s"(ld));
    float2* Cw = C + (bm + wm + 4 * kh) * ld + bn + wn + c;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          float2 v;
          if (FORM == TN_GEMM_3M) {
            v.x = acc[0][i][j][r] - acc[1][i][j][r];
            v.y = acc[P - 1][i][j][r] - acc[0][i][j][r] - acc[1][i][j][r];
          } else {
            v.x = acc[0][i][j][r];
            v.y = acc[1][i][j][r];
          }
          float2* p = Cw + (32 * i + 8 * (r >> 2) + (r & 3)) * ld + 32 * j;
          if constexpr (ADD) {
            const float2 o = *p;
            v.x += o.x;
            v.y += o.y;
          }
          *p = v;
        }
#pragma unroll
        for (int q = 0; q < P; ++q) acc[q][i][j] = floatx16{};
        __builtin_amdgcn_sched_barrier(0);  // one 32x32 block's loads in flight at a time
      }
  };
  bool first = true;
  int it = 0;
  for (int64_t k0 = 0; k0 < k_len; k0 += BK, ++it) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (GA == 0) {
        As[0][lk + 2 * j][lrow] = ra[j].x;
        As[1][lk + 2 * j][lrow] = ra[j].y;
        As[0][lk + 2 * j + 1][lrow] = ra[j].z;
        As[1][lk + 2 * j + 1][lrow] = ra[j].w;
      }
      Bs[0][lk + 2 * j][lrow] = rb[j].x;
      Bs[1][lk + 2 * j][lrow] = rb[j].y;
      Bs[0][lk + 2 * j + 1][lrow] = rb[j].z;
      Bs[1][lk + 2 * j + 1][lrow] = rb[j].w;
    }
    if constexpr (GA != 0) {
      float* a0 = &As[0][0][0];
      float* a1 = &As[1][0][0];
#pragma unroll
      for (int j = 0; j < LPT; ++j) {
        const int i0 = (int)(eidx[j] & 0xffffu), i1 = (int)(eidx[j] >> 16);
        a0[i0] = rg[j].x;
        a1[i0] = rg[j].y;
        a0[i1] = rg[j].z;
        a1[i1] = rg[j].w;
      }
    }
    if (chunk > 0 && it > 0 && it % chunk == 0) {
      if (first)
        flush(std::false_type{});
      else
        flush(std::true_type{});
      first = false;
    }
    __syncthreads();
    if (k0 + BK < k_len) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if constexpr (GA == 0) ra[j] = *reinterpret_cast<const float4*>(Ap + k0 + BK + 2 * j);
        rb[j] = *reinterpret_cast<const float4*>(Bp + k0 + BK + 2 * j);
      }
      if constexpr (GA != 0) {
        kofs = ((kofs | ~g.maskK) + g.incK) & g.maskK;
        load_a();
      }
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const int kr = kk + kh;
      float a[P][2], b[P][2];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a[p][i] = As[p][kr][wm + 32 * i + c];
          b[p][i] = Bs[p][kr][wn + 32 * i + c];
        }
      if (P == 3)  // 3M operand sums, formed in FP32 from the staged re/im
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a[P - 1][i] = a[0][i] + a[1][i];
          b[P - 1][i] = b[0][i] + b[1][i];
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (FORM == TN_GEMM_3M) {
            acc[0][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][i], b[0][j], acc[0][i][j], 0, 0, 0);
            acc[1][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1][i], b[1][j], acc[1][i][j], 0, 0, 0);
            acc[P - 1][i][j] =
                __builtin_amdgcn_mfma_f32_32x32x2f32(a[P - 1][i], b[P - 1][j], acc[P - 1][i][j], 0, 0, 0);
          } else {
            acc[0][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][i], b[0][j], acc[0][i][j], 0, 0, 0);
            acc[0][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(-a[1][i], b[1][j], acc[0][i][j], 0, 0, 0);
            acc[1][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][i], b[1][j], acc[1][i][j], 0, 0, 0);
            acc[1][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1][i], b[0][j], acc[1][i][j], 0, 0, 0);
          }
        }
    }
  }
  if (first)
    flush(std::false_type{});
  else
    flush(std::true_type{});
}

// C[i] = sum over slabs s (in order) of W[s][i], summed in FP64 and rounded
// once.
__global__ __launch_bounds__(256) void k_splitk_sum(const float2* __restrict__ W, float2* __restrict__ C, int64_t n,
                                                   int slabs) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double r = 0.0, im = 0.0;
    for (int sl = 0; sl < slabs; ++sl) {
      const float2 v = W[(int64_t)sl * n + i];
      r += (double)v.x;
      im += (double)v.y;
    }
    C[i] = make_float2((float)r, (float)im);
  }
}

bool gemm_shape_ok(int64_t M, int64_t N, int64_t K) {
  return M > 0 && N > 0 && K > 0 && M % GBM == 0 && N % GBN == 0 && K % GBK == 0;
}

hipError_t launch_gemm_c64(const float2* A, const float2* B, float2* C, int64_t M, int64_t N, int64_t K,
                           int64_t batch, int form, hipStream_t s, float2* work, int splits, int tile) {
  if (!gemm_shape_ok(M, N, K) || batch < 0) return hipErrorInvalidValue;
  if (batch == 0) return hipSuccess;
  if (splits < 1) splits = 1;
  const bool fits128 = (M % 128 == 0) && (N % 128 == 0);
  if (tile == 128 && !fits128) return hipErrorInvalidValue;
  if (tile == 64 && splits > 1) return hipErrorInvalidValue;
  const bool big = fits128 && tile != 64;
  const int chunk = kAccChain / 16;  // K stages of the 128x128 kernel per FP32 chain
  if (splits > 1) {
    if (batch != 1 || !work || K % (16 * splits) != 0 || splits > 65535) return hipErrorInvalidValue;
    const int64_t kl = K / splits;
    const int64_t n = M * N;
    if (!big) {  // 64x64 tiles, one slab per blockIdx.z
      if (N / GBN > 65535) return hipErrorInvalidValue;
      dim3 grid((unsigned)(M / GBM), (unsigned)(N / GBN), (unsigned)splits);
      if (form == TN_GEMM_3M)
        hipLaunchKernelGGL(k_cgemm<TN_GEMM_3M>, grid, dim3(256), 0, s, A, B, work, N, K, kl, kl, kl, n,
                           kAccChain / GBK);
      else
        hipLaunchKernelGGL(k_cgemm<TN_GEMM_4M>, grid, dim3(256), 0, s, A, B, work, N, K, kl, kl, kl, n,
                           kAccChain / GBK);
      hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0, s,
                         work, C, n, splits);
      return hipGetLastError();
    }
    const int64_t Mt = M / 128, Nt = N / 128;
    dim3 grid((unsigned)(Mt * Nt * splits));
    if (form == TN_GEMM_3M)
      hipLaunchKernelGGL((k_cgemm128<TN_GEMM_3M, 0>), grid, dim3(256), 0, s, A, B, work, N, K, kl, kl, kl, M * N, Mt, Nt,
                         chunk, GatherA{});
    else
      hipLaunchKernelGGL((k_cgemm128<TN_GEMM_4M, 0>), grid, dim3(256), 0, s, A, B, work, N, K, kl, kl, kl, M * N, Mt, Nt,
                         chunk, GatherA{});
    hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0, s,
                       work, C, n, splits);
    return hipGetLastError();
  }
  if (batch > 65535) return hipErrorInvalidValue;
  // short contractions are store-bound: the 64x64 kernel keeps more
  // workgroups in flight
  if (big && (K > 64 || tile == 128)) {
    const int64_t Mt = M / 128, Nt = N / 128;
    dim3 grid((unsigned)(Mt * Nt * batch));
    if (form == TN_GEMM_3M)
      hipLaunchKernelGGL((k_cgemm128<TN_GEMM_3M, 0>), grid, dim3(256), 0, s, A, B, C, N, K, K, M * K, N * K, M * N, Mt, Nt,
                         chunk, GatherA{});
    else
      hipLaunchKernelGGL((k_cgemm128<TN_GEMM_4M, 0>), grid, dim3(256), 0, s, A, B, C, N, K, K, M * K, N * K, M * N, Mt, Nt,
                         chunk, GatherA{});
    return hipGetLastError();
  }
  if (N / GBN > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)(M / GBM), (unsigned)(N / GBN), (unsigned)batch);
  if (form == TN_GEMM_3M)
    hipLaunchKernelGGL(k_cgemm<TN_GEMM_3M>, grid, dim3(256), 0, s, A, B, C, N, K, K, M * K, N * K, M * N,
                       kAccChain / GBK);
  else
    hipLaunchKernelGGL(k_cgemm<TN_GEMM_4M>, grid, dim3(256), 0, s, A, B, C, N, K, K, M * K, N * K, M * N,
                       kAccChain / GBK);
  return hipGetLastError();
}

static uint64_t dep_host(uint64_t x, const Runs& r) {
  uint64_t o = 0;
  for (int i = 0; i < r.n; ++i) o |= ((x >> r.src[i]) & ((1ull << r.len[i]) - 1ull)) << r.dst[i];
  return o;
}

hipError_t launch_gemm_c64_ga(const float2* A, const float2* B, float2* C, const IndexOp& idx, int form,
                              hipStream_t s) {
  if (!gemm_gather_ok(idx)) return hipErrorInvalidValue;
  const int64_t M = (int64_t)1 << idx.nM, N = (int64_t)1 << idx.nN, K = (int64_t)1 << idx.nK;
  GatherA g{};
  skew_map(idx, 4, 0, &g.mp);
  g.aM = idx.aM;
  g.maskK = dep_host((uint64_t)(K - 1) & ~(uint64_t)15, idx.aK);
  g.incK = K > 16 ? dep_host(16, idx.aK) : 0;
  if (g.mp.pos[0] != 0) return hipErrorInvalidValue;  // A's lowest bit must belong to the chunk
  const int chunk = kAccChain / 16;
  const int64_t Mt = M / 128, Nt = N / 128;
  const dim3 grid((unsigned)(Mt * Nt));
  if (form == TN_GEMM_3M)
    hipLaunchKernelGGL((k_cgemm128<TN_GEMM_3M, 1>), grid, dim3(256), 0, s, A, B, C, N, K, K, 0, 0, 0, Mt, Nt, chunk, g);
  else
    hipLaunchKernelGGL((k_cgemm128<TN_GEMM_4M, 1>), grid, dim3(256), 0, s, A, B, C, N, K, K, 0, 0, 0, Mt, Nt, chunk, g);
  return hipGetLastError();
}

}  // namespace tnrcs
