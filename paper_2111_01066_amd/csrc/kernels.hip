// gfx950 kernels of the tnrcs library: slice binding, tiled binary-index
// permutation, complex GEMM from real MFMA products (4M / 3M), generic
// gathered contraction, FP64 slice accumulation and FP64 reductions.
//
// Paper anchors: each pairwise contraction is an index permutation followed by
// a complex matrix product (Supplement Eq. (matmul)); slicing sums smaller
// networks (main text, customized-TNC section); XEB / Porter-Thomas checks
// (main text Eq. (fxeb)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "kernels.h"

namespace tnrcs {

typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint64_t dep(uint64_t x, const Runs& r) {
  uint64_t o = 0;
  for (int i = 0; i < r.n; ++i) o |= ((x >> r.src[i]) & ((1ull << r.len[i]) - 1ull)) << r.dst[i];
  return o;
}

// ---------------------------------------------------------------- control --

__global__ void k_set_ctrl(Ctrl* ctrl, int64_t cursor, void* amp) {
  ctrl->cursor = cursor;
  ctrl->amp = (double*)amp;
}

hipError_t launch_set_ctrl(Ctrl* ctrl, int64_t cursor, void* amp, hipStream_t s) {
  hipLaunchKernelGGL(k_set_ctrl, dim3(1), dim3(1), 0, s, ctrl, cursor, amp);
  return hipGetLastError();
}

// ------------------------------------------------------------------- bind --
// Copies, for every sliced leaf, the sub-tensor selected by the current slice
// id (its sliced wires are the leaf's top bits) into the bound-leaf region.

__global__ __launch_bounds__(256) void k_bind(const float2* __restrict__ leaves, float2* __restrict__ bound,
                                              const BindDesc* __restrict__ descs, const Ctrl* __restrict__ ctrl) {
  const BindDesc& d = descs[blockIdx.y];
  const int64_t s = ctrl->cursor;
  int64_t off = 0;
  for (int i = 0; i < d.n_sl; ++i) off |= ((s >> d.sbit[i]) & 1ll) << d.pos[i];
  const float2* src = leaves + d.src_off + off;
  float2* dst = bound + d.dst_off;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < d.n_elems;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

hipError_t launch_bind(const float2* leaves, float2* bound, const BindDesc* descs, int n_desc, int64_t max_elems,
                       const Ctrl* ctrl, hipStream_t s) {
  if (n_desc <= 0) return hipSuccess;
  int64_t gx = std::min<int64_t>((max_elems + 255) / 256, 1024);
  hipLaunchKernelGGL(k_bind, dim3((unsigned)std::max<int64_t>(gx, 1), n_desc), dim3(256), 0, s, leaves, bound,
                     descs, ctrl);
  return hipGetLastError();
}

// ---------------------------------------------------------------- permute --
// Tile = the input-fast bits I plus the output-fast bits O of the index.  A
// tile is read with runs of 2^|I| consecutive input elements, staged in LDS,
// and written with runs of 2^|O| consecutive output elements.

constexpr int kPermTileBits = 12;
constexpr int kPermThreads = 256;

struct PermArgs {
  int64_t n_tiles;
  int64_t stride;  // batch stride (elements)
  int32_t tbits;
  Runs in_tile;   // tile element e (input-ascending T order) -> input offset
  Runs out_tile;  // tile element f (output-ascending T order) -> output offset
  Runs f2e;       // f -> e
  Runs id_in;     // tile id -> input offset
  Runs id_out;    // tile id -> output offset
};

__device__ __forceinline__ int lds_pad(int e) { return e + (e >> 4); }

// Tile of 2^TB elements, 256 threads, 2^TB / 256 elements per thread; all of
// a thread's loads are issued before any LDS store so they are in flight
// together.  The per-element parts of the offsets that depend only on the
// unrolled iteration are tabulated once in LDS.
template <int TB>
__global__ __launch_bounds__(kPermThreads) void k_permute(const float2* __restrict__ in, float2* __restrict__ out,
                                                         const PermArgs a) {
  constexpr int NT = 1 << TB;
  constexpr int PER = NT / kPermThreads;
  __shared__ float2 tile[NT + NT / 16];
  __shared__ uint64_t hi_in[PER], hi_out[PER];
  __shared__ int hi_fe[PER];
  const int tid = threadIdx.x;
  if (tid < PER) {
    hi_in[tid] = dep((uint64_t)tid * kPermThreads, a.in_tile);
    hi_out[tid] = dep((uint64_t)tid * kPermThreads, a.out_tile);
    hi_fe[tid] = (int)dep((uint64_t)tid * kPermThreads, a.f2e);
  }
  const float2* src = in + (int64_t)blockIdx.y * a.stride;
  float2* dst = out + (int64_t)blockIdx.y * a.stride;
  const uint64_t e_t = dep((uint64_t)tid, a.in_tile);
  const uint64_t f_t = dep((uint64_t)tid, a.out_tile);
  const int fe_t = (int)dep((uint64_t)tid, a.f2e);
  __syncthreads();
  for (int64_t t = blockIdx.x; t < a.n_tiles; t += gridDim.x) {
    const uint64_t ib = dep((uint64_t)t, a.id_in) | e_t;
    const uint64_t ob = dep((uint64_t)t, a.id_out) | f_t;
    float2 v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) v[i] = src[ib | hi_in[i]];
#pragma unroll
    for (int i = 0; i < PER; ++i) tile[lds_pad(i * kPermThreads + tid)] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) v[i] = tile[lds_pad(fe_t | hi_fe[i])];
#pragma unroll
    for (int i = 0; i < PER; ++i) dst[ob | hi_out[i]] = v[i];
    __syncthreads();
  }
}

// Tensors below 256 elements: one element per thread, direct gather.
__global__ __launch_bounds__(256) void k_permute_small(const float2* __restrict__ in, float2* __restrict__ out,
                                                      const PermArgs a) {
  const int64_t n = (int64_t)1 << a.tbits;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const float2* src = in + (int64_t)blockIdx.y * a.stride;
    float2* dst = out + (int64_t)blockIdx.y * a.stride;
    dst[dep((uint64_t)e, a.out_tile)] = src[dep((uint64_t)e, a.f2e)];
  }
}

hipError_t launch_permute_c64(const float2* in, float2* out, int rank, const int32_t* perm, int64_t batch,
                              hipStream_t s) {
  // inverse map: input position p -> output position inv[p]
  std::vector<int> inv(rank, -1);
  for (int q = 0; q < rank; ++q) {
    if (perm[q] < 0 || perm[q] >= rank || inv[perm[q]] >= 0) return hipErrorInvalidValue;
    inv[perm[q]] = q;
  }
  if (batch <= 0) return hipSuccess;
  if (batch > 65535) return hipErrorInvalidValue;
  PermArgs A{};
  A.stride = (int64_t)1 << rank;
  if (rank < 8) {
    // out index f: output position q holds input bit perm[q]
    std::vector<int> po, pi;
    for (int q = 0; q < rank; ++q) po.push_back(q);
    for (int q = 0; q < rank; ++q) pi.push_back(perm[q]);
    A.tbits = rank;
    A.n_tiles = 1;
    if (!make_runs(po, &A.out_tile) || !make_runs(pi, &A.f2e)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_permute_small, dim3(1, (unsigned)batch), dim3(256), 0, s, in, out, A);
    return hipGetLastError();
  }
  // choose the tile: grow input-fast and output-fast bit sets alternately
  std::vector<bool> inT(rank, false);
  int tb = 0, a = 0, b = 0;
  const int cap = std::min(kPermTileBits, rank);
  while (tb < cap) {
    bool grew = false;
    if (a < rank && (a <= b || b >= rank)) {
      if (!inT[a]) {
        inT[a] = true;
        ++tb;
      }
      ++a;
      grew = true;
    } else if (b < rank) {
      int p = perm[b];
      if (!inT[p]) {
        inT[p] = true;
        ++tb;
      }
      ++b;
      grew = true;
    }
    if (!grew) break;
  }
  std::vector<int> Tin, Tout, R;
  for (int p = 0; p < rank; ++p) (inT[p] ? Tin : R).push_back(p);
  Tout = Tin;
  std::sort(Tout.begin(), Tout.end(), [&](int x, int y) { return inv[x] < inv[y]; });
  A.tbits = (int)Tin.size();
  A.n_tiles = (int64_t)1 << (rank - A.tbits);
  std::vector<int> p1, p2, p3, p4, p5;
  for (int p : Tin) p1.push_back(p);
  for (int p : Tout) p2.push_back(inv[p]);
  for (int p : Tout) p3.push_back((int)(std::find(Tin.begin(), Tin.end(), p) - Tin.begin()));
  for (int p : R) p4.push_back(p);
  for (int p : R) p5.push_back(inv[p]);
  if (!make_runs(p1, &A.in_tile) || !make_runs(p2, &A.out_tile) || !make_runs(p3, &A.f2e) ||
      !make_runs(p4, &A.id_in) || !make_runs(p5, &A.id_out))
    return hipErrorInvalidValue;
  const int64_t grid = std::min<int64_t>(A.n_tiles, 16384);
  const dim3 g((unsigned)grid, (unsigned)batch);
  switch (A.tbits) {
    case 8:
      hipLaunchKernelGGL(k_permute<8>, g, dim3(kPermThreads), 0, s, in, out, A);
      break;
    case 9:
      hipLaunchKernelGGL(k_permute<9>, g, dim3(kPermThreads), 0, s, in, out, A);
      break;
    case 10:
      hipLaunchKernelGGL(k_permute<10>, g, dim3(kPermThreads), 0, s, in, out, A);
      break;
    case 11:
      hipLaunchKernelGGL(k_permute<11>, g, dim3(kPermThreads), 0, s, in, out, A);
      break;
    case 12:
      hipLaunchKernelGGL(k_permute<12>, g, dim3(kPermThreads), 0, s, in, out, A);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------- GEMM --
// C[M][N] = sum_k A[M][K] B[N][K], complex64 in and out, FP32 accumulation on
// v_mfma_f32_32x32x2_f32.  4M form: Cr += ArBr + (-Ai)Bi, Ci += ArBi + AiBr
// (four real products).  3M form: T1 = ArBr, T2 = AiBi,
// T3 = (Ar+Ai)(Br+Bi); Cr = T1 - T2, Ci = T3 - T1 - T2 (three products).
// Workgroup tile 64x64, four waves of 32x32, K staged through LDS in steps of
// 16 with re/im split into planar arrays.

constexpr int GBM = 64, GBN = 64, GBK = 16;

template <int FORM>
__global__ __launch_bounds__(256) void k_cgemm(const float2* __restrict__ A, const float2* __restrict__ B,
                                              float2* __restrict__ C, int64_t M, int64_t N, int64_t K) {
  __shared__ float As[2][GBK][GBM + 4];
  __shared__ float Bs[2][GBK][GBN + 4];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t bm = (int64_t)blockIdx.x * GBM, bn = (int64_t)blockIdx.y * GBN;
  const int64_t z = blockIdx.z;
  A += z * M * K;
  B += z * N * K;
  C += z * M * N;
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  floatx16 c0 = {}, c1 = {}, c2 = {};
  const int lrow = tid >> 2, lk = (tid & 3) * 4;
  const float2* Ap = A + (bm + lrow) * K + lk;
  const float2* Bp = B + (bn + lrow) * K + lk;
  for (int64_t k0 = 0; k0 < K; k0 += GBK) {
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
  const int j = lane & 31;
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
    C[(bm + wm + i) * N + bn + wn + j] = v;
  }
}

// 128x128 workgroup tile, four waves of 64x64 (2x2 blocks of 32x32 MFMA
// tiles), K staged through LDS 16 at a time; the next K tile is loaded into
// registers while the current one is multiplied.  Planar LDS: re, im (and,
// for 3M, re+im formed once per element when the tile is stored).  blockIdx.z
// selects a batch entry or a split-K slab through the strides sA, sB, sC.
template <int FORM>
__global__ __launch_bounds__(256) void k_cgemm128(const float2* __restrict__ A, const float2* __restrict__ B,
                                                 float2* __restrict__ C, int64_t N, int64_t K, int64_t k_len,
                                                 int64_t sA, int64_t sB, int64_t sC) {
  constexpr int P = (FORM == TN_GEMM_3M) ? 3 : 2;
  constexpr int BM = 128, BN = 128, BK = 16, LD = BM + 2;
  __shared__ float As[P][BK][LD];
  __shared__ float Bs[P][BK][LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t bm = (int64_t)blockIdx.x * BM, bn = (int64_t)blockIdx.y * BN;
  const int64_t z = blockIdx.z;
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
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ra[j] = *reinterpret_cast<const float4*>(Ap + 2 * j);
    rb[j] = *reinterpret_cast<const float4*>(Bp + 2 * j);
  }
  const int c = lane & 31, kh = lane >> 5;
  for (int64_t k0 = 0; k0 < k_len; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      As[0][lk + 2 * j][lrow] = ra[j].x;
      As[1][lk + 2 * j][lrow] = ra[j].y;
      As[0][lk + 2 * j + 1][lrow] = ra[j].z;
      As[1][lk + 2 * j + 1][lrow] = ra[j].w;
      Bs[0][lk + 2 * j][lrow] = rb[j].x;
      Bs[1][lk + 2 * j][lrow] = rb[j].y;
      Bs[0][lk + 2 * j + 1][lrow] = rb[j].z;
      Bs[1][lk + 2 * j + 1][lrow] = rb[j].w;
      if (P == 3) {
        As[P - 1][lk + 2 * j][lrow] = ra[j].x + ra[j].y;
        As[P - 1][lk + 2 * j + 1][lrow] = ra[j].z + ra[j].w;
        Bs[P - 1][lk + 2 * j][lrow] = rb[j].x + rb[j].y;
        Bs[P - 1][lk + 2 * j + 1][lrow] = rb[j].z + rb[j].w;
      }
    }
    __syncthreads();
    if (k0 + BK < k_len) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        ra[j] = *reinterpret_cast<const float4*>(Ap + k0 + BK + 2 * j);
        rb[j] = *reinterpret_cast<const float4*>(Bp + k0 + BK + 2 * j);
      }
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const int kr = kk + kh;
      float a[P][2], b[P][2];
#pragma unroll
      for (int p = 0; p < P; ++p)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a[p][i] = As[p][kr][wm + 32 * i + c];
          b[p][i] = Bs[p][kr][wn + 32 * i + c];
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
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wm + 32 * i + 8 * (r >> 2) + 4 * kh + (r & 3);
        const int col = wn + 32 * j + c;
        float2 v;
        if (FORM == TN_GEMM_3M) {
          v.x = acc[0][i][j][r] - acc[1][i][j][r];
          v.y = acc[P - 1][i][j][r] - acc[0][i][j][r] - acc[1][i][j][r];
        } else {
          v.x = acc[0][i][j][r];
          v.y = acc[1][i][j][r];
        }
        C[(bm + row) * N + bn + col] = v;
      }
}

// C[i] = sum over slabs s (in order) of W[s][i].
__global__ __launch_bounds__(256) void k_splitk_sum(const float2* __restrict__ W, float2* __restrict__ C, int64_t n,
                                                   int slabs) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float r = 0.f, im = 0.f;
    for (int sl = 0; sl < slabs; ++sl) {
      const float2 v = W[(int64_t)sl * n + i];
      r += v.x;
      im += v.y;
    }
    C[i] = make_float2(r, im);
  }
}

bool gemm_shape_ok(int64_t M, int64_t N, int64_t K) {
  return M > 0 && N > 0 && K > 0 && M % GBM == 0 && N % GBN == 0 && K % GBK == 0;
}

hipError_t launch_gemm_c64(const float2* A, const float2* B, float2* C, int64_t M, int64_t N, int64_t K,
                           int64_t batch, int form, hipStream_t s, float2* work, int splits) {
  if (!gemm_shape_ok(M, N, K) || batch < 0) return hipErrorInvalidValue;
  if (batch == 0) return hipSuccess;
  if (splits < 1) splits = 1;
  const bool big = (M % 128 == 0) && (N % 128 == 0);
  if (splits > 1) {
    if (batch != 1 || !work || !big || K % (16 * splits) != 0 || splits > 65535) return hipErrorInvalidValue;
    const int64_t kl = K / splits;
    dim3 grid((unsigned)(M / 128), (unsigned)(N / 128), (unsigned)splits);
    if (form == TN_GEMM_3M)
      hipLaunchKernelGGL(k_cgemm128<TN_GEMM_3M>, grid, dim3(256), 0, s, A, B, work, N, K, kl, kl, kl, M * N);
    else
      hipLaunchKernelGGL(k_cgemm128<TN_GEMM_4M>, grid, dim3(256), 0, s, A, B, work, N, K, kl, kl, kl, M * N);
    const int64_t n = M * N;
    hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0, s,
                       work, C, n, splits);
    return hipGetLastError();
  }
  if (batch > 65535) return hipErrorInvalidValue;
  if (big) {
    dim3 grid((unsigned)(M / 128), (unsigned)(N / 128), (unsigned)batch);
    if (form == TN_GEMM_3M)
      hipLaunchKernelGGL(k_cgemm128<TN_GEMM_3M>, grid, dim3(256), 0, s, A, B, C, N, K, K, M * K, N * K, M * N);
    else
      hipLaunchKernelGGL(k_cgemm128<TN_GEMM_4M>, grid, dim3(256), 0, s, A, B, C, N, K, K, M * K, N * K, M * N);
    return hipGetLastError();
  }
  dim3 grid((unsigned)(M / GBM), (unsigned)(N / GBN), (unsigned)batch);
  if (form == TN_GEMM_3M)
    hipLaunchKernelGGL(k_cgemm<TN_GEMM_3M>, grid, dim3(256), 0, s, A, B, C, M, N, K);
  else
    hipLaunchKernelGGL(k_cgemm<TN_GEMM_4M>, grid, dim3(256), 0, s, A, B, C, M, N, K);
  return hipGetLastError();
}

// ---------------------------------------------------------------- generic --
// One output element per thread: C[(m<<nN)|n] = sum_k A[dep(m)|dep(k)] B[dep(n)|dep(k)].

__global__ __launch_bounds__(256) void k_generic(const float2* __restrict__ A, const float2* __restrict__ B,
                                                float2* __restrict__ C, const IndexOp op) {
  const int64_t nC = (int64_t)1 << (op.nM + op.nN);
  const int64_t nK = (int64_t)1 << op.nK;
  const uint64_t nmask = (1ull << op.nN) - 1ull;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nC; c += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t m = (uint64_t)c >> op.nN, n = (uint64_t)c & nmask;
    const uint64_t ab = dep(m, op.aM), bb = dep(n, op.bN);
    float re = 0.f, im = 0.f;
    for (int64_t k = 0; k < nK; ++k) {
      const float2 x = A[ab | dep((uint64_t)k, op.aK)];
      const float2 y = B[bb | dep((uint64_t)k, op.bK)];
      re = fmaf(x.x, y.x, re);
      re = fmaf(-x.y, y.y, re);
      im = fmaf(x.x, y.y, im);
      im = fmaf(x.y, y.x, im);
    }
    C[c] = make_float2(re, im);
  }
}

hipError_t launch_generic_c64(const float2* A, const float2* B, float2* C, const IndexOp& op, hipStream_t s) {
  const int64_t nC = (int64_t)1 << (op.nM + op.nN);
  int64_t grid = std::min<int64_t>((nC + 255) / 256, 16384);
  hipLaunchKernelGGL(k_generic, dim3((unsigned)grid), dim3(256), 0, s, A, B, C, op);
  return hipGetLastError();
}

// ---------------------------------------------------------------- split-K --
// Few outputs (<= 64) and a long contraction: the K range is split over a
// fixed grid; each thread accumulates all outputs over its k's (consecutive
// threads take consecutive k, so the gathers are coalesced wherever the low
// K bits are the operands' low bits), the block reduces in LDS, and one
// block sums the per-block partials in a fixed order.

template <int NOUT>
__global__ __launch_bounds__(256) void k_splitk_part(const float2* __restrict__ A, const float2* __restrict__ B,
                                                    float2* __restrict__ part, const IndexOp op) {
  __shared__ uint64_t am[NOUT], bn[NOUT];
  __shared__ float red[2][256];
  const int nout = 1 << (op.nM + op.nN);
  const uint64_t nmask = (1ull << op.nN) - 1ull;
  const int tid = threadIdx.x;
  if (tid < nout) {
    am[tid] = dep((uint64_t)tid >> op.nN, op.aM);
    bn[tid] = dep((uint64_t)tid & nmask, op.bN);
  }
  __syncthreads();
  float acc_r[NOUT], acc_i[NOUT];
#pragma unroll
  for (int o = 0; o < NOUT; ++o) acc_r[o] = acc_i[o] = 0.f;
  const int64_t nK = (int64_t)1 << op.nK;
  for (int64_t k = (int64_t)blockIdx.x * 256 + tid; k < nK; k += (int64_t)gridDim.x * 256) {
    const uint64_t ak = dep((uint64_t)k, op.aK), bk = dep((uint64_t)k, op.bK);
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
      if (o < nout) {
        const float2 x = A[am[o] | ak];
        const float2 y = B[bn[o] | bk];
        acc_r[o] = fmaf(x.x, y.x, acc_r[o]);
        acc_r[o] = fmaf(-x.y, y.y, acc_r[o]);
        acc_i[o] = fmaf(x.x, y.y, acc_i[o]);
        acc_i[o] = fmaf(x.y, y.x, acc_i[o]);
      }
    }
  }
#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    if (o < nout) {  // uniform across the block
      red[0][tid] = acc_r[o];
      red[1][tid] = acc_i[o];
      __syncthreads();
      for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
          red[0][tid] += red[0][tid + w];
          red[1][tid] += red[1][tid + w];
        }
        __syncthreads();
      }
      if (tid == 0) part[(int64_t)blockIdx.x * nout + o] = make_float2(red[0][0], red[1][0]);
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(256) void k_splitk_final(const float2* __restrict__ part, int nblk, int nout,
                                                     float2* __restrict__ C) {
  __shared__ float red[2][256];
  const int tid = threadIdx.x;
  for (int o = 0; o < nout; ++o) {
    float r = 0.f, i = 0.f;
    for (int g = tid; g < nblk; g += 256) {
      const float2 v = part[(int64_t)g * nout + o];
      r += v.x;
      i += v.y;
    }
    red[0][tid] = r;
    red[1][tid] = i;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) {
        red[0][tid] += red[0][tid + w];
        red[1][tid] += red[1][tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) C[o] = make_float2(red[0][0], red[1][0]);
    __syncthreads();
  }
}

int64_t splitk_blocks(const IndexOp& op) { return splitk_grid(op.nK); }

hipError_t launch_splitk_c64(const float2* A, const float2* B, float2* C, float2* part, const IndexOp& op,
                             hipStream_t s) {
  const int nout = 1 << (op.nM + op.nN);
  if (nout > 64) return hipErrorInvalidValue;
  const int64_t g = splitk_blocks(op);
  if (nout <= 4)
    hipLaunchKernelGGL(k_splitk_part<4>, dim3((unsigned)g), dim3(256), 0, s, A, B, part, op);
  else if (nout <= 16)
    hipLaunchKernelGGL(k_splitk_part<16>, dim3((unsigned)g), dim3(256), 0, s, A, B, part, op);
  else
    hipLaunchKernelGGL(k_splitk_part<64>, dim3((unsigned)g), dim3(256), 0, s, A, B, part, op);
  hipLaunchKernelGGL(k_splitk_final, dim3(1), dim3(256), 0, s, part, (int)g, nout, C);
  return hipGetLastError();
}

// ------------------------------------------------------------ accumulate --
// amp[y] += (double) root[dep(y)] for the current slice; raises the
// non-finite flag; advances the slice cursor.

__global__ __launch_bounds__(256) void k_accum(const float2* __restrict__ root, const Runs y2root, int n_open,
                                              Ctrl* ctrl) {
  double* amp = ctrl->amp;
  const int64_t n = (int64_t)1 << n_open;
  bool bad = false;
  for (int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; y < n; y += (int64_t)gridDim.x * blockDim.x) {
    const float2 v = root[dep((uint64_t)y, y2root)];
    bad |= !(isfinite(v.x) && isfinite(v.y));
    amp[2 * y] += (double)v.x;
    amp[2 * y + 1] += (double)v.y;
  }
  if (bad) atomicOr(&ctrl->flags, (unsigned)TN_FLAG_NONFINITE);
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->cursor += 1;
}

hipError_t launch_accum(const float2* root, const AccumDesc& d, Ctrl* ctrl, hipStream_t s) {
  const int64_t n = (int64_t)1 << d.n_open;
  int64_t grid = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_accum, dim3((unsigned)grid), dim3(256), 0, s, root, d.y2root, d.n_open, ctrl);
  return hipGetLastError();
}

// ------------------------------------------------------------- reductions --
// Deterministic two-pass FP64 sums: fixed grid of per-block partials, then
// one block sums the partials in a fixed order.

constexpr int kRedBlocks = 1024;

__device__ double block_sum(double v) {
  __shared__ double sh[256];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_norm2_part(const double* __restrict__ amp, int64_t n, double* part) {
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double re = amp[2 * i], im = amp[2 * i + 1];
    s += re * re + im * im;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_xeb_part(const double* __restrict__ amp, int64_t n,
                                                 const int64_t* __restrict__ idx, int64_t n_idx, double* part) {
  double s1 = 0, s2 = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_idx;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = idx[i];
    if (j < 0 || j >= n) continue;
    const double re = amp[2 * j], im = amp[2 * j + 1];
    const double p = re * re + im * im;
    s1 += p;
    s2 += p * p;
  }
  s1 = block_sum(s1);
  s2 = block_sum(s2);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1;
    part[2 * blockIdx.x + 1] = s2;
  }
}

__global__ __launch_bounds__(256) void k_final_sum(const double* __restrict__ part, int nblk, int width,
                                                  double* out) {
  for (int w = 0; w < width; ++w) {
    double s = 0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += part[i * width + w];
    s = block_sum(s);
    if (threadIdx.x == 0) out[w] = s;
  }
}

hipError_t launch_norm2(const double* amp, int64_t n, double* out, hipStream_t s) {
  double* part = nullptr;
  hipError_t e = hipMallocAsync((void**)&part, kRedBlocks * sizeof(double), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_norm2_part, dim3(kRedBlocks), dim3(256), 0, s, amp, n, part);
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, s, part, kRedBlocks, 1, out);
  e = hipGetLastError();
  hipError_t e2 = hipFreeAsync(part, s);
  return e != hipSuccess ? e : e2;
}

hipError_t launch_xeb(const double* amp, int64_t n, const int64_t* idx, int64_t n_idx, double* out, hipStream_t s) {
  double* part = nullptr;
  hipError_t e = hipMallocAsync((void**)&part, 2 * kRedBlocks * sizeof(double), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_xeb_part, dim3(kRedBlocks), dim3(256), 0, s, amp, n, idx, n_idx, part);
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, s, part, kRedBlocks, 2, out);
  e = hipGetLastError();
  hipError_t e2 = hipFreeAsync(part, s);
  return e != hipSuccess ? e : e2;
}

__global__ __launch_bounds__(256) void k_hist(const double* __restrict__ amp, int64_t n, double scale, double xmax,
                                             int n_bins, unsigned long long* counts) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double re = amp[2 * i], im = amp[2 * i + 1];
    const double x = scale * (re * re + im * im);
    int b = x >= xmax ? n_bins - 1 : (int)(x / xmax * n_bins);
    if (b < 0) b = 0;
    if (b >= n_bins) b = n_bins - 1;
    atomicAdd(&counts[b], 1ull);
  }
}

hipError_t launch_hist(const double* amp, int64_t n, double scale, double xmax, int n_bins,
                       unsigned long long* counts, hipStream_t s) {
  int64_t grid = std::min<int64_t>((n + 255) / 256, 4096);
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hist, dim3((unsigned)grid), dim3(256), 0, s, amp, n, scale, xmax, n_bins, counts);
  return hipGetLastError();
}

}  // namespace tnrcs
