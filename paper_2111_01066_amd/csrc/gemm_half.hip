// Complex GEMM on FP16 / BF16 matrix cores with FP32 accumulation, for the
// scaled half-precision storage (the matrix product of Supplement Eq. (matmul)
// in the mixed-precision mode the main text names).
//
// C[m][n] = sum_k A[m][k] B[n][k]: A, B, C are (re, im) pairs of FP16 or BF16
// holding value * 2^-e.  The FP32 accumulator holds A_st * B_st; the epilogue
// multiplies by the op's output scale 2^-s before rounding to the storage
// format, so C's exponent is e_A + e_B + s.  v_mfma_f32_32x32x16_{f16,bf16};
// 128x128 workgroup tile, four waves of 64x64 (2x2 blocks of 32x32), K staged
// through LDS as planar re / im (and, for 3M, re+im formed in FP32 and rounded
// once) rows of BK halves; the next K tile is prefetched into registers while
// the current one is multiplied.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "elem.h"
#include "gather.h"
#include "kernels.h"

namespace tnrcs {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename H>
struct Frag;
template <>
struct Frag<_Float16> {
  typedef half8 T;
  static __device__ __forceinline__ floatx16 mfma(T a, T b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Frag<__bf16> {
  typedef bf16x8 T;
  static __device__ __forceinline__ floatx16 mfma(T a, T b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

template <typename H>
__device__ __forceinline__ uint16_t hbits(float x) {
  H h = (H)x;
  return __builtin_bit_cast(uint16_t, h);
}
template <typename H>
__device__ __forceinline__ float hval(uint32_t bits16) {
  return (float)__builtin_bit_cast(H, (uint16_t)bits16);
}

// Stores one K stage (registers -> LDS buffer), deinterleaving (re, im)
// words into planar rows: two complex words give one 32-bit pair of re halves
// and one of im halves (v_perm_b32 byte selects).
template <int P, int BM, int LDK, int NV, typename H>
__device__ __forceinline__ void store_stage(H (*S)[BM][LDK], const uint4* r, int row, int k0) {
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const uint32_t w[4] = {r[j].x, r[j].y, r[j].z, r[j].w};
    const uint32_t re01 = __builtin_amdgcn_perm(w[1], w[0], 0x05040100u);
    const uint32_t re23 = __builtin_amdgcn_perm(w[3], w[2], 0x05040100u);
    const uint32_t im01 = __builtin_amdgcn_perm(w[1], w[0], 0x07060302u);
    const uint32_t im23 = __builtin_amdgcn_perm(w[3], w[2], 0x07060302u);
    *reinterpret_cast<uint2*>(&S[0][row][k0 + 4 * j]) = make_uint2(re01, re23);
    *reinterpret_cast<uint2*>(&S[1][row][k0 + 4 * j]) = make_uint2(im01, im23);
    if (P == 3) {
      uint32_t sm[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) sm[q] = hbits<H>(hval<H>(w[q] & 0xFFFFu) + hval<H>(w[q] >> 16));
      *reinterpret_cast<uint2*>(&S[P - 1][row][k0 + 4 * j]) = make_uint2(sm[0] | (sm[1] << 16), sm[2] | (sm[3] << 16));
    }
  }
}

template <int FORM, int BK, int WTM, int WTN, int OCC, typename H, typename E>
__global__ __launch_bounds__(256, OCC) void k_hgemm(const E* __restrict__ A, const E* __restrict__ B,
                                                 void* __restrict__ Cout, int64_t N, int64_t K, int64_t k_len,
                                                 int64_t sA, int64_t sB, int64_t sC, float out_scale,
                                                 float* maxslot, int to_work, int64_t Mt, int64_t Nt) {
  typedef typename Frag<H>::T F;
  constexpr int P = (FORM == TN_GEMM_3M) ? 3 : 2;
  constexpr int BM = 64 * WTM, BN = 64 * WTN, LDK = BK + 8;
  constexpr int TPRA = 256 / BM, TPRB = 256 / BN;  // threads per operand row
  constexpr int NVA = BK / TPRA / 4;  // uint4 (4 complex) loads per thread per stage, A
  constexpr int NVB = BK / TPRB / 4;  // same for B
  // two LDS buffers: the MFMAs read one stage while the next is stored
  __shared__ __attribute__((aligned(16))) H As[2][P][BM][LDK];
  __shared__ __attribute__((aligned(16))) H Bs[2][P][BN][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t tm, tn, z;
  xcd_tile(blockIdx.x, Mt, Nt, gridDim.x, tm, tn, z);
  const int64_t bm = tm * BM, bn = tn * BN;
  A += z * sA;
  B += z * sB;
  const int wm = (wave & 1) * 32 * WTM, wn = (wave >> 1) * 32 * WTN;
  floatx16 acc[P][WTM][WTN];
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int j = 0; j < WTN; ++j) acc[p][i][j] = floatx16{};
  const int arow = tid / TPRA, ak = (tid % TPRA) * (BK / TPRA);
  const int brow = tid / TPRB, bk = (tid % TPRB) * (BK / TPRB);
  const uint4* Ap = reinterpret_cast<const uint4*>(A + (bm + arow) * K + ak);
  const uint4* Bp = reinterpret_cast<const uint4*>(B + (bn + brow) * K + bk);
  uint4 ra[NVA], rb[NVB];
#pragma unroll
  for (int j = 0; j < NVA; ++j) ra[j] = Ap[j];
#pragma unroll
  for (int j = 0; j < NVB; ++j) rb[j] = Bp[j];
  store_stage<P, BM, LDK, NVA, H>(As[0], ra, arow, ak);
  store_stage<P, BN, LDK, NVB, H>(Bs[0], rb, brow, bk);
  if (BK < k_len) {
#pragma unroll
    for (int j = 0; j < NVA; ++j) ra[j] = Ap[BK / 4 + j];
#pragma unroll
    for (int j = 0; j < NVB; ++j) rb[j] = Bp[BK / 4 + j];
  }
  __syncthreads();
  const int c = lane & 31, kq = (lane >> 5) * 8;
  int cur = 0;
  for (int64_t k0 = 0; k0 < k_len; k0 += BK) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      F a[P][WTM], b[P][WTN];
#pragma unroll
      for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int i = 0; i < WTM; ++i) a[p][i] = *reinterpret_cast<const F*>(&As[cur][p][wm + 32 * i + c][kk + kq]);
#pragma unroll
        for (int j = 0; j < WTN; ++j) b[p][j] = *reinterpret_cast<const F*>(&Bs[cur][p][wn + 32 * j + c][kk + kq]);
      }
      if (FORM == TN_GEMM_3M) {
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
          for (int j = 0; j < WTN; ++j) {
            acc[0][i][j] = Frag<H>::mfma(a[0][i], b[0][j], acc[0][i][j]);
            acc[1][i][j] = Frag<H>::mfma(a[1][i], b[1][j], acc[1][i][j]);
            acc[P - 1][i][j] = Frag<H>::mfma(a[P - 1][i], b[P - 1][j], acc[P - 1][i][j]);
          }
      } else {
        // two passes over the (i, j) blocks, so that the two products
        // accumulated into one register block are 2*WTM*WTN MFMAs apart
#pragma unroll
        for (int i = 0; i < WTM; ++i)
#pragma unroll
          for (int j = 0; j < WTN; ++j) {
            acc[0][i][j] = Frag<H>::mfma(a[0][i], b[0][j], acc[0][i][j]);
            acc[1][i][j] = Frag<H>::mfma(a[0][i], b[1][j], acc[1][i][j]);
          }
#pragma unroll
        for (int i = 0; i < WTM; ++i) {
          uint4 t = __builtin_bit_cast(uint4, a[1][i]);
          t.x ^= 0x80008000u;
          t.y ^= 0x80008000u;
          t.z ^= 0x80008000u;
          t.w ^= 0x80008000u;
          const F na = __builtin_bit_cast(F, t);
#pragma unroll
          for (int j = 0; j < WTN; ++j) {
            acc[0][i][j] = Frag<H>::mfma(na, b[1][j], acc[0][i][j]);
            acc[1][i][j] = Frag<H>::mfma(a[1][i], b[0][j], acc[1][i][j]);
          }
        }
      }
    }
    if (k0 + BK < k_len) {
      store_stage<P, BM, LDK, NVA, H>(As[cur ^ 1], ra, arow, ak);
      store_stage<P, BN, LDK, NVB, H>(Bs[cur ^ 1], rb, brow, bk);
      if (k0 + 2 * BK < k_len) {
        const int64_t adv = (k0 + 2 * BK) / 4;  // uint4 = 4 complex elements
#pragma unroll
        for (int j = 0; j < NVA; ++j) ra[j] = Ap[adv + j];
#pragma unroll
        for (int j = 0; j < NVB; ++j) rb[j] = Bp[adv + j];
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  float mx = 0.f;
  const int kh = lane >> 5;
  auto result = [&](int i, int j, int r, float& re, float& im) {
    if (FORM == TN_GEMM_3M) {
      re = acc[0][i][j][r] - acc[1][i][j][r];
      im = acc[P - 1][i][j][r] - acc[0][i][j][r] - acc[1][i][j][r];
    } else {
      re = acc[0][i][j][r];
      im = acc[1][i][j][r];
    }
  };
  if (to_work) {
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int j = 0; j < WTN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = wm + 32 * i + 8 * (r >> 2) + 4 * kh + (r & 3);
          const int col = wn + 32 * j + c;
          float re, im;
          result(i, j, r, re, im);
          reinterpret_cast<float2*>(Cout)[z * sC + (bm + row) * N + bn + col] = make_float2(re, im);
          if ((r & 15) == 15) __builtin_amdgcn_sched_barrier(0);
        }
  } else {
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int j = 0; j < WTN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = wm + 32 * i + 8 * (r >> 2) + 4 * kh + (r & 3);
          const int col = wn + 32 * j + c;
          float re, im;
          result(i, j, r, re, im);
          mx = mag_max(mx, re, im);
          reinterpret_cast<E*>(Cout)[z * sC + (bm + row) * N + bn + col] = from_f2<E>(re * out_scale, im * out_scale);
          // keep the accumulator reads of one 32x32 block together (hoisting
          // them all at once exhausts the registers of the widest tiles)
          if ((r & 15) == 15) __builtin_amdgcn_sched_barrier(0);
        }
  }
  // the block reduction reuses the (now idle) stage buffers: no LDS beyond
  // the two stages, so two workgroups fit in one CU's LDS
  if (!to_work) record_max_in(maxslot, mx, reinterpret_cast<float*>(&As[0][0][0][0]));
}

// Ping-pong schedule (4M form): eight waves, two per SIMD, in two groups of
// four.  In each K stage one group runs its MFMAs on the stage in LDS while
// the other stores its share of the next stage (loaded into registers one
// stage earlier) into the other LDS buffer and issues the global loads of
// the stage after; a barrier hands the roles over, and a second one ends the
// stage.  The MFMA pipe of a SIMD is fed by one wave at a time, without the
// stage stores and barriers of a single-wave loop between its MFMAs.
// 256x128 workgroup tile, 64x64 per wave; needs M % 256 == N % 128 ==
// k_len % 32 == 0.
template <typename H, typename E>
__global__ __launch_bounds__(512, 1) void k_hgemm_pp(const E* __restrict__ A, const E* __restrict__ B,
                                                   void* __restrict__ Cout, int64_t N, int64_t K, int64_t k_len,
                                                   int64_t sA, int64_t sB, int64_t sC, float out_scale,
                                                   float* maxslot, int to_work, int64_t Mt, int64_t Nt) {
  typedef typename Frag<H>::T F;
  constexpr int BK = 32, BM = 256, BN = 128, LDK = BK + 8, P = 2;
  __shared__ __attribute__((aligned(16))) H As[2][P][BM][LDK];
  __shared__ __attribute__((aligned(16))) H Bs[2][P][BN][LDK];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int grp = wave >> 2;  // group 0 computes first in every stage
  const int gt = tid & 255;   // thread index within the group
  int64_t tm, tn, z;
  xcd_tile(blockIdx.x, Mt, Nt, gridDim.x, tm, tn, z);
  const int64_t bm = tm * BM, bn = tn * BN;
  A += z * sA;
  B += z * sB;
  const int wm = (wave & 3) * 64, wn = grp * 64;
  floatx16 acc[2][2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[p][i][j] = floatx16{};
  // this thread's share of every stage: 16 complex of A row grp*128 + gt/2
  // and 8 complex of B row grp*64 + gt/4
  const int arow = grp * 128 + (gt >> 1), ak = (gt & 1) * 16;
  const int brow = grp * 64 + (gt >> 2), bk = (gt & 3) * 8;
  const uint4* Ap = reinterpret_cast<const uint4*>(A + (bm + arow) * K + ak);
  const uint4* Bp = reinterpret_cast<const uint4*>(B + (bn + brow) * K + bk);
  uint4 ra[4], rb[2];
  const int64_t nst = k_len / BK;
  auto load = [&](int64_t st) {
    const int64_t o = st * (BK / 4);
#pragma unroll
    for (int j = 0; j < 4; ++j) ra[j] = Ap[o + j];
#pragma unroll
    for (int j = 0; j < 2; ++j) rb[j] = Bp[o + j];
  };
  auto store = [&](int buf) {
    store_stage<P, BM, LDK, 4, H>(As[buf], ra, arow, ak);
    store_stage<P, BN, LDK, 2, H>(Bs[buf], rb, brow, bk);
  };
  const int c = lane & 31, kq = (lane >> 5) * 8;
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      F a[P][2], b[P][2];
#pragma unroll
      for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int i = 0; i < 2; ++i) a[p][i] = *reinterpret_cast<const F*>(&As[buf][p][wm + 32 * i + c][kk + kq]);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[p][j] = *reinterpret_cast<const F*>(&Bs[buf][p][wn + 32 * j + c][kk + kq]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[0][i][j] = Frag<H>::mfma(a[0][i], b[0][j], acc[0][i][j]);
          acc[1][i][j] = Frag<H>::mfma(a[0][i], b[1][j], acc[1][i][j]);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        uint4 t = __builtin_bit_cast(uint4, a[1][i]);
        t.x ^= 0x80008000u;
        t.y ^= 0x80008000u;
        t.z ^= 0x80008000u;
        t.w ^= 0x80008000u;
        const F na = __builtin_bit_cast(F, t);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[0][i][j] = Frag<H>::mfma(na, b[1][j], acc[0][i][j]);
          acc[1][i][j] = Frag<H>::mfma(a[1][i], b[0][j], acc[1][i][j]);
        }
      }
    }
  };
  load(0);
  store(0);
  load(nst > 1 ? 1 : 0);
  __syncthreads();
  // one loop per group (the same barriers in the same order), so that the
  // registers a group's loads land in stay put across its MFMAs.  nx: the
  // stage after next, clamped: past the end the last stage is re-read and
  // its copy goes to the buffer nobody reads any more.
  // (the compiler may still move MFMAs, which touch registers only, across
  // a barrier into the neighbouring phase; fencing them in measured slower)
  auto handover = [&]() { __syncthreads(); };
  if (grp == 0) {
    for (int64_t st = 0; st < nst; ++st) {
      const int cur = (int)(st & 1);
      compute(cur);
      handover();
      store(cur ^ 1);
      load(st + 2 < nst ? st + 2 : nst - 1);
      handover();
    }
  } else {
    for (int64_t st = 0; st < nst; ++st) {
      const int cur = (int)(st & 1);
      store(cur ^ 1);
      load(st + 2 < nst ? st + 2 : nst - 1);
      handover();
      compute(cur);
      handover();
    }
  }
  float mx = 0.f;
  const int kh = lane >> 5;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wm + 32 * i + 8 * (r >> 2) + 4 * kh + (r & 3);
        const int col = wn + 32 * j + c;
        const float re = acc[0][i][j][r], im = acc[1][i][j][r];
        const int64_t o = z * sC + (bm + row) * N + bn + col;
        if (to_work) {
          reinterpret_cast<float2*>(Cout)[o] = make_float2(re, im);
        } else {
          mx = mag_max(mx, re, im);
          reinterpret_cast<E*>(Cout)[o] = from_f2<E>(re * out_scale, im * out_scale);
        }
        if ((r & 15) == 15) __builtin_amdgcn_sched_barrier(0);
      }
  if (!to_work) record_max_in(maxslot, mx, reinterpret_cast<float*>(&As[0][0][0][0]));
}

// A read in place (4M, 128x128 tiles, stages of 32 k, two waves per SIMD):
// the stage's 128 x 32 A entries are gathered through the chunk map in A's
// address order, four consecutive addresses per 16-byte load.  Those four
// entries differ in A's two lowest index bits, which are the lowest row or
// k bits; MODE says which (0: k0 k1, four k of one row; 1: k0 then row 0;
// 2: row 0 then k0; 3: row 0 row 1, four rows at one k), and so how they are
// deinterleaved into the planar [row][k] LDS rows.  The stage's K offset
// moves by a carrying add restricted to A's K bits above 4 (in increasing
// positions).  B is [N][K] and C is [M][N], as in k_hgemm.
struct GatherAH {
  SkewMap mp;
  Runs aM;
  uint64_t maskK = 0, incK = 0;
};

template <int MODE, typename H, typename E>
__global__ __launch_bounds__(256, 2) void k_hgemm_ga(const E* __restrict__ A, const E* __restrict__ B,
                                                   E* __restrict__ C, int64_t N, int64_t K, float out_scale,
                                                   float* maxslot, int64_t Mt, int64_t Nt, const GatherAH g) {
  typedef typename Frag<H>::T F;
  constexpr int BK = 32, BM = 128, BN = 128, LDK = BK + 8, P = 2, WTM = 2, WTN = 2;
  constexpr int NVB = BK / (256 / BN) / 4;  // B: uint4 loads per thread per stage
  __shared__ __attribute__((aligned(16))) H As[2][P][BM][LDK];
  __shared__ __attribute__((aligned(16))) H Bs[2][P][BN][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t tm, tn, z;
  xcd_tile(blockIdx.x, Mt, Nt, gridDim.x, tm, tn, z);
  const int64_t bm = tm * BM, bn = tn * BN;
  const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
  floatx16 acc[P][WTM][WTN];
#pragma unroll
  for (int p = 0; p < P; ++p)
#pragma unroll
    for (int i = 0; i < WTM; ++i)
#pragma unroll
      for (int j = 0; j < WTN; ++j) acc[p][i][j] = floatx16{};
  // this thread's four loads of a stage: offset of the first entry from the
  // stage's first entry, and the LDS index (row * LDK + k) of that entry
  uint32_t eoff[4];
  int lidx[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint64_t off;
    int m, k;
    skew_split(g.mp, (j * 256 + tid) * 4, off, m, k);
    eoff[j] = (uint32_t)off;
    lidx[j] = m * LDK + k;
  }
  const uint64_t abase = dep_u<12>((uint64_t)bm, g.aM);
  uint64_t kofs = 0;
  const int brow = tid / 2, bk = (tid % 2) * 16;
  const uint4* Bp = reinterpret_cast<const uint4*>(B + (bn + brow) * K + bk);
  uint4 ra[4], rb[NVB];
  auto load_a = [&]() {
    const E* base = A + (abase + kofs);
#pragma unroll
    for (int j = 0; j < 4; ++j) ra[j] = *reinterpret_cast<const uint4*>(base + eoff[j]);
  };
  auto store_a = [&](H (*S)[BM][LDK]) {
    H* re = &S[0][0][0];
    H* im = &S[1][0][0];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t w[4] = {ra[j].x, ra[j].y, ra[j].z, ra[j].w};
      const int i0 = lidx[j];
      if constexpr (MODE == 0) {  // k, k+1, k+2, k+3 of one row
        *reinterpret_cast<uint2*>(re + i0) = make_uint2(__builtin_amdgcn_perm(w[1], w[0], 0x05040100u),
                                                        __builtin_amdgcn_perm(w[3], w[2], 0x05040100u));
        *reinterpret_cast<uint2*>(im + i0) = make_uint2(__builtin_amdgcn_perm(w[1], w[0], 0x07060302u),
                                                        __builtin_amdgcn_perm(w[3], w[2], 0x07060302u));
      } else if constexpr (MODE == 1) {  // (m, k), (m, k+1), (m+1, k), (m+1, k+1)
        *reinterpret_cast<uint32_t*>(re + i0) = __builtin_amdgcn_perm(w[1], w[0], 0x05040100u);
        *reinterpret_cast<uint32_t*>(im + i0) = __builtin_amdgcn_perm(w[1], w[0], 0x07060302u);
        *reinterpret_cast<uint32_t*>(re + i0 + LDK) = __builtin_amdgcn_perm(w[3], w[2], 0x05040100u);
        *reinterpret_cast<uint32_t*>(im + i0 + LDK) = __builtin_amdgcn_perm(w[3], w[2], 0x07060302u);
      } else if constexpr (MODE == 2) {  // (m, k), (m+1, k), (m, k+1), (m+1, k+1)
        *reinterpret_cast<uint32_t*>(re + i0) = __builtin_amdgcn_perm(w[2], w[0], 0x05040100u);
        *reinterpret_cast<uint32_t*>(im + i0) = __builtin_amdgcn_perm(w[2], w[0], 0x07060302u);
        *reinterpret_cast<uint32_t*>(re + i0 + LDK) = __builtin_amdgcn_perm(w[3], w[1], 0x05040100u);
        *reinterpret_cast<uint32_t*>(im + i0 + LDK) = __builtin_amdgcn_perm(w[3], w[1], 0x07060302u);
      } else {  // rows m .. m+3 at one k
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          re[i0 + q * LDK] = __builtin_bit_cast(H, (uint16_t)(w[q] & 0xFFFFu));
          im[i0 + q * LDK] = __builtin_bit_cast(H, (uint16_t)(w[q] >> 16));
        }
      }
    }
  };
  auto load_b = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < NVB; ++j) rb[j] = Bp[k0 / 4 + j];
  };
  load_a();
  load_b(0);
  store_a(As[0]);
  store_stage<P, BN, LDK, NVB, H>(Bs[0], rb, brow, bk);
  if (BK < K) {
    kofs = ((kofs | ~g.maskK) + g.incK) & g.maskK;
    load_a();
    load_b(BK);
  }
  __syncthreads();
  const int c = lane & 31, kq = (lane >> 5) * 8;
  int cur = 0;
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      F a[P][WTM], b[P][WTN];
#pragma unroll
      for (int p = 0; p < P; ++p) {
#pragma unroll
        for (int i = 0; i < WTM; ++i) a[p][i] = *reinterpret_cast<const F*>(&As[cur][p][wm + 32 * i + c][kk + kq]);
#pragma unroll
        for (int j = 0; j < WTN; ++j) b[p][j] = *reinterpret_cast<const F*>(&Bs[cur][p][wn + 32 * j + c][kk + kq]);
      }
#pragma unroll
      for (int i = 0; i < WTM; ++i)
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
          acc[0][i][j] = Frag<H>::mfma(a[0][i], b[0][j], acc[0][i][j]);
          acc[1][i][j] = Frag<H>::mfma(a[0][i], b[1][j], acc[1][i][j]);
        }
#pragma unroll
      for (int i = 0; i < WTM; ++i) {
        uint4 t = __builtin_bit_cast(uint4, a[1][i]);
        t.x ^= 0x80008000u;
        t.y ^= 0x80008000u;
        t.z ^= 0x80008000u;
        t.w ^= 0x80008000u;
        const F na = __builtin_bit_cast(F, t);
#pragma unroll
        for (int j = 0; j < WTN; ++j) {
          acc[0][i][j] = Frag<H>::mfma(na, b[1][j], acc[0][i][j]);
          acc[1][i][j] = Frag<H>::mfma(a[1][i], b[0][j], acc[1][i][j]);
        }
      }
    }
    if (k0 + BK < K) {
      store_a(As[cur ^ 1]);
      store_stage<P, BN, LDK, NVB, H>(Bs[cur ^ 1], rb, brow, bk);
      if (k0 + 2 * BK < K) {
        kofs = ((kofs | ~g.maskK) + g.incK) & g.maskK;
        load_a();
        load_b(k0 + 2 * BK);
      }
    }
    __syncthreads();
    cur ^= 1;
  }
  float mx = 0.f;
  const int kh = lane >> 5;
#pragma unroll
  for (int i = 0; i < WTM; ++i)
#pragma unroll
    for (int j = 0; j < WTN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wm + 32 * i + 8 * (r >> 2) + 4 * kh + (r & 3);
        const int col = wn + 32 * j + c;
        const float re = acc[0][i][j][r], im = acc[1][i][j][r];
        mx = mag_max(mx, re, im);
        C[(bm + row) * N + bn + col] = from_f2<E>(re * out_scale, im * out_scale);
        if ((r & 15) == 15) __builtin_amdgcn_sched_barrier(0);
      }
  record_max_in(maxslot, mx, reinterpret_cast<float*>(&As[0][0][0][0]));
}

static uint64_t dep_host_h(uint64_t x, const Runs& r) {
  uint64_t o = 0;
  for (int i = 0; i < r.n; ++i) o |= ((x >> r.src[i]) & ((1ull << r.len[i]) - 1ull)) << r.dst[i];
  return o;
}

template <int MODE, typename H, typename E>
static void hgemm_ga_launch(const E* A, const E* B, E* C, int64_t M, int64_t N, int64_t K, float scale,
                            float* maxslot, const GatherAH& g, hipStream_t s) {
  const int64_t Mt = M / 128, Nt = N / 128;
  hipLaunchKernelGGL((k_hgemm_ga<MODE, H, E>), dim3((unsigned)(Mt * Nt)), dim3(256), 0, s, A, B, C, N, K, scale,
                     maxslot, Mt, Nt, g);
}

template <typename H, typename E>
static hipError_t hgemm_ga_t(const E* A, const E* B, E* C, const IndexOp& idx, float scale, float* maxslot,
                             hipStream_t s) {
  const int64_t M = (int64_t)1 << idx.nM, N = (int64_t)1 << idx.nN, K = (int64_t)1 << idx.nK;
  GatherAH g{};
  if (!skew_map(idx, 5, 0, &g.mp) || g.mp.v != 12) return hipErrorInvalidValue;
  g.aM = idx.aM;
  g.maskK = dep_host_h((uint64_t)(K - 1) & ~(uint64_t)31, idx.aK);
  g.incK = K > 32 ? dep_host_h(32, idx.aK) : 0;
  // the two lowest chunk bits are A's positions 0 and 1
  if (g.mp.pos[0] != 0 || g.mp.pos[1] != 1) return hipErrorInvalidValue;
  const bool k0 = g.mp.kb[0] == 0, k1 = g.mp.kb[1] == 1, m0 = g.mp.mb[0] == 0, m1 = g.mp.mb[1] == 1;
  if (k0 && k1) hgemm_ga_launch<0, H, E>(A, B, C, M, N, K, scale, maxslot, g, s);
  else if (k0 && g.mp.mb[1] == 0) hgemm_ga_launch<1, H, E>(A, B, C, M, N, K, scale, maxslot, g, s);
  else if (m0 && g.mp.kb[1] == 0) hgemm_ga_launch<2, H, E>(A, B, C, M, N, K, scale, maxslot, g, s);
  else if (m0 && m1) hgemm_ga_launch<3, H, E>(A, B, C, M, N, K, scale, maxslot, g, s);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gemm_half_ga(int dtype, const void* A, const void* B, void* C, const IndexOp& idx, float out_scale,
                               float* maxslot, hipStream_t s) {
  if (!gemm_gather_ok(idx) || idx.nK < 5) return hipErrorInvalidValue;
  if (dtype == TN_DTYPE_F16S)
    return hgemm_ga_t<_Float16, cf16>((const cf16*)A, (const cf16*)B, (cf16*)C, idx, out_scale, maxslot, s);
  if (dtype == TN_DTYPE_BF16S)
    return hgemm_ga_t<__bf16, cbf16>((const cbf16*)A, (const cbf16*)B, (cbf16*)C, idx, out_scale, maxslot, s);
  return hipErrorInvalidValue;
}

// C[i] = (sum over slabs s, in order, of W[s][i]) * scale, rounded to E.
template <typename E>
__global__ __launch_bounds__(256) void k_hsplit_sum(const float2* __restrict__ W, E* __restrict__ C, int64_t n,
                                                   int slabs, float out_scale, float* maxslot) {
  float mx = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float r = 0.f, im = 0.f;
    for (int sl = 0; sl < slabs; ++sl) {
      const float2 v = W[(int64_t)sl * n + i];
      r += v.x;
      im += v.y;
    }
    mx = mag_max(mx, r, im);
    C[i] = from_f2<E>(r * out_scale, im * out_scale);
  }
  record_max(maxslot, mx);
}

bool hgemm_shape_ok(int64_t M, int64_t N, int64_t K) {
  return M > 0 && N > 0 && K > 0 && M % 64 == 0 && N % 64 == 0 && K % 16 == 0 && (M / 64) * (N / 64) < (1ll << 31);
}

template <int FORM, typename H, typename E>
static void hgemm_dispatch(int64_t M, int64_t z, hipStream_t s, const E* A, const E* B, void* C, int64_t N, int64_t K,
                           int64_t kl, int64_t sA, int64_t sB, int64_t sC, float scale, float* maxslot, int to_work,
                           int tile, int occ) {
  // short contractions are store-bound: 64x64 tiles keep more workgroups in
  // flight; otherwise 128x128 tiles with 32-deep K stages
  const bool small = tile == 64 || (tile == 0 && kl <= 64) || (M % 128) || (N % 128);
  if (small) {
    const int64_t Mt = M / 64, Nt = N / 64;
    const dim3 grid((unsigned)(Mt * Nt * z));
    if (kl % 32 == 0)
      hipLaunchKernelGGL((k_hgemm<FORM, 32, 1, 1, 2, H, E>), grid, dim3(256), 0, s, A, B, C, N, K, kl, sA, sB, sC,
                         scale, maxslot, to_work, Mt, Nt);
    else
      hipLaunchKernelGGL((k_hgemm<FORM, 16, 1, 1, 2, H, E>), grid, dim3(256), 0, s, A, B, C, N, K, kl, sA, sB, sC,
                         scale, maxslot, to_work, Mt, Nt);
    return;
  }
  if constexpr (FORM == TN_GEMM_4M) {
    if (occ == 3 && M % 256 == 0 && kl % 32 == 0) {
      const int64_t Mt = M / 256, Nt = N / 128;
      hipLaunchKernelGGL((k_hgemm_pp<H, E>), dim3((unsigned)(Mt * Nt * z)), dim3(512), 0, s, A, B, C, N, K, kl, sA,
                         sB, sC, scale, maxslot, to_work, Mt, Nt);
      return;
    }
  }
  // two waves per SIMD (registers capped at 256) hide latency on short K;
  // one wave per SIMD (no cap) pipelines long K better
  if (occ == 0 || occ == 3) occ = kl >= 16384 ? 1 : 2;
  const int64_t Mt = M / 128, Nt = N / 128;
  const dim3 grid((unsigned)(Mt * Nt * z));
  if (kl % 32 == 0) {
    if (occ == 1)
      hipLaunchKernelGGL((k_hgemm<FORM, 32, 2, 2, 1, H, E>), grid, dim3(256), 0, s, A, B, C, N, K, kl, sA, sB, sC,
                         scale, maxslot, to_work, Mt, Nt);
    else
      hipLaunchKernelGGL((k_hgemm<FORM, 32, 2, 2, 2, H, E>), grid, dim3(256), 0, s, A, B, C, N, K, kl, sA, sB, sC,
                         scale, maxslot, to_work, Mt, Nt);
  } else {
    hipLaunchKernelGGL((k_hgemm<FORM, 16, 2, 2, 2, H, E>), grid, dim3(256), 0, s, A, B, C, N, K, kl, sA, sB, sC, scale,
                       maxslot, to_work, Mt, Nt);
  }
}

template <typename H, typename E>
static hipError_t hgemm_t(const E* A, const E* B, E* C, int64_t M, int64_t N, int64_t K, int64_t batch, int form,
                          hipStream_t s, float2* work, int splits, float scale, float* maxslot, int tile, int occ) {
  if (splits > 1) {
    const int64_t kl = K / splits;
    if (form == TN_GEMM_3M)
      hgemm_dispatch<TN_GEMM_3M, H, E>(M, splits, s, A, B, work, N, K, kl, kl, kl, M * N, 1.f, nullptr, 1, tile, occ);
    else
      hgemm_dispatch<TN_GEMM_4M, H, E>(M, splits, s, A, B, work, N, K, kl, kl, kl, M * N, 1.f, nullptr, 1, tile, occ);
    const int64_t n = M * N;
    hipLaunchKernelGGL(k_hsplit_sum<E>, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0, s,
                       work, C, n, splits, scale, maxslot);
    return hipGetLastError();
  }
  if (form == TN_GEMM_3M)
    hgemm_dispatch<TN_GEMM_3M, H, E>(M, batch, s, A, B, C, N, K, K, M * K, N * K, M * N, scale, maxslot, 0, tile, occ);
  else
    hgemm_dispatch<TN_GEMM_4M, H, E>(M, batch, s, A, B, C, N, K, K, M * K, N * K, M * N, scale, maxslot, 0, tile, occ);
  return hipGetLastError();
}

hipError_t launch_gemm_half(int dtype, const void* A, const void* B, void* C, int64_t M, int64_t N, int64_t K,
                            int64_t batch, int form, hipStream_t s, float2* work, int splits, float out_scale,
                            float* maxslot, int tile, int occ) {
  if (!hgemm_shape_ok(M, N, K) || batch < 0) return hipErrorInvalidValue;
  if (tile == 128 && ((M % 128) || (N % 128))) return hipErrorInvalidValue;
  if (batch == 0) return hipSuccess;
  if (splits < 1) splits = 1;
  if (splits > 1 && (batch != 1 || !work || K % (16 * splits) != 0 || splits > 65535)) return hipErrorInvalidValue;
  if (batch > 65535) return hipErrorInvalidValue;
  if (dtype == TN_DTYPE_F16S)
    return hgemm_t<_Float16, cf16>((const cf16*)A, (const cf16*)B, (cf16*)C, M, N, K, batch, form, s, work, splits,
                                   out_scale, maxslot, tile, occ);
  if (dtype == TN_DTYPE_BF16S)
    return hgemm_t<__bf16, cbf16>((const cbf16*)A, (const cbf16*)B, (cbf16*)C, M, N, K, batch, form, s, work,
                                  splits, out_scale, maxslot, tile, occ);
  return hipErrorInvalidValue;
}

}  // namespace tnrcs
