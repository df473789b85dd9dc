// Skewed contraction on FP32 matrix cores: many rows against a narrow
// operand (Supplement, CPU-architecture section, Fig. S7: the large operand
// is streamed once, the small one stays in fast local memory, the result is
// written once).
//
// C[(m << nN) | n] = sum_k A[dep(m, aM) | dep(k, aK)] * B[dep(n, bN) | dep(k, bK)]
// for N = 2^nN <= 64 outputs per row and any K = 2^nK >= 2, M = 2^nM >= 128
// rows.  The operands are read in their stored layouts through bit-deposit
// maps, so no permute runs before or after.  A workgroup of four waves takes
// 128 consecutive rows per pass (32 per wave); the pass's A rows are gathered
// chunk by chunk (16 k at a time) into LDS as planar FP32 re / im planes and
// multiplied on v_mfma_f32_32x32x2_f32 against B, which is kept in LDS for
// the whole kernel when it fits (else staged chunk by chunk with A).  Each
// wave's 32 x 32 output tiles (one or two for N <= 32 / 64; columns n >= N
// multiply zero rows of B and are not stored) go straight from the
// accumulators to C, whose rows of a pass are one contiguous range.  3M
// form on the matrix cores: T1 = ArBr, T2 = AiBi, T3 = (Ar+Ai)(Br+Bi).  Scaled
// half storage is widened to FP32 when staged and rounded once on store.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "elem.h"
#include "kernels.h"

namespace tnrcs {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kSkewPM = 128;  // rows per pass
constexpr int kSkewKC = 16;   // K staged per chunk
constexpr int kSkewLDA = kSkewPM + 4;

// LDS of one workgroup (bytes): A chunk planes, B planes (resident: all of
// K; else one chunk), A's and B's K offset tables, the pass's row offsets.
static size_t skew_lds(int nK, int np, bool bres) {
  const size_t K = (size_t)1 << nK;
  const size_t kb = bres ? K : (size_t)std::min<int64_t>(K, kSkewKC);
  return 2 * kSkewKC * kSkewLDA * 4 + 2 * kb * (np + 4) * 4 + 2 * K * 8 + kSkewPM * 8 + 64 * 8;
}

// MFAST: consecutive threads gather consecutive rows m (A's lowest bits are
// M bits); otherwise consecutive k (A's lowest bits are K bits).
template <int NT, bool MFAST, typename E>
__global__ __launch_bounds__(256, 2) void k_skew(const E* __restrict__ A, const E* __restrict__ B, E* __restrict__ C,
                                             const IndexOp op, float* maxslot, int bres) {
  constexpr int NP = 32 * NT, LDB = NP + 4;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int K = 1 << op.nK, N = 1 << op.nN;
  const int KC = K < kSkewKC ? K : kSkewKC;
  const int KB = bres ? K : KC;  // B rows held in LDS
  float* As = reinterpret_cast<float*>(smem);            // [2][KC][LDA]
  float* Bs = As + 2 * kSkewKC * kSkewLDA;               // [2][KB][LDB]
  uint64_t* kA = reinterpret_cast<uint64_t*>(Bs + 2 * KB * LDB);  // [K]
  uint64_t* kB = kA + K;                                 // [K]
  uint64_t* am = kB + K;                                 // [PM]
  uint64_t* bn = am + kSkewPM;                           // [64]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 31, kh = lane >> 5;
  for (int k = tid; k < K; k += 256) {
    kA[k] = dep((uint64_t)k, op.aK);
    kB[k] = dep((uint64_t)k, op.bK);
  }
  if (tid < 64) bn[tid] = tid < N ? dep((uint64_t)tid, op.bN) : 0;
  __syncthreads();
  // B rows [k0, k0 + kn) into LDS rows [0, kn): Bs[p][k][n], zero for n >= N
  auto stage_b = [&](int k0, int kn) {
    for (int i = tid; i < kn * NP; i += 256) {
      const int n = i % NP, k = i / NP;
      const float2 v = n < N ? to_f2(B[bn[n] | kB[k0 + k]]) : make_float2(0.f, 0.f);
      Bs[k * LDB + n] = v.x;
      Bs[(KB + k) * LDB + n] = v.y;
    }
  };
  if (bres) stage_b(0, K);
  const int64_t passes = ((int64_t)1 << op.nM) / kSkewPM;
  float mx = 0.f;
  for (int64_t ps = blockIdx.x; ps < passes; ps += gridDim.x) {
    const int64_t m0 = ps * kSkewPM;
    if (tid < kSkewPM) am[tid] = dep((uint64_t)(m0 + tid), op.aM);
    floatx16 acc[3][NT];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[p][j] = floatx16{};
    for (int k0 = 0; k0 < K; k0 += KC) {
      __syncthreads();  // previous chunk consumed; am[] visible
      // gather the chunk: PM x KC entries (KC even, so a multiple of 256),
      // all of a thread's loads issued before its LDS stores
      constexpr int EPT = kSkewPM * kSkewKC / 256;
      const int n_el = kSkewPM * KC;
      E v[EPT];
      int mi[EPT], ki[EPT];
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int i = tid + q * 256;
        if (MFAST) {
          mi[q] = i % kSkewPM;
          ki[q] = i / kSkewPM;
        } else {
          ki[q] = i % KC;
          mi[q] = i / KC;
        }
        if (i < n_el) v[q] = A[am[mi[q]] | kA[k0 + ki[q]]];
      }
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        if (tid + q * 256 < n_el) {
          const float2 x = to_f2(v[q]);
          As[ki[q] * kSkewLDA + mi[q]] = x.x;
          As[(kSkewKC + ki[q]) * kSkewLDA + mi[q]] = x.y;
        }
      }
      if (!bres) stage_b(k0, KC);
      __syncthreads();
      const int kb0 = bres ? k0 : 0;
      for (int kk = 0; kk < KC; kk += 2) {
        const int kr = kk + kh;
        const float ar = As[kr * kSkewLDA + wave * 32 + c];
        const float ai = As[(kSkewKC + kr) * kSkewLDA + wave * 32 + c];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const float br = Bs[(kb0 + kr) * LDB + 32 * j + c];
          const float bi = Bs[(KB + kb0 + kr) * LDB + 32 * j + c];
          acc[0][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, acc[0][j], 0, 0, 0);
          acc[1][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, bi, acc[1][j], 0, 0, 0);
          acc[2][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar + ai, br + bi, acc[2][j], 0, 0, 0);
        }
      }
    }
    // C rows m0 .. m0 + 127 are contiguous: row r of this wave's tile j,
    // column c -> C[(m0 + 32 wave + row) * N + 32 j + c]
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int col = 32 * j + c;
      if (col < N) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = wave * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
          const float cr = acc[0][j][r] - acc[1][j][r];
          const float ci = acc[2][j][r] - acc[0][j][r] - acc[1][j][r];
          mx = mag_max(mx, cr, ci);
          C[((m0 + row) << op.nN) | col] = from_f2<E>(cr * op.out_scale, ci * op.out_scale);
        }
      }
    }
  }
  record_max_in(maxslot, mx, reinterpret_cast<float*>(am));
}

bool skew_ok(const IndexOp& op) { return op.nN <= 6 && op.nK >= 1 && op.nK <= 10 && op.nM >= 7; }

template <int NT, typename E>
static hipError_t launch_skew_t(const E* A, const E* B, E* C, const IndexOp& op, float* maxslot, hipStream_t s) {
  const bool mfast = op.aM.n >= 1 && op.aM.src[0] == 0 && op.aM.dst[0] == 0;
  const int np = 32 * NT;
  const bool bres = skew_lds(op.nK, np, true) <= 64 * 1024;
  const size_t lds = skew_lds(op.nK, np, bres);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  const int64_t passes = ((int64_t)1 << op.nM) / kSkewPM;
  const dim3 g((unsigned)std::min<int64_t>(passes, 2048));
  if (mfast)
    hipLaunchKernelGGL((k_skew<NT, true, E>), g, dim3(256), lds, s, A, B, C, op, maxslot, bres ? 1 : 0);
  else
    hipLaunchKernelGGL((k_skew<NT, false, E>), g, dim3(256), lds, s, A, B, C, op, maxslot, bres ? 1 : 0);
  return hipGetLastError();
}

template <typename E>
static hipError_t launch_skew_e(const E* A, const E* B, E* C, const IndexOp& op, float* maxslot, hipStream_t s) {
  if (op.nN <= 5) return launch_skew_t<1, E>(A, B, C, op, maxslot, s);
  return launch_skew_t<2, E>(A, B, C, op, maxslot, s);
}

hipError_t launch_skew(int dtype, const void* A, const void* B, void* C, const IndexOp& op, float* maxslot,
                       hipStream_t s) {
  if (!skew_ok(op)) return hipErrorInvalidValue;
  if (dtype == TN_DTYPE_F16S) return launch_skew_e<cf16>((const cf16*)A, (const cf16*)B, (cf16*)C, op, maxslot, s);
  if (dtype == TN_DTYPE_BF16S)
    return launch_skew_e<cbf16>((const cbf16*)A, (const cbf16*)B, (cbf16*)C, op, maxslot, s);
  return launch_skew_e<float2>((const float2*)A, (const float2*)B, (float2*)C, op, maxslot, s);
}

}  // namespace tnrcs
