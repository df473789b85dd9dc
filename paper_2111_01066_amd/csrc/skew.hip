// Skewed contraction on FP32 matrix cores: many rows against a narrow
// operand (Supplement, CPU-architecture section, Fig. S7: the large operand
// is streamed once, the small one stays in fast local memory, the result is
// written once).
//
// C[(m << nN) | n] = sum_k A[dep(m, aM) | dep(k, aK)] * B[dep(n, bN) | dep(k, bK)]
// for N = 2^nN <= 64 outputs per row and K = 2^nK >= 2, M = 2^nM >= 128 rows.
// The operands are read in their stored layouts, so no permute runs before
// or after.  A workgroup of four waves takes 128 consecutive rows per pass
// (32 per wave) and walks K in chunks of up to 16.  A chunk's 128 x 16 A
// entries sit at 2^11 addresses spanned by 11 bits of A's index; the
// workgroup reads them in address order (consecutive threads, consecutive
// addresses; 16-byte loads when A's lowest bits belong to the chunk), so a
// chunk is a few long contiguous runs whatever the interleaving of M and K
// bits in A's layout.  The chunk goes to LDS as planar FP32 re / im planes
// and is multiplied on v_mfma_f32_32x32x2_f32 against B, kept in LDS for the
// whole kernel when it fits (else staged per chunk); the next chunk's loads
// are issued before the current chunk's products, so loads and matrix work
// overlap.  Each wave's 32 x 32 output tiles (one or two for N <= 32 / 64;
// columns n >= N multiply zero rows of B and are not stored) go straight from
// the accumulators to C, whose rows of a pass are one contiguous range.  3M
// form: T1 = ArBr, T2 = AiBi, T3 = (Ar+Ai)(Br+Bi).  Scaled half storage is
// widened to FP32 when staged and rounded once on store.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "elem.h"
#include "gather.h"
#include "kernels.h"

namespace tnrcs {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef unsigned int skew_u32x4 __attribute__((ext_vector_type(4)));
// A is read once and C written once per launch, both far larger than the
// caches: nontemporal loads and stores (about 3 % faster on the 2^32-entry
// steps of the 53-qubit network)
template <typename E>
__device__ __forceinline__ E skew_ld_nt(const E* p) {
  E e;
  if constexpr (sizeof(E) == 8) {
    const unsigned long long w = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p));
    __builtin_memcpy(&e, &w, 8);
  } else {
    const unsigned w = __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p));
    __builtin_memcpy(&e, &w, 4);
  }
  return e;
}
template <typename E>
__device__ __forceinline__ void skew_st_nt(E* p, E e) {
  if constexpr (sizeof(E) == 8) {
    unsigned long long w;
    __builtin_memcpy(&w, &e, 8);
    __builtin_nontemporal_store(w, reinterpret_cast<unsigned long long*>(p));
  } else {
    unsigned w;
    __builtin_memcpy(&w, &e, 4);
    __builtin_nontemporal_store(w, reinterpret_cast<unsigned*>(p));
  }
}

constexpr int kSkewPM = 128;  // rows per pass
constexpr int kSkewKC = 16;   // K staged per chunk (fewer when K is smaller)
constexpr int kSkewLDA = 160;  // LDS k-row stride (floats): 128 rows + 32, so rows k and k+1 sit 32 banks apart

// LDS of one workgroup (bytes): A chunk planes, B planes (resident: all of
// K; else one chunk), B's K offset table, its N offsets, and A's offset of
// every chunk's first k.
static size_t skew_lds(int nK, int np, bool bres) {
  const size_t K = (size_t)1 << nK;
  const size_t kc = (size_t)std::min<int64_t>(K, kSkewKC);
  const size_t kb = bres ? K : kc;
  return 2 * kc * kSkewLDA * 4 + 2 * kb * (np + 4) * 4 + K * 8 + 64 * 8 + (K / kc) * 8;
}

// VEC consecutive chunk elements per load (VEC > 1: A's lowest log2(VEC)
// index bits are the chunk's lowest bits, one 16-byte load).  LPT loads per
// thread cover the 2^v chunk entries; DEPTH chunks are loaded ahead; KC k
// per chunk (16, or K when K < 16).
template <int NT, int VEC, int LPT, int DEPTH, int KC, typename E>
__global__ __launch_bounds__(256, 2) void k_skew(const E* __restrict__ A, const E* __restrict__ B, E* __restrict__ C,
                                                const IndexOp op, const SkewMap mp, float* maxslot, int bres) {
  constexpr int NP = 32 * NT, LDB = NP + 4;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int K = 1 << op.nK, N = 1 << op.nN;
  const int KB = bres ? K : KC;  // B rows held in LDS
  const int lnch = op.nK - __builtin_ctz(KC);  // log2 of the chunks per pass
  float* As = reinterpret_cast<float*>(smem);                      // [2][KC][LDA]
  float* Bs = As + 2 * KC * kSkewLDA;                              // [2][KB][LDB]
  uint64_t* kB = reinterpret_cast<uint64_t*>(Bs + 2 * KB * LDB);  // [K]
  uint64_t* bn = kB + K;                                           // [64]
  uint64_t* kA0 = bn + 64;                                         // [K / KC]: A offset of chunk ch's k0
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 31, kh = lane >> 5;
  for (int k = tid; k < K; k += 256) kB[k] = dep((uint64_t)k, op.bK);
  for (int ch = tid; ch < K / KC; ch += 256) kA0[ch] = dep((uint64_t)ch * KC, op.aK);
  if (tid < 64) bn[tid] = tid < N ? dep((uint64_t)tid, op.bN) : 0;
  // this thread's chunk entries: load j covers elements (j * 256 + tid) * VEC + u
  // (the launcher picks LPT * 256 * VEC = 2^v, so every thread has LPT full loads)
  uint64_t eoff[LPT];
  int eidx[LPT][VEC];  // LDS index of each entry
#pragma unroll
  for (int j = 0; j < LPT; ++j) {
#pragma unroll
    for (int u = 0; u < VEC; ++u) {
      const int e = (j * 256 + tid) * VEC + u;
      uint64_t off;
      int m, k;
      skew_split(mp, e, off, m, k);
      if (u == 0) eoff[j] = off;
      eidx[j][u] = k * kSkewLDA + (m ^ skew_h(mp, m, k));
    }
  }
  // this lane's matrix-core operand entries: row 32 wave + c, k = kk + kh
  int aidx[KC / 2];
#pragma unroll
  for (int s2 = 0; s2 < KC / 2; ++s2) {
    const int k = 2 * s2 + kh, m = wave * 32 + c;
    aidx[s2] = k * kSkewLDA + (m ^ skew_h(mp, m, k));
  }
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
  const int64_t my_passes = passes > (int64_t)blockIdx.x ? (passes - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
  const int64_t items = my_passes << lnch;
  // A offset of a chunk: dep(m0, aM) | dep(k0, aK).  Both parts are
  // advanced in the deposited domain instead of being recomputed (dep walks
  // the run lists, which costs memory reads): the row part moves by
  // dep(gridDim.x * PM) per pass through an add whose carries skip the bits
  // that are not row bits (they are set to 1 first), the k part is tabulated
  // per chunk.  One cursor for the chunk being prefetched.
  const uint64_t mask_m = dep(((uint64_t)1 << op.nM) - kSkewPM, op.aM);  // row bits 7.. of A
  const uint64_t inc_m = dep((uint64_t)gridDim.x * kSkewPM, op.aM);
  uint64_t pf_m = dep((uint64_t)blockIdx.x * kSkewPM, op.aM);
  int pf_ch = 0;
  // DEPTH chunks in flight: chunk it lives in register set it % DEPTH from
  // its loads until its LDS store, and set it % DEPTH is reloaded with chunk
  // it + DEPTH right after that store
  E v[DEPTH][LPT][VEC];
  auto load_next = [&](E (&dst)[LPT][VEC]) {
    const E* base = A + (pf_m | kA0[pf_ch]);
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
      if constexpr (VEC == 1) {
        dst[j][0] = skew_ld_nt(base + eoff[j]);
      } else {
        const skew_u32x4 w = __builtin_nontemporal_load(reinterpret_cast<const skew_u32x4*>(base + eoff[j]));
        __builtin_memcpy(&dst[j][0], &w, 16);
      }
    }
    if (++pf_ch == (1 << lnch)) {
      pf_ch = 0;
      pf_m = ((pf_m | ~mask_m) + inc_m) & mask_m;
    }
  };
  floatx16 acc[3][NT];
  float mx = 0.f;
#pragma unroll
  for (int d = 0; d < DEPTH; ++d)
    if (d < items) load_next(v[d]);
  for (int64_t it0 = 0; it0 < items; it0 += DEPTH) {
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
      const int64_t it = it0 + d;
      if (it >= items) break;
      const int ch = (int)(it & ((1 << lnch) - 1));
      const int64_t m0 = ((int64_t)blockIdx.x + (it >> lnch) * (int64_t)gridDim.x) * kSkewPM;
      __syncthreads();  // the previous chunk's products have read As (and Bs)
#pragma unroll
      for (int j = 0; j < LPT; ++j) {
#pragma unroll
        for (int u = 0; u < VEC; ++u) {
          const float2 x = to_f2(v[d][j][u]);
          As[eidx[j][u]] = x.x;
          As[KC * kSkewLDA + eidx[j][u]] = x.y;
        }
      }
      if (it + DEPTH < items) load_next(v[d]);
      if (!bres) stage_b(ch * KC, KC);
      __syncthreads();
      if (ch == 0) {
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
          for (int j = 0; j < NT; ++j) acc[p][j] = floatx16{};
      }
      const int kb0 = bres ? ch * KC : 0;
      // the chunk's operands first (all LDS reads in flight together), then
      // the products
      float ar[KC / 2], ai[KC / 2], br[KC / 2][NT], bi[KC / 2][NT];
#pragma unroll
      for (int s2 = 0; s2 < KC / 2; ++s2) {
        ar[s2] = As[aidx[s2]];
        ai[s2] = As[KC * kSkewLDA + aidx[s2]];
        const int kr = kb0 + 2 * s2 + kh;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          br[s2][j] = Bs[kr * LDB + 32 * j + c];
          bi[s2][j] = Bs[(KB + kr) * LDB + 32 * j + c];
        }
      }
#pragma unroll
      for (int s2 = 0; s2 < KC / 2; ++s2) {
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          acc[0][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[s2], br[s2][j], acc[0][j], 0, 0, 0);
          acc[1][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[s2], bi[s2][j], acc[1][j], 0, 0, 0);
          acc[2][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[s2] + ai[s2], br[s2][j] + bi[s2][j], acc[2][j], 0,
                                                           0, 0);
        }
      }
      if (ch == (1 << lnch) - 1) {
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
              skew_st_nt(C + (((m0 + row) << op.nN) | col), from_f2<E>(cr * op.out_scale, ci * op.out_scale));
            }
          }
        }
      }
    }
  }
  __syncthreads();
  record_max_in(maxslot, mx, reinterpret_cast<float*>(bn));
}

// Steady-state form for B resident in LDS and K = KC * NCH <= 64: one loop
// iteration is one pass of 128 rows, its NCH chunks unrolled, so the loads,
// LDS stores, matrix products and C stores of a pass are straight-line code
// the compiler can schedule with exact memory counters.  Prefetch distance:
// PD passes (the NCH * PD register slots hold the chunks of the next PD
// passes; a chunk's slot is reloaded as soon as the chunk is in LDS, so
// the loads spread over the pass); past the last pass the loads repeat the
// last pass's chunks (read, never used).
// STG: rows of at most 16 outputs (NT = 1): a pass's 128 x N outputs are one
// contiguous range of C; they are staged in the (then idle) A chunk planes
// and written in 16-byte runs instead of one 8- or 4-byte store per lane.
template <int NT, int VEC, int KC, int NCH, int PD, int STG, typename E>
__global__ __launch_bounds__(256, 2) void k_skew_p(const E* __restrict__ A, const E* __restrict__ B,
                                                  E* __restrict__ C, const IndexOp op, const SkewMap mp,
                                                  float* maxslot) {
  constexpr int NP = 32 * NT, LDB = NP + 4, K = KC * NCH;
  constexpr int LPT = (kSkewPM * KC) / 256 / VEC;  // loads per thread per chunk
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int N = 1 << op.nN;
  float* As = reinterpret_cast<float*>(smem);  // [2][KC][LDA]
  float* Bs = As + 2 * KC * kSkewLDA;          // [2][K][LDB]
  uint64_t* bn = reinterpret_cast<uint64_t*>(Bs + 2 * K * LDB);  // [64]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 31, kh = lane >> 5;
  if (tid < 64) bn[tid] = tid < N ? dep((uint64_t)tid, op.bN) : 0;
  uint64_t kA0[NCH];  // A offset of each chunk's first k (uniform)
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) kA0[ch] = dep((uint64_t)ch * KC, op.aK);
  uint64_t eoff[LPT];
  int eidx[LPT][VEC];
#pragma unroll
  for (int j = 0; j < LPT; ++j) {
#pragma unroll
    for (int u = 0; u < VEC; ++u) {
      uint64_t off;
      int m, k;
      skew_split(mp, (j * 256 + tid) * VEC + u, off, m, k);
      if (u == 0) eoff[j] = off;
      eidx[j][u] = k * kSkewLDA + (m ^ skew_h(mp, m, k));
    }
  }
  int aidx[KC / 2];
#pragma unroll
  for (int s2 = 0; s2 < KC / 2; ++s2) {
    const int k = 2 * s2 + kh, m = wave * 32 + c;
    aidx[s2] = k * kSkewLDA + (m ^ skew_h(mp, m, k));
  }
  __syncthreads();
  for (int i = tid; i < K * NP; i += 256) {
    const int n = i % NP, k = i / NP;
    const float2 v = n < N ? to_f2(B[bn[n] | dep((uint64_t)k, op.bK)]) : make_float2(0.f, 0.f);
    Bs[k * LDB + n] = v.x;
    Bs[(K + k) * LDB + n] = v.y;
  }
  const int64_t passes = ((int64_t)1 << op.nM) / kSkewPM;
  const int64_t my_passes = passes > (int64_t)blockIdx.x ? (passes - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
  const uint64_t mask_m = dep(((uint64_t)1 << op.nM) - kSkewPM, op.aM);
  const uint64_t inc_m = dep((uint64_t)gridDim.x * kSkewPM, op.aM);
  uint64_t pf_m = dep((uint64_t)blockIdx.x * kSkewPM, op.aM);  // row part of the next pass to prefetch
  int64_t pf_left = my_passes;                                   // passes not yet prefetched
  E v[PD][NCH][LPT][VEC];
  // chunk ch of the pass being prefetched into dst; after its last chunk the
  // cursor moves to the next pass (the last pass is reloaded at the tail)
  auto load_chunk = [&](E (&dst)[LPT][VEC], int ch) {
    const E* base = A + (pf_m | kA0[ch]);
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
      if constexpr (VEC == 1) {
        dst[j][0] = skew_ld_nt(base + eoff[j]);
      } else {
        const skew_u32x4 w = __builtin_nontemporal_load(reinterpret_cast<const skew_u32x4*>(base + eoff[j]));
        __builtin_memcpy(&dst[j][0], &w, 16);
      }
    }
    if (ch == NCH - 1) {
      if (pf_left > 1) pf_m = ((pf_m | ~mask_m) + inc_m) & mask_m;
      --pf_left;
    }
  };
#pragma unroll
  for (int d = 0; d < PD; ++d)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) load_chunk(v[d][ch], ch);
  float mx = 0.f;
  for (int64_t p0 = 0; p0 < my_passes; p0 += PD) {
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      const int64_t pi = p0 + d;
      if (pi >= my_passes) break;
      const int64_t m0 = ((int64_t)blockIdx.x + pi * (int64_t)gridDim.x) * kSkewPM;
      floatx16 acc[3][NT];
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[q][j] = floatx16{};
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        __syncthreads();  // the previous chunk's products have read As (B is staged before the first)
#pragma unroll
        for (int j = 0; j < LPT; ++j)
#pragma unroll
          for (int u = 0; u < VEC; ++u) {
            const float2 x = to_f2(v[d][ch][j][u]);
            As[eidx[j][u]] = x.x;
            As[KC * kSkewLDA + eidx[j][u]] = x.y;
          }
        // the slot is free: the same chunk PD passes ahead
        load_chunk(v[d][ch], ch);
        __syncthreads();
        float ar[KC / 2], ai[KC / 2], br[KC / 2][NT], bi[KC / 2][NT];
#pragma unroll
        for (int s2 = 0; s2 < KC / 2; ++s2) {
          ar[s2] = As[aidx[s2]];
          ai[s2] = As[KC * kSkewLDA + aidx[s2]];
          const int kr = ch * KC + 2 * s2 + kh;
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            br[s2][j] = Bs[kr * LDB + 32 * j + c];
            bi[s2][j] = Bs[(K + kr) * LDB + 32 * j + c];
          }
        }
#pragma unroll
        for (int s2 = 0; s2 < KC / 2; ++s2)
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            acc[0][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[s2], br[s2][j], acc[0][j], 0, 0, 0);
            acc[1][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai[s2], bi[s2][j], acc[1][j], 0, 0, 0);
            acc[2][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[s2] + ai[s2], br[s2][j] + bi[s2][j], acc[2][j],
                                                             0, 0, 0);
          }
      }
      if constexpr (STG) {
        __syncthreads();  // every wave has multiplied the pass's last chunk
        E* Cs = reinterpret_cast<E*>(As);
        if (c < N) {
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = wave * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
            const float cr = acc[0][0][r] - acc[1][0][r];
            const float ci = acc[2][0][r] - acc[0][0][r] - acc[1][0][r];
            mx = mag_max(mx, cr, ci);
            Cs[row * N + c] = from_f2<E>(cr * op.out_scale, ci * op.out_scale);
          }
        }
        __syncthreads();
        constexpr int EPV = 16 / (int)sizeof(E);
        E* Cp = C + (m0 << op.nN);
        for (int i = tid * EPV; i < kSkewPM * N; i += 256 * EPV)
          __builtin_nontemporal_store(*reinterpret_cast<const skew_u32x4*>(Cs + i),
                                      reinterpret_cast<skew_u32x4*>(Cp + i));
      } else {
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
              skew_st_nt(C + (((m0 + row) << op.nN) | col), from_f2<E>(cr * op.out_scale, ci * op.out_scale));
            }
          }
        }
      }
    }
  }
  __syncthreads();
  record_max_in(maxslot, mx, reinterpret_cast<float*>(bn));
}

static size_t skew_p_lds(int kc, int K, int np) { return 2 * kc * kSkewLDA * 4 + 2 * K * (np + 4) * 4 + 64 * 8; }

// Scaled FP16 / BF16 storage on the half-precision matrix cores
// (v_mfma_f32_32x32x16_{f16,bf16}: 16 k per instruction, FP32 accumulation)
// in the 4M form, Cr = Ar Br + (-Ai) Bi, Ci = Ar Bi + Ai Br: the products of
// the stored 16-bit values are exact in the FP32 accumulator, so no operand
// sum is rounded.  Same pass structure as k_skew_p with KC = 16; the chunk
// goes to LDS as planar 16-bit rows [m][k] (k contiguous, rows padded to 24
// entries) so that each lane reads its eight consecutive k in one 16-byte
// load, and B is resident as planar rows [n][k].
typedef _Float16 skew_half8 __attribute__((ext_vector_type(8)));
typedef __bf16 skew_bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kSkewHS = 24;  // LDS row stride of the 16-bit planes (entries)

template <typename E>
struct SkewHalf;
template <>
struct SkewHalf<cf16> {
  typedef _Float16 H;
  typedef skew_half8 V;
  static __device__ __forceinline__ floatx16 mfma(V a, V b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct SkewHalf<cbf16> {
  typedef __bf16 H;
  typedef skew_bf16x8 V;
  static __device__ __forceinline__ floatx16 mfma(V a, V b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

template <int NT, int VEC, int NCH, int PD, typename E>
__global__ __launch_bounds__(256, 2) void k_skew_ph(const E* __restrict__ A, const E* __restrict__ B,
                                                   E* __restrict__ C, const IndexOp op, const SkewMap mp,
                                                   float* maxslot) {
  typedef typename SkewHalf<E>::H H;
  typedef typename SkewHalf<E>::V V;
  constexpr int KC = 16, NP = 32 * NT, K = KC * NCH;
  constexpr int LPT = (kSkewPM * KC) / 256 / VEC;
  constexpr int KS = K + 8;  // B row stride (entries): 16-byte aligned rows
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int N = 1 << op.nN;
  H* As = reinterpret_cast<H*>(smem);            // [2][PM][kSkewHS]
  H* Bs = As + 2 * kSkewPM * kSkewHS;            // [2][NP][KS]
  uint64_t* bn = reinterpret_cast<uint64_t*>(Bs + 2 * NP * KS);  // [64]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 31, kh = lane >> 5;
  if (tid < 64) bn[tid] = tid < N ? dep((uint64_t)tid, op.bN) : 0;
  uint64_t kA0[NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) kA0[ch] = dep((uint64_t)ch * KC, op.aK);
  uint64_t eoff[LPT];
  int eidx[LPT][VEC];  // LDS index m * kSkewHS + k of each entry
#pragma unroll
  for (int j = 0; j < LPT; ++j) {
#pragma unroll
    for (int u = 0; u < VEC; ++u) {
      uint64_t off;
      int m, k;
      skew_split(mp, (j * 256 + tid) * VEC + u, off, m, k);
      if (u == 0) eoff[j] = off;
      eidx[j][u] = m * kSkewHS + k;
    }
  }
  __syncthreads();
  for (int i = tid; i < K * NP; i += 256) {
    const int k = i % K, n = i / K;
    E v{};
    if (n < N) v = B[bn[n] | dep((uint64_t)k, op.bK)];
    Bs[n * KS + k] = v.re;
    Bs[(NP + n) * KS + k] = v.im;
  }
  const int64_t passes = ((int64_t)1 << op.nM) / kSkewPM;
  const int64_t my_passes = passes > (int64_t)blockIdx.x ? (passes - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
  const uint64_t mask_m = dep(((uint64_t)1 << op.nM) - kSkewPM, op.aM);
  const uint64_t inc_m = dep((uint64_t)gridDim.x * kSkewPM, op.aM);
  uint64_t pf_m = dep((uint64_t)blockIdx.x * kSkewPM, op.aM);
  int64_t pf_left = my_passes;
  E v[PD][NCH][LPT][VEC];
  auto load_chunk = [&](E (&dst)[LPT][VEC], int ch) {
    const E* base = A + (pf_m | kA0[ch]);
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
      if constexpr (VEC == 1) {
        dst[j][0] = skew_ld_nt(base + eoff[j]);
      } else {
        const skew_u32x4 w = __builtin_nontemporal_load(reinterpret_cast<const skew_u32x4*>(base + eoff[j]));
        __builtin_memcpy(&dst[j][0], &w, 16);
      }
    }
    if (ch == NCH - 1) {
      if (pf_left > 1) pf_m = ((pf_m | ~mask_m) + inc_m) & mask_m;
      --pf_left;
    }
  };
#pragma unroll
  for (int d = 0; d < PD; ++d)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) load_chunk(v[d][ch], ch);
  const int arow = (wave * 32 + c) * kSkewHS + 8 * kh;  // this lane's 8 k of its row
  float mx = 0.f;
  for (int64_t p0 = 0; p0 < my_passes; p0 += PD) {
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      const int64_t pi = p0 + d;
      if (pi >= my_passes) break;
      const int64_t m0 = ((int64_t)blockIdx.x + pi * (int64_t)gridDim.x) * kSkewPM;
      floatx16 acc[2][NT];
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[q][j] = floatx16{};
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < LPT; ++j)
#pragma unroll
          for (int u = 0; u < VEC; ++u) {
            As[eidx[j][u]] = v[d][ch][j][u].re;
            As[kSkewPM * kSkewHS + eidx[j][u]] = v[d][ch][j][u].im;
          }
        load_chunk(v[d][ch], ch);
        __syncthreads();
        const V ar = *reinterpret_cast<const V*>(As + arow);
        const V ai = *reinterpret_cast<const V*>(As + kSkewPM * kSkewHS + arow);
        const V nai = -ai;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const int brow = (32 * j + c) * KS + ch * KC + 8 * kh;
          const V br = *reinterpret_cast<const V*>(Bs + brow);
          const V bi = *reinterpret_cast<const V*>(Bs + NP * KS + brow);
          acc[0][j] = SkewHalf<E>::mfma(ar, br, acc[0][j]);
          acc[0][j] = SkewHalf<E>::mfma(nai, bi, acc[0][j]);
          acc[1][j] = SkewHalf<E>::mfma(ar, bi, acc[1][j]);
          acc[1][j] = SkewHalf<E>::mfma(ai, br, acc[1][j]);
        }
      }
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const int col = 32 * j + c;
        if (col < N) {
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = wave * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
            const float cr = acc[0][j][r], ci = acc[1][j][r];
            mx = mag_max(mx, cr, ci);
            skew_st_nt(C + (((m0 + row) << op.nN) | col), from_f2<E>(cr * op.out_scale, ci * op.out_scale));
          }
        }
      }
    }
  }
  __syncthreads();
  record_max_in(maxslot, mx, reinterpret_cast<float*>(bn));
}

static size_t skew_ph_lds(int K, int np) { return 2 * kSkewPM * kSkewHS * 2 + 2 * np * (K + 8) * 2 + 64 * 8; }

// Scaled FP16 / BF16 with a long sum (128 <= K <= 2^10): B does not stay
// in LDS (Fig. S7b's case), so each 16-k chunk of B (2^nN x 16 entries,
// re-read from L2 by every pass) is staged beside the chunk of A.  Chunks
// run in a runtime loop, two per iteration so that each has its own
// registers: the chunk two ahead is loaded while the current one is
// multiplied.  The chunks' K offsets in A and B move by one XOR per chunk
// with prefix tables (B's K bits need not keep their order).  Past the last
// pass the loads repeat the last pass's chunks (read, never used).
constexpr int kSkewBS = 24;  // LDS row stride of a staged B chunk (entries)

template <int NT, int VEC, typename E>
__global__ __launch_bounds__(256, 2) void k_skew_phc(const E* __restrict__ A, const E* __restrict__ B,
                                                    E* __restrict__ C, const IndexOp op, const SkewMap mp,
                                                    float* maxslot) {
  typedef typename SkewHalf<E>::H H;
  typedef typename SkewHalf<E>::V V;
  constexpr int KC = 16, NP = 32 * NT;
  constexpr int LPT = (kSkewPM * KC) / 256 / VEC;
  constexpr int NBT = NP * KC / 256;  // B entries per thread per chunk
  __shared__ __attribute__((aligned(16))) H As[2 * kSkewPM * kSkewHS];  // re, im planes [PM][HS]
  __shared__ __attribute__((aligned(16))) H Bs[2 * NP * kSkewBS];       // re, im planes [NP][BS]
  __shared__ uint64_t pre_a[12], pre_b[12];
  __shared__ float red[16];
  const int N = 1 << op.nN;
  const int nch = 1 << (op.nK - 4);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 31, kh = lane >> 5;
  // prefix tables: chunk ch -> ch + 1 flips the chunk-index bits 0 .. ctz(ch + 1)
  if (tid < op.nK - 4) {
    uint64_t xa = 0, xb = 0;
    for (int j = 0; j <= tid; ++j) {
      xa ^= dep((uint64_t)KC << j, op.aK);
      xb ^= dep((uint64_t)KC << j, op.bK);
    }
    pre_a[tid] = xa;
    pre_b[tid] = xb;
  }
  uint64_t eoff[LPT];
  int eidx[LPT][VEC];  // LDS index m * kSkewHS + k of each A entry
#pragma unroll
  for (int j = 0; j < LPT; ++j) {
#pragma unroll
    for (int u = 0; u < VEC; ++u) {
      uint64_t off;
      int m, k;
      skew_split(mp, (j * 256 + tid) * VEC + u, off, m, k);
      if (u == 0) eoff[j] = off;
      eidx[j][u] = m * kSkewHS + k;
    }
  }
  uint64_t boff[NBT];
  int bidx[NBT];
  bool bval[NBT];
#pragma unroll
  for (int r = 0; r < NBT; ++r) {
    const int i = r * 256 + tid, n = i / KC, k = i % KC;
    bval[r] = n < N;
    boff[r] = bval[r] ? (dep((uint64_t)n, op.bN) | dep((uint64_t)k, op.bK)) : 0;
    bidx[r] = n * kSkewBS + k;
  }
  const int64_t passes = ((int64_t)1 << op.nM) / kSkewPM;
  const int64_t my_passes = passes > (int64_t)blockIdx.x ? (passes - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
  const uint64_t mask_m = dep(((uint64_t)1 << op.nM) - kSkewPM, op.aM);
  const uint64_t inc_m = dep((uint64_t)gridDim.x * kSkewPM, op.aM);
  __syncthreads();
  // the chunk being prefetched: its pass's row offset, chunk index and K offsets
  uint64_t pf_m = dep((uint64_t)blockIdx.x * kSkewPM, op.aM), pf_ka = 0, pf_kb = 0;
  int pf_ch = 0;
  int64_t pf_left = my_passes;  // passes not yet fully prefetched
  E v[2][LPT][VEC];
  E w[2][NBT];
  auto prefetch = [&](int d) {
    const E* base = A + (pf_m | pf_ka);
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
      if constexpr (VEC == 1) {
        v[d][j][0] = skew_ld_nt(base + eoff[j]);
      } else {
        const skew_u32x4 x = __builtin_nontemporal_load(reinterpret_cast<const skew_u32x4*>(base + eoff[j]));
        __builtin_memcpy(&v[d][j][0], &x, 16);
      }
    }
#pragma unroll
    for (int r = 0; r < NBT; ++r) w[d][r] = B[pf_kb | boff[r]];
    if (++pf_ch == nch) {
      pf_ch = 0;
      pf_ka = pf_kb = 0;
      if (pf_left > 1) pf_m = ((pf_m | ~mask_m) + inc_m) & mask_m;
      --pf_left;
    } else {
      const int t = __builtin_ctz((unsigned)pf_ch);
      pf_ka ^= pre_a[t];
      pf_kb ^= pre_b[t];
    }
  };
  prefetch(0);
  prefetch(1);
  const int arow = (wave * 32 + c) * kSkewHS + 8 * kh;
  float mx = 0.f;
  for (int64_t pi = 0; pi < my_passes; ++pi) {
    const int64_t m0 = ((int64_t)blockIdx.x + pi * (int64_t)gridDim.x) * kSkewPM;
    floatx16 acc[2][NT];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[q][j] = floatx16{};
    for (int ch = 0; ch < nch; ch += 2) {
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        __syncthreads();  // the previous chunk's products have read As and Bs
#pragma unroll
        for (int j = 0; j < LPT; ++j)
#pragma unroll
          for (int u = 0; u < VEC; ++u) {
            As[eidx[j][u]] = v[d][j][u].re;
            As[kSkewPM * kSkewHS + eidx[j][u]] = v[d][j][u].im;
          }
#pragma unroll
        for (int r = 0; r < NBT; ++r) {
          const E x = bval[r] ? w[d][r] : E{};
          Bs[bidx[r]] = x.re;
          Bs[NP * kSkewBS + bidx[r]] = x.im;
        }
        prefetch(d);  // two chunks ahead
        __syncthreads();
        const V ar = *reinterpret_cast<const V*>(As + arow);
        const V ai = *reinterpret_cast<const V*>(As + kSkewPM * kSkewHS + arow);
        const V nai = -ai;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const int brow = (32 * j + c) * kSkewBS + 8 * kh;
          const V br = *reinterpret_cast<const V*>(Bs + brow);
          const V bi = *reinterpret_cast<const V*>(Bs + NP * kSkewBS + brow);
          acc[0][j] = SkewHalf<E>::mfma(ar, br, acc[0][j]);
          acc[0][j] = SkewHalf<E>::mfma(nai, bi, acc[0][j]);
          acc[1][j] = SkewHalf<E>::mfma(ar, bi, acc[1][j]);
          acc[1][j] = SkewHalf<E>::mfma(ai, br, acc[1][j]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int col = 32 * j + c;
      if (col < N) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = wave * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
          const float cr = acc[0][j][r], ci = acc[1][j][r];
          mx = mag_max(mx, cr, ci);
          skew_st_nt(C + (((m0 + row) << op.nN) | col), from_f2<E>(cr * op.out_scale, ci * op.out_scale));
        }
      }
    }
  }
  __syncthreads();
  record_max_in(maxslot, mx, red);
}

bool skew_ok(const IndexOp& op) { return op.nN <= 6 && op.nK >= 1 && op.nK <= 10 && op.nM >= 7; }

bool skew_map(const IndexOp& op, int kcb, int lv, SkewMap* mp) {
  struct Var {
    int pos, m, k;
  };
  std::vector<Var> vars;
  for (int j = 0; j < 7; ++j) vars.push_back({run_pos(op.aM, j), j, -1});
  for (int j = 0; j < kcb; ++j) vars.push_back({run_pos(op.aK, j), -1, j});
  for (const Var& x : vars)
    if (x.pos < 0) return false;
  std::sort(vars.begin(), vars.end(), [](const Var& a, const Var& b) { return a.pos < b.pos; });
  mp->v = (int)vars.size();
  for (int i = 0; i < mp->v; ++i) {
    mp->pos[i] = (int8_t)vars[i].pos;
    mp->mb[i] = (int8_t)vars[i].m;
    mp->kb[i] = (int8_t)vars[i].k;
  }
  // swizzle: a half-wave's store instruction covers chunk bits lv .. lv+4;
  // row bits 0..4 among them are bank bits already, the others (k bits, row
  // bits 5 and 6) are sent to the bank bits left free
  for (int i = 0; i < 5; ++i) mp->hk[i] = 0;
  mp->hm[0] = mp->hm[1] = 0;
  unsigned used = 0;
  for (int i = lv; i < std::min(mp->v, lv + 5); ++i)
    if (mp->mb[i] >= 0 && mp->mb[i] < 5) used |= 1u << mp->mb[i];
  int next = 0;
  for (int i = lv; i < std::min(mp->v, lv + 5); ++i) {
    const bool direct = mp->mb[i] >= 0 && mp->mb[i] < 5;
    if (direct) continue;
    while (next < 5 && (used >> next & 1)) ++next;
    if (next >= 5) break;
    used |= 1u << next;
    if (mp->kb[i] >= 0)
      mp->hk[mp->kb[i]] = (int8_t)(1 << next);
    else
      mp->hm[mp->mb[i] - 5] = (int8_t)(1 << next);
  }
  return true;
}

template <int NT, int VEC, int KC, typename E>
static hipError_t launch_skew_v(const E* A, const E* B, E* C, const IndexOp& op, const SkewMap& mp, float* maxslot,
                                hipStream_t s) {
  const int np = 32 * NT;
  const bool bres = skew_lds(op.nK, np, true) <= 64 * 1024;
  const size_t lds = skew_lds(op.nK, np, bres);
  if (lds > 64 * 1024) return hipErrorInvalidValue;
  const int64_t passes = ((int64_t)1 << op.nM) / kSkewPM;
  const dim3 g((unsigned)std::min<int64_t>(passes, 2048));
  // loads per thread: 2^v entries over 256 threads, VEC per load (v >= 8,
  // and VEC > 1 only when 2^v >= 256 VEC)
  const int lpt = ((1 << mp.v) / 256) / VEC;
  if (lpt < 1 || lpt * 256 * VEC != (1 << mp.v)) return hipErrorInvalidValue;
  const int bres_i = bres ? 1 : 0;
  // chunks loaded ahead: about 128 bytes per thread in flight
  switch (lpt) {
    case 1:
      hipLaunchKernelGGL((k_skew<NT, VEC, 1, 4, KC, E>), g, dim3(256), lds, s, A, B, C, op, mp, maxslot, bres_i);
      break;
    case 2:
      hipLaunchKernelGGL((k_skew<NT, VEC, 2, (VEC * sizeof(E) >= 8 ? 4 : 2), KC, E>), g, dim3(256), lds, s, A, B,
                         C, op, mp, maxslot, bres_i);
      break;
    case 4:
      hipLaunchKernelGGL((k_skew<NT, VEC, 4, 2, KC, E>), g, dim3(256), lds, s, A, B, C, op, mp, maxslot, bres_i);
      break;
    default:
      if constexpr (VEC == 1)  // 2^11 entries, one per load (with 16-byte loads at most 4 per thread)
        hipLaunchKernelGGL((k_skew<NT, VEC, 8, 2, KC, E>), g, dim3(256), lds, s, A, B, C, op, mp, maxslot, bres_i);
      else
        return hipErrorInvalidValue;
      break;
  }
  return hipGetLastError();
}

template <int NT, int VEC, typename E>
static hipError_t launch_skew_kc(const E* A, const E* B, E* C, const IndexOp& op, const SkewMap& mp,
                                 float* maxslot, hipStream_t s) {
  switch (op.nK) {
    case 1: return launch_skew_v<NT, VEC, 2, E>(A, B, C, op, mp, maxslot, s);
    case 2: return launch_skew_v<NT, VEC, 4, E>(A, B, C, op, mp, maxslot, s);
    case 3: return launch_skew_v<NT, VEC, 8, E>(A, B, C, op, mp, maxslot, s);
    default: return launch_skew_v<NT, VEC, kSkewKC, E>(A, B, C, op, mp, maxslot, s);
  }
}

template <int NT, int VEC, int KC, int NCH, typename E>
static hipError_t launch_skew_pass(const E* A, const E* B, E* C, const IndexOp& op, const SkewMap& mp,
                                   float* maxslot, hipStream_t s) {
  constexpr int PD = NCH >= 4 ? 1 : 2;  // prefetch distance in passes: NCH * PD chunks
  const size_t lds = skew_p_lds(KC, KC * NCH, 32 * NT);
  const int64_t passes = ((int64_t)1 << op.nM) / kSkewPM;
  const dim3 g((unsigned)std::min<int64_t>(passes, 512));
  // staged output rows: at most 16 per row, fitting the A chunk planes
  const bool stg = NT == 1 && op.nN <= 4 &&
                   (size_t)kSkewPM * ((size_t)1 << op.nN) * sizeof(E) <= (size_t)2 * KC * kSkewLDA * sizeof(float) &&
                   kSkewPM * ((int64_t)1 << op.nN) * (int64_t)sizeof(E) >= 16;
  if (stg)
    hipLaunchKernelGGL((k_skew_p<NT, VEC, KC, NCH, PD, 1, E>), g, dim3(256), lds, s, A, B, C, op, mp, maxslot);
  else
    hipLaunchKernelGGL((k_skew_p<NT, VEC, KC, NCH, PD, 0, E>), g, dim3(256), lds, s, A, B, C, op, mp, maxslot);
  return hipGetLastError();
}

template <int NT, int VEC, typename E>
static hipError_t launch_skew_pk(const E* A, const E* B, E* C, const IndexOp& op, const SkewMap& mp, float* maxslot,
                                 hipStream_t s) {
  switch (op.nK) {
    case 1:
      if constexpr (VEC == 1) return launch_skew_pass<NT, VEC, 2, 1, E>(A, B, C, op, mp, maxslot, s);
      break;
    case 2:
      if constexpr (VEC <= 2) return launch_skew_pass<NT, VEC, 4, 1, E>(A, B, C, op, mp, maxslot, s);
      break;
    case 3: return launch_skew_pass<NT, VEC, 8, 1, E>(A, B, C, op, mp, maxslot, s);
    case 4: return launch_skew_pass<NT, VEC, 16, 1, E>(A, B, C, op, mp, maxslot, s);
    case 5: return launch_skew_pass<NT, VEC, 16, 2, E>(A, B, C, op, mp, maxslot, s);
    case 6: return launch_skew_pass<NT, VEC, 16, 4, E>(A, B, C, op, mp, maxslot, s);
    default: break;
  }
  return hipErrorInvalidValue;
}

template <int NT, typename E>
static hipError_t launch_skew_t(const E* A, const E* B, E* C, const IndexOp& op, float* maxslot, hipStream_t s) {
  constexpr int VEC = 16 / (int)sizeof(E);
  constexpr int LV = VEC == 4 ? 2 : 1;
  const int kcb = std::min(op.nK, 4);
  // 16-byte loads: the chunk's lowest bits are A's lowest bits, and every
  // thread gets at least one full vector
  SkewMap mp{};
  if (!skew_map(op, kcb, LV, &mp)) return hipErrorInvalidValue;
  bool vec = (1 << mp.v) >= 256 * VEC;
  for (int i = 0; i < LV; ++i) vec = vec && mp.pos[i] == i;
  // pass kernel: K <= 64 with B resident
  const bool pass = op.nK <= 6 && skew_p_lds(1 << kcb, 1 << op.nK, 32 * NT) <= 64 * 1024;
  if (vec) {
    if (pass) return launch_skew_pk<NT, VEC, E>(A, B, C, op, mp, maxslot, s);
    return launch_skew_kc<NT, VEC, E>(A, B, C, op, mp, maxslot, s);
  }
  if (!skew_map(op, kcb, 0, &mp)) return hipErrorInvalidValue;
  if (pass) return launch_skew_pk<NT, 1, E>(A, B, C, op, mp, maxslot, s);
  return launch_skew_kc<NT, 1, E>(A, B, C, op, mp, maxslot, s);
}

template <int NT, int VEC, int NCH, typename E>
static hipError_t launch_skew_half(const E* A, const E* B, E* C, const IndexOp& op, const SkewMap& mp,
                                   float* maxslot, hipStream_t s) {
  constexpr int PD = NCH >= 4 ? 1 : 2;
  const size_t lds = skew_ph_lds(16 * NCH, 32 * NT);
  const int64_t passes = ((int64_t)1 << op.nM) / kSkewPM;
  const dim3 g((unsigned)std::min<int64_t>(passes, 512));
  hipLaunchKernelGGL((k_skew_ph<NT, VEC, NCH, PD, E>), g, dim3(256), lds, s, A, B, C, op, mp, maxslot);
  return hipGetLastError();
}

// 16-bit storage with 16 <= K <= 64: the half-precision matrix cores
template <int NT, typename E>
static hipError_t launch_skew_h(const E* A, const E* B, E* C, const IndexOp& op, float* maxslot, hipStream_t s) {
  constexpr int VEC = 16 / (int)sizeof(E);
  SkewMap mp{};
  if (!skew_map(op, 4, 2, &mp)) return hipErrorInvalidValue;
  const bool vec = mp.pos[0] == 0 && mp.pos[1] == 1;
  if (vec) {
    switch (op.nK) {
      case 4: return launch_skew_half<NT, VEC, 1, E>(A, B, C, op, mp, maxslot, s);
      case 5: return launch_skew_half<NT, VEC, 2, E>(A, B, C, op, mp, maxslot, s);
      default: return launch_skew_half<NT, VEC, 4, E>(A, B, C, op, mp, maxslot, s);
    }
  }
  switch (op.nK) {
    case 4: return launch_skew_half<NT, 1, 1, E>(A, B, C, op, mp, maxslot, s);
    case 5: return launch_skew_half<NT, 1, 2, E>(A, B, C, op, mp, maxslot, s);
    default: return launch_skew_half<NT, 1, 4, E>(A, B, C, op, mp, maxslot, s);
  }
}

// 16-bit storage with 128 <= K <= 2^10: B staged chunk by chunk
template <int NT, typename E>
static hipError_t launch_skew_hc(const E* A, const E* B, E* C, const IndexOp& op, float* maxslot, hipStream_t s) {
  constexpr int VEC = 16 / (int)sizeof(E);
  SkewMap mp{};
  if (!skew_map(op, 4, 2, &mp)) return hipErrorInvalidValue;
  const int64_t passes = ((int64_t)1 << op.nM) / kSkewPM;
  const dim3 g((unsigned)std::min<int64_t>(passes, 512));
  if (mp.pos[0] == 0 && mp.pos[1] == 1)
    hipLaunchKernelGGL((k_skew_phc<NT, VEC, E>), g, dim3(256), 0, s, A, B, C, op, mp, maxslot);
  else
    hipLaunchKernelGGL((k_skew_phc<NT, 1, E>), g, dim3(256), 0, s, A, B, C, op, mp, maxslot);
  return hipGetLastError();
}

template <typename E>
static hipError_t launch_skew_e(const E* A, const E* B, E* C, const IndexOp& op, float* maxslot, hipStream_t s) {
  if constexpr (sizeof(E) == 4) {
    if (op.nK >= 4 && op.nK <= 6) {
      if (op.nN <= 5) return launch_skew_h<1, E>(A, B, C, op, maxslot, s);
      return launch_skew_h<2, E>(A, B, C, op, maxslot, s);
    }
    if (op.nK >= 7 && op.nK <= 10) {
      if (op.nN <= 5) return launch_skew_hc<1, E>(A, B, C, op, maxslot, s);
      return launch_skew_hc<2, E>(A, B, C, op, maxslot, s);
    }
  }
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
