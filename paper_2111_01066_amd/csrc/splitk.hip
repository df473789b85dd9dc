// Split-K contraction that reads both operands in place (gfx950): a long sum
// into at most 8 x 8 outputs, C[m][n] = sum_k A[m][k] B[n][k], with A and B
// in any bit layout.  It takes the place of the permutes that would bring
// each operand to [free wires, K] first (a long sum into few outputs is one
// skewed step of the network, Supplement Fig. S7: each operand is read once).
//
// The sum is cut into chunks of 2^8 k.  A chunk's k bits are the contracted
// bits that sit at the lowest positions of A and of B, so one chunk of A
// (2^nM rows x 256 k) and one of B are each a set of runs of consecutive
// addresses.  Each is loaded in address order (the chunk map of the skewed
// kernels) in loads of up to 16 bytes and staged in LDS as planar FP32 rows;
// thread t then multiplies chunk entry k = t into its 2^nM x 2^nN
// accumulators.
// Block b takes the chunks b, b + G, b + 2G, ... (G = gridDim.x, a power of
// two): from one to the next the bits lg .. lg + ctz(i + 1) of the chunk
// index flip (lg = log2 G), so the chunk's offsets in A and B move by one XOR
// each with prefix tables.  Two chunks are held in registers: the next one
// loads while the current one is multiplied.  Each block leaves its partial
// sums; the split-K final kernel adds them in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "elem.h"
#include "gather.h"
#include "kernels.h"

namespace tnrcs {

namespace {

constexpr int kChunkK = 1 << kSplitChunkLog2;  // k per chunk
constexpr int kChunkS = kChunkK + 4;           // LDS row stride (floats)

struct SplitChunk {
  SkewMap ma, mb;   // chunk element -> offset, row (m of A, n of B), chunk k
  Runs oA, oB;      // chunk index bit i -> its A / B position
  int32_t n_outer;  // chunk index bits
};

typedef unsigned int sk_u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int sk_u32x2 __attribute__((ext_vector_type(2)));

// W consecutive entries at p, nontemporal (each entry is read once).
template <int W, typename E>
__device__ __forceinline__ void ld_nt(const E* p, E (&v)[W]) {
  constexpr int nb = W * (int)sizeof(E);
  if constexpr (nb == 16) {
    const sk_u32x4 w = __builtin_nontemporal_load(reinterpret_cast<const sk_u32x4*>(p));
    __builtin_memcpy(v, &w, 16);
  } else if constexpr (nb == 8) {
    const sk_u32x2 w = __builtin_nontemporal_load(reinterpret_cast<const sk_u32x2*>(p));
    __builtin_memcpy(v, &w, 8);
  } else {
    static_assert(nb == 4, "4, 8 or 16 bytes");
    const unsigned w = __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p));
    __builtin_memcpy(v, &w, 4);
  }
}

template <int NM, int NN, typename E>
__global__ __launch_bounds__(256, 2) void k_splitk_chunk(const E* __restrict__ A, const E* __restrict__ B,
                                                        float2* __restrict__ part, const SplitChunk sc) {
  constexpr int VE = 16 / (int)sizeof(E);
  constexpr int WA = NM < VE ? NM : VE, WB = NN < VE ? NN : VE;  // entries per load
  constexpr int LA = NM / WA, LB = NN / WB;                      // loads per thread and chunk
  __shared__ float As[2 * NM * kChunkS], Bs[2 * NN * kChunkS];  // re plane, then im plane
  __shared__ uint64_t pre_a[64], pre_b[64];
  __shared__ float red[2][256];
  const int tid = threadIdx.x;
  const int lg = __builtin_ctz(gridDim.x);
  if (tid < sc.n_outer - lg) {
    uint64_t xa = 0, xb = 0;
    for (int j = 0; j <= tid; ++j) {
      xa ^= dep((uint64_t)1 << (lg + j), sc.oA);
      xb ^= dep((uint64_t)1 << (lg + j), sc.oB);
    }
    pre_a[tid] = xa;
    pre_b[tid] = xb;
  }
  // this thread's loads: chunk elements (j * 256 + tid) * W + u, their offset
  // from the chunk's first entry and their LDS slot row * stride + k
  uint64_t ea[LA], eb[LB];
  int sa[LA][WA], sb[LB][WB];
#pragma unroll
  for (int j = 0; j < LA; ++j)
#pragma unroll
    for (int u = 0; u < WA; ++u) {
      uint64_t off;
      int r, k;
      skew_split(sc.ma, (j * 256 + tid) * WA + u, off, r, k);
      if (u == 0) ea[j] = off;
      sa[j][u] = r * kChunkS + k;
    }
#pragma unroll
  for (int j = 0; j < LB; ++j)
#pragma unroll
    for (int u = 0; u < WB; ++u) {
      uint64_t off;
      int r, k;
      skew_split(sc.mb, (j * 256 + tid) * WB + u, off, r, k);
      if (u == 0) eb[j] = off;
      sb[j][u] = r * kChunkS + k;
    }
  __syncthreads();
  const int64_t iters = ((int64_t)1 << sc.n_outer) >> lg;  // a power of two, at least 1
  uint64_t pa = dep((uint64_t)blockIdx.x, sc.oA), pb = dep((uint64_t)blockIdx.x, sc.oB);
  int64_t pi = 0;  // iteration of the chunk being prefetched
  E va[2][LA][WA], vb[2][LB][WB];
  auto prefetch = [&](int d) {
#pragma unroll
    for (int j = 0; j < LA; ++j) ld_nt<WA>(A + (pa | ea[j]), va[d][j]);
#pragma unroll
    for (int j = 0; j < LB; ++j) ld_nt<WB>(B + (pb | eb[j]), vb[d][j]);
    if (++pi < iters) {
      const int t = __builtin_ctzll((unsigned long long)pi);
      pa ^= pre_a[t];
      pb ^= pre_b[t];
    }
  };
  float acc_r[NM][NN], acc_i[NM][NN];
#pragma unroll
  for (int i = 0; i < NM; ++i)
#pragma unroll
    for (int j = 0; j < NN; ++j) acc_r[i][j] = acc_i[i][j] = 0.f;
  prefetch(0);
  if (iters > 1) prefetch(1);
  for (int64_t it = 0; it < iters; it += 2) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      if (d == 1 && iters == 1) break;
      __syncthreads();  // the previous chunk's products have read As and Bs
#pragma unroll
      for (int j = 0; j < LA; ++j)
#pragma unroll
        for (int u = 0; u < WA; ++u) {
          const float2 x = to_f2(va[d][j][u]);
          As[sa[j][u]] = x.x;
          As[NM * kChunkS + sa[j][u]] = x.y;
        }
#pragma unroll
      for (int j = 0; j < LB; ++j)
#pragma unroll
        for (int u = 0; u < WB; ++u) {
          const float2 y = to_f2(vb[d][j][u]);
          Bs[sb[j][u]] = y.x;
          Bs[NN * kChunkS + sb[j][u]] = y.y;
        }
      __syncthreads();
      if (it + d + 2 < iters) prefetch(d);
      float yr[NN], yi[NN];
#pragma unroll
      for (int n = 0; n < NN; ++n) {
        yr[n] = Bs[n * kChunkS + tid];
        yi[n] = Bs[NN * kChunkS + n * kChunkS + tid];
      }
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const float xr = As[m * kChunkS + tid], xi = As[NM * kChunkS + m * kChunkS + tid];
#pragma unroll
        for (int n = 0; n < NN; ++n) {
          acc_r[m][n] = fmaf(xr, yr[n], acc_r[m][n]);
          acc_r[m][n] = fmaf(-xi, yi[n], acc_r[m][n]);
          acc_i[m][n] = fmaf(xr, yi[n], acc_i[m][n]);
          acc_i[m][n] = fmaf(xi, yr[n], acc_i[m][n]);
        }
      }
    }
  }
  // block sum in a fixed order: butterfly within each wave, then the four
  // wave sums in wave order
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int m = 0; m < NM; ++m)
#pragma unroll
    for (int n = 0; n < NN; ++n) {
      float r = acc_r[m][n], q = acc_i[m][n];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        r += __shfl_xor(r, o);
        q += __shfl_xor(q, o);
      }
      if (lane == 0) {
        red[0][wave * 64 + m * NN + n] = r;
        red[1][wave * 64 + m * NN + n] = q;
      }
    }
  __syncthreads();
  constexpr int nout = NM * NN;
  if (tid < nout) {
    float r = 0.f, q = 0.f;
    for (int w = 0; w < 4; ++w) {
      r += red[0][w * 64 + tid];
      q += red[1][w * 64 + tid];
    }
    part[(int64_t)blockIdx.x * nout + tid] = make_float2(r, q);
  }
}

template <int NM, typename E>
void launch_nn(int nN, dim3 g, const E* A, const E* B, float2* part, const SplitChunk& sc, hipStream_t s) {
  switch (nN) {
    case 0: hipLaunchKernelGGL((k_splitk_chunk<NM, 1, E>), g, dim3(256), 0, s, A, B, part, sc); break;
    case 1: hipLaunchKernelGGL((k_splitk_chunk<NM, 2, E>), g, dim3(256), 0, s, A, B, part, sc); break;
    case 2: hipLaunchKernelGGL((k_splitk_chunk<NM, 4, E>), g, dim3(256), 0, s, A, B, part, sc); break;
    default: hipLaunchKernelGGL((k_splitk_chunk<NM, 8, E>), g, dim3(256), 0, s, A, B, part, sc); break;
  }
}

template <typename E>
void launch_t(int nM, int nN, dim3 g, const void* A, const void* B, float2* part, const SplitChunk& sc,
              hipStream_t s) {
  const E* a = (const E*)A;
  const E* b = (const E*)B;
  switch (nM) {
    case 0: launch_nn<1, E>(nN, g, a, b, part, sc, s); break;
    case 1: launch_nn<2, E>(nN, g, a, b, part, sc, s); break;
    case 2: launch_nn<4, E>(nN, g, a, b, part, sc, s); break;
    default: launch_nn<8, E>(nN, g, a, b, part, sc, s); break;
  }
}

// Chunk map of 2^nr rows (row bit j at rpos[j]) x 2^8 k (chunk k bit i at
// kpos[i]), in address order.
bool chunk_map(const std::vector<int>& rpos, const std::vector<int>& kpos, SkewMap* mp) {
  struct Var {
    int pos, r, k;
  };
  std::vector<Var> vars;
  for (int j = 0; j < (int)rpos.size(); ++j) vars.push_back({rpos[j], j, -1});
  for (int i = 0; i < (int)kpos.size(); ++i) vars.push_back({kpos[i], -1, i});
  if ((int)vars.size() > kSkewMaxV) return false;
  for (const Var& x : vars)
    if (x.pos < 0 || x.pos >= 64) return false;
  std::sort(vars.begin(), vars.end(), [](const Var& a, const Var& b) { return a.pos < b.pos; });
  *mp = SkewMap{};
  mp->v = (int)vars.size();
  for (int i = 0; i < mp->v; ++i) {
    mp->pos[i] = (int8_t)vars[i].pos;
    mp->mb[i] = (int8_t)vars[i].r;
    mp->kb[i] = (int8_t)vars[i].k;
  }
  return true;
}

}  // namespace

bool splitk_chunk_aligned(const IndexOp& op) {
  const int l = std::min(op.nK, kSplitChunkLog2);
  auto low = [&](const Runs& r) { return r.n >= 1 && r.src[0] == 0 && r.dst[0] == 0 && r.len[0] >= l; };
  return low(op.aK) && low(op.bK);
}

hipError_t launch_splitk_chunk(int dtype, const void* A, const void* B, float2* part, const IndexOp& op,
                               int64_t* nblk, hipStream_t s) {
  if (!splitk_chunk_ok(op.nM, op.nN, op.nK)) return hipErrorInvalidValue;
  const int nK = op.nK;
  std::vector<int> pa(nK), pb(nK);
  for (int j = 0; j < nK; ++j) {
    pa[j] = run_pos(op.aK, j);
    pb[j] = run_pos(op.bK, j);
    if (pa[j] < 0 || pb[j] < 0) return hipErrorInvalidValue;
  }
  // the chunk's k bits: those below position `la` of A and `lb` of B (runs
  // of 2^la and 2^lb entries: 128 bytes when the chunk has room), then the
  // next lowest of A and B in turn up to 8
  const int eb = dtype == TN_DTYPE_C64 ? 8 : 4;
  const int want = eb == 8 ? 4 : 5;
  std::vector<int> ch;
  auto has = [&](int j) { return std::find(ch.begin(), ch.end(), j) != ch.end(); };
  auto pick = [&](int la, int lb) {
    ch.clear();
    for (int j = 0; j < nK; ++j)
      if (pa[j] < la) ch.push_back(j);
    for (int j = 0; j < nK; ++j)
      if (pb[j] < lb && !has(j)) ch.push_back(j);
    return (int)ch.size() <= kSplitChunkLog2;
  };
  if (!pick(want, want) && !pick(want, 4) && !pick(4, want) && !pick(4, 4)) return hipErrorInvalidValue;
  std::vector<int> oa(nK), ob(nK);
  for (int j = 0; j < nK; ++j) oa[j] = ob[j] = j;
  std::sort(oa.begin(), oa.end(), [&](int x, int y) { return pa[x] < pa[y]; });
  std::sort(ob.begin(), ob.end(), [&](int x, int y) { return pb[x] < pb[y]; });
  for (int ia = 0, ib = 0, side = 0; (int)ch.size() < kSplitChunkLog2; side ^= 1) {
    if (side == 0) {
      while (has(oa[ia])) ++ia;
      ch.push_back(oa[ia]);
    } else {
      while (has(ob[ib])) ++ib;
      ch.push_back(ob[ib]);
    }
  }
  SplitChunk sc{};
  std::vector<int> rpa, rpb, kpa, kpb;
  for (int j = 0; j < op.nM; ++j) rpa.push_back(run_pos(op.aM, j));
  for (int j = 0; j < op.nN; ++j) rpb.push_back(run_pos(op.bN, j));
  for (int j : ch) {
    kpa.push_back(pa[j]);
    kpb.push_back(pb[j]);
  }
  if (!chunk_map(rpa, kpa, &sc.ma) || !chunk_map(rpb, kpb, &sc.mb)) return hipErrorInvalidValue;
  // the other k bits index the chunks, in A's position order (the chunks
  // of neighbouring blocks lie close together in A)
  std::vector<int> outer_a, outer_b;
  for (int j : oa)
    if (!has(j)) {
      outer_a.push_back(pa[j]);
      outer_b.push_back(pb[j]);
    }
  sc.n_outer = (int)outer_a.size();
  if (!make_runs(outer_a, &sc.oA) || !make_runs(outer_b, &sc.oB)) return hipErrorInvalidValue;
  // 16-byte loads need the entries of one load at consecutive addresses:
  // the chunk holds each operand's lowest positions
  const int ve = 16 / eb;
  auto low_ok = [&](const SkewMap& mp, int rows) {
    const int w = std::min(ve, rows);
    for (int i = 0; (1 << i) < w; ++i)
      if (mp.pos[i] != i) return false;
    return true;
  };
  if (!low_ok(sc.ma, 1 << op.nM) || !low_ok(sc.mb, 1 << op.nN)) return hipErrorInvalidValue;
  // grid: a power of two within the partial-sum buffer (splitk_blocks) and
  // the chunk count, 512 blocks (two per CU) unless a thread's FP32 sum would
  // exceed kAccChain terms
  const int64_t chunks = (int64_t)1 << sc.n_outer;
  const int64_t cap = std::min<int64_t>(splitk_blocks(op), chunks);
  int64_t g = std::min<int64_t>(512, cap);
  while (chunks / g > kAccChain && g * 2 <= cap) g *= 2;
  if ((g & (g - 1)) != 0) return hipErrorInvalidValue;
  *nblk = g;
  const dim3 grid((unsigned)g);
  if (dtype == TN_DTYPE_F16S)
    launch_t<cf16>(op.nM, op.nN, grid, A, B, part, sc, s);
  else if (dtype == TN_DTYPE_BF16S)
    launch_t<cbf16>(op.nM, op.nN, grid, A, B, part, sc, s);
  else
    launch_t<float2>(op.nM, op.nN, grid, A, B, part, sc, s);
  return hipGetLastError();
}

}  // namespace tnrcs
