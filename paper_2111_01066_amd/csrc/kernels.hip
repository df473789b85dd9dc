// gfx950 kernels of the tnrcs library other than the GEMMs: slice binding,
// tiled binary-index permutation, gathered contraction (one output per
// thread, output tiles for short sums, or split over K for few outputs), FP64 slice accumulation with the
// numeric-range checks of scaled storage, and FP64 reductions.  Every data
// kernel is templated on the storage element: complex64, or an FP16 / BF16
// pair holding value * 2^-e for a per-tensor exponent e.
//
// Paper anchors: each pairwise contraction is an index permutation followed by
// a complex matrix product (Supplement Eq. (matmul)); slicing sums smaller
// networks (main text, customized-TNC section); XEB / Porter-Thomas checks
// (main text Eq. (fxeb)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "elem.h"
#include "kernels.h"

namespace tnrcs {

// ---------------------------------------------------------------- control --

__global__ void k_set_ctrl(Ctrl* ctrl, int64_t cursor, void* amp, int clear_flags) {
  ctrl->cursor = cursor;
  ctrl->amp = (double*)amp;
  if (clear_flags) ctrl->flags = 0u;
}

hipError_t launch_set_ctrl(Ctrl* ctrl, int64_t cursor, void* amp, hipStream_t s, bool clear_flags) {
  hipLaunchKernelGGL(k_set_ctrl, dim3(1), dim3(1), 0, s, ctrl, cursor, amp, clear_flags ? 1 : 0);
  return hipGetLastError();
}

// dst[i] += src[i] over n complex128 entries (a checked slice joins the sum).
__global__ __launch_bounds__(256) void k_add_amp(const double* __restrict__ src, double* __restrict__ dst,
                                                int64_t n2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] += src[i];
}

hipError_t launch_add_amp(const double* src, double* dst, int64_t n, hipStream_t s) {
  const int64_t n2 = 2 * n;
  hipLaunchKernelGGL(k_add_amp, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n2 + 255) / 256, 4096))),
                     dim3(256), 0, s, src, dst, n2);
  return hipGetLastError();
}

// Fills n 32-bit words with hashed pseudo-random values of the storage
// format (FP32 in [-1, 1) for complex64; two FP16 / BF16 halves of random
// sign with magnitudes in [0.5, 1) otherwise): tuning data with the power
// draw of real operands (the matrix cores run measurably faster on zeros).
__global__ __launch_bounds__(256) void k_fill_random(uint32_t* __restrict__ p, int64_t n, int kind) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t h = (uint32_t)i * 2654435761u + (uint32_t)(i >> 32);
    h ^= h >> 15;
    h *= 0x2c1b3c6du;
    h ^= h >> 12;
    h *= 0x297a2d39u;
    h ^= h >> 15;
    uint32_t w;
    if (kind == TN_DTYPE_C64) {
      w = __float_as_uint((float)(int32_t)h * 0x1p-31f);
    } else if (kind == TN_DTYPE_F16S) {
      w = ((h & 0x83FFu) | 0x3800u) | ((((h >> 16) & 0x83FFu) | 0x3800u) << 16);
    } else {
      w = ((h & 0x807Fu) | 0x3F00u) | ((((h >> 16) & 0x807Fu) | 0x3F00u) << 16);
    }
    p[i] = w;
  }
}

hipError_t launch_fill_random(void* p, int64_t bytes, int dtype, hipStream_t s) {
  const int64_t n = bytes / 4;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_random, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 16384)), dim3(256), 0, s,
                     (uint32_t*)p, n, dtype);
  return hipGetLastError();
}

// ------------------------------------------------------------------- bind --
// Copies, for every sliced leaf, the sub-tensor selected by the current slice
// id (its sliced wires are the leaf's top bits) into the bound-leaf region.

template <typename E>
__global__ __launch_bounds__(256) void k_bind(const E* __restrict__ leaves, E* __restrict__ bound,
                                              const BindDesc* __restrict__ descs, Ctrl* ctrl, int n_desc,
                                              const double2* __restrict__ kappa) {
  const BindDesc& d = descs[blockIdx.y];
  const int64_t s = ctrl->cursor;
  if (kappa && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    // product over the sliced leaves of the factor of the sub-block this slice uses
    double kr = 1.0, ki = 0.0;
    for (int i = 0; i < n_desc; ++i) {
      const BindDesc& di = descs[i];
      int64_t b = 0;
      for (int j = 0; j < di.n_sl; ++j) b |= ((s >> di.sbit[j]) & 1ll) << (di.n_sl - 1 - j);
      const double2 f = kappa[di.kappa_off + b];
      const double t = kr * f.x - ki * f.y;
      ki = kr * f.y + ki * f.x;
      kr = t;
    }
    ctrl->kap_re = kr;
    ctrl->kap_im = ki;
  }
  int64_t off = 0;
  for (int i = 0; i < d.n_sl; ++i) off |= ((s >> d.sbit[i]) & 1ll) << d.pos[i];
  const E* src = leaves + d.src_off + off;
  E* dst = bound + d.dst_off;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < d.n_elems;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

hipError_t launch_bind(int elem_bytes, const void* leaves, void* bound, const BindDesc* descs, int n_desc,
                       int64_t max_elems, Ctrl* ctrl, const double2* kappa, hipStream_t s) {
  if (n_desc <= 0) return hipSuccess;
  const int64_t gx = std::max<int64_t>(std::min<int64_t>((max_elems + 255) / 256, 1024), 1);
  const dim3 g((unsigned)gx, n_desc);
  if (elem_bytes == 8)
    hipLaunchKernelGGL(k_bind<float2>, g, dim3(256), 0, s, (const float2*)leaves, (float2*)bound, descs, ctrl, n_desc,
                       kappa);
  else
    hipLaunchKernelGGL(k_bind<uint32_t>, g, dim3(256), 0, s, (const uint32_t*)leaves, (uint32_t*)bound, descs,
                       ctrl, n_desc, kappa);
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

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Both global sides move 16-byte groups of G = 16 / sizeof(E) adjacent
// elements: input positions 0..log2(G)-1 and output positions 0..log2(G)-1
// are always in the tile, so a group is adjacent in memory on the read side
// (in e order) and on the write side (in f order).  LDS padding of G
// elements per 32 keeps groups adjacent and 16-byte aligned while spreading
// power-of-two strides over the banks.
template <int G>
__device__ __forceinline__ int lds_pad(int e) {
  return e + (e >> 5) * G;
}

// Tile of 2^TB elements (up to 2^12 complex64 or 2^13 four-byte elements,
// 32 KB either way), 256 threads, 2^TB / 256 elements per thread.  All of
// a thread's loads are issued before any LDS store so they are in flight
// together, and the next tile's loads are issued before the current tile
// is read back from LDS and written out, so they overlap; the writes are
// streaming (non-temporal) stores.  The parts of the offsets that depend
// only on the unrolled iteration are tabulated once in LDS; the tile-id
// parts are updated by one XOR per tile, so the loop does no bit-deposit
// walks.
// Past the last tile the prefetch repeats the last tile (read and staged,
// never written out).
template <int TB, typename E>
__global__ __launch_bounds__(kPermThreads) void k_permute(const E* __restrict__ in, E* __restrict__ out,
                                                         const PermArgs a) {
  constexpr int G = 16 / sizeof(E);
  constexpr int NT = 1 << TB;
  constexpr int PG = NT / kPermThreads / G;  // groups per thread
  __shared__ __attribute__((aligned(16))) E tile[NT + (NT / 32) * G];
  __shared__ uint64_t hi_in[PG], hi_out[PG];
  __shared__ int hi_fe[PG];
  __shared__ int fe_low[G];
  const int tid = threadIdx.x;
  if (tid < PG) {
    hi_in[tid] = dep((uint64_t)tid * G * kPermThreads, a.in_tile);
    hi_out[tid] = dep((uint64_t)tid * G * kPermThreads, a.out_tile);
    hi_fe[tid] = (int)dep((uint64_t)tid * G * kPermThreads, a.f2e);
  }
  if (tid < G) fe_low[tid] = (int)dep((uint64_t)tid, a.f2e);
  const E* src = in + (int64_t)blockIdx.y * a.stride;
  E* dst = out + (int64_t)blockIdx.y * a.stride;
  const uint64_t e_t = dep((uint64_t)tid * G, a.in_tile);
  const uint64_t f_t = dep((uint64_t)tid * G, a.out_tile);
  const int fe_t = (int)dep((uint64_t)tid * G, a.f2e);
  // tile-id parts of the offsets.  Block b takes tiles t_i = b + i P (P =
  // gridDim.x, a power of two like the tile count), so dep(t_i) = dep(b) XOR
  // dep(i P), and from i to i + 1 the bits 0..ctz(i + 1) of i flip: the
  // offsets move by one XOR with a prefix table of dep(2^j P) (the tile-id
  // map need not preserve bit order, so no carrying add)
  __shared__ uint64_t pre_in[40], pre_out[40];
  const int lg = __builtin_ctzll((unsigned long long)gridDim.x);
  const int nb = __builtin_ctzll((unsigned long long)a.n_tiles) - lg;  // bits of the iteration index
  if (tid < nb) {
    uint64_t xi = 0, xo = 0;
    for (int j = 0; j <= tid; ++j) {
      xi ^= dep((uint64_t)1 << (lg + j), a.id_in);
      xo ^= dep((uint64_t)1 << (lg + j), a.id_out);
    }
    pre_in[tid] = xi;
    pre_out[tid] = xo;
  }
  const uint64_t din = dep((uint64_t)blockIdx.x, a.id_in);
  uint64_t dout = dep((uint64_t)blockIdx.x, a.id_out);
  const int64_t my_tiles = a.n_tiles > (int64_t)blockIdx.x ? (a.n_tiles - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
  __syncthreads();
  int fl[G];
#pragma unroll
  for (int g = 0; g < G; ++g) fl[g] = fe_low[g];
  uint64_t pf_in = din;  // input offset of the tile being prefetched
  int64_t pf_i = 0;      // its iteration index
  u32x4 v[PG];
  auto load_tile = [&]() {
    const uint64_t ib = pf_in | e_t;
#pragma unroll
    for (int i = 0; i < PG; ++i) v[i] = *reinterpret_cast<const u32x4*>(src + (ib | hi_in[i]));
    if (pf_i + 1 < my_tiles) {
      ++pf_i;
      pf_in ^= pre_in[__builtin_ctzll((unsigned long long)pf_i)];
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int i = 0; i < PG; ++i) *reinterpret_cast<u32x4*>(&tile[lds_pad<G>(G * (i * kPermThreads + tid))]) = v[i];
  };
  if (my_tiles > 0) {
    load_tile();
    stage();
    __syncthreads();
    load_tile();
  }
  // per tile: write out the staged tile, then stage the prefetched one and
  // prefetch the next: the wait for the prefetched loads comes after this
  // tile's stores in every iteration, so the stores may still be in flight
  for (int64_t i_t = 0; i_t < my_tiles; ++i_t) {
    const uint64_t ob = dout | f_t;
#pragma unroll
    for (int i = 0; i < PG; ++i) {
      const int e0 = fe_t | hi_fe[i];
      E w[G];
#pragma unroll
      for (int g = 0; g < G; ++g) w[g] = tile[lds_pad<G>(e0 | fl[g])];
      u32x4 x;
      __builtin_memcpy(&x, w, 16);
      __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(dst + (ob | hi_out[i])));
    }
    if (i_t + 1 < my_tiles) dout ^= pre_out[__builtin_ctzll((unsigned long long)(i_t + 1))];
    __syncthreads();
    stage();
    __syncthreads();
    load_tile();
  }
}

// Tensors below 256 elements: one element per thread, direct gather.
template <typename E>
__global__ __launch_bounds__(256) void k_permute_small(const E* __restrict__ in, E* __restrict__ out,
                                                      const PermArgs a) {
  const int64_t n = (int64_t)1 << a.tbits;
  const E* src = in + (int64_t)blockIdx.y * a.stride;
  E* dst = out + (int64_t)blockIdx.y * a.stride;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) dst[dep((uint64_t)e, a.out_tile)] = src[dep((uint64_t)e, a.f2e)];
}

template <typename E>
static void launch_perm_tb(int tb, dim3 g, const E* in, E* out, const PermArgs& A, hipStream_t s) {
  switch (tb) {
    case 10:
      hipLaunchKernelGGL((k_permute<10, E>), g, dim3(kPermThreads), 0, s, in, out, A);
      break;
    case 11:
      hipLaunchKernelGGL((k_permute<11, E>), g, dim3(kPermThreads), 0, s, in, out, A);
      break;
    case 12:
      hipLaunchKernelGGL((k_permute<12, E>), g, dim3(kPermThreads), 0, s, in, out, A);
      break;
    default:
      if constexpr (sizeof(E) == 4) hipLaunchKernelGGL((k_permute<13, E>), g, dim3(kPermThreads), 0, s, in, out, A);
      break;
  }
}

hipError_t launch_permute(int elem_bytes, const void* in, void* out, int rank, const int32_t* perm, int64_t batch,
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
  if (rank < 10) {
    // out index f: output position q holds input bit perm[q]
    std::vector<int> po, pi;
    for (int q = 0; q < rank; ++q) po.push_back(q);
    for (int q = 0; q < rank; ++q) pi.push_back(perm[q]);
    A.tbits = rank;
    A.n_tiles = 1;
    if (!make_runs(po, &A.out_tile) || !make_runs(pi, &A.f2e)) return hipErrorInvalidValue;
    if (elem_bytes == 8)
      hipLaunchKernelGGL(k_permute_small<float2>, dim3(1, (unsigned)batch), dim3(256), 0, s, (const float2*)in,
                         (float2*)out, A);
    else
      hipLaunchKernelGGL(k_permute_small<uint32_t>, dim3(1, (unsigned)batch), dim3(256), 0, s,
                         (const uint32_t*)in, (uint32_t*)out, A);
    return hipGetLastError();
  }
  // choose the tile: grow input-fast and output-fast bit sets alternately
  std::vector<bool> inT(rank, false);
  int tb = 0, a = 0, b = 0;
  const int cap = std::min(elem_bytes == 4 ? kPermTileBits + 1 : kPermTileBits, rank);
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
  if (A.tbits < 10 || A.tbits > (elem_bytes == 4 ? kPermTileBits + 1 : kPermTileBits)) return hipErrorInvalidValue;
  const int64_t grid = std::min<int64_t>(A.n_tiles, 16384);
  const dim3 g((unsigned)grid, (unsigned)batch);
  if (elem_bytes == 8)
    launch_perm_tb<float2>(A.tbits, g, (const float2*)in, (float2*)out, A, s);
  else
    launch_perm_tb<uint32_t>(A.tbits, g, (const uint32_t*)in, (uint32_t*)out, A, s);
  return hipGetLastError();
}

// ---------------------------------------------------------------- generic --
// One output element per thread: C[(m<<nN)|n] = sum_k A[dep(m)|dep(k)] B[dep(n)|dep(k)],
// accumulated in FP32, multiplied by the op's output scale before storage.
// The K offsets of both operands are tabulated once per block in LDS for the
// low kTabBits bits of k (dep is additive over disjoint bit ranges), so the
// inner loop is two LDS reads and two gathered loads per term.

constexpr int kTabBits = 10;

template <typename E>
__global__ __launch_bounds__(256) void k_generic(const E* __restrict__ A, const E* __restrict__ B,
                                                E* __restrict__ C, const IndexOp op, float* maxslot) {
  __shared__ uint64_t atab[1 << kTabBits], btab[1 << kTabBits];
  const int lo_bits = op.nK < kTabBits ? op.nK : kTabBits;
  const int n_lo = 1 << lo_bits;
  for (int k = threadIdx.x; k < n_lo; k += blockDim.x) {
    atab[k] = dep((uint64_t)k, op.aK);
    btab[k] = dep((uint64_t)k, op.bK);
  }
  __syncthreads();
  const int64_t nC = (int64_t)1 << (op.nM + op.nN);
  const int64_t n_hi = (int64_t)1 << (op.nK - lo_bits);
  const uint64_t nmask = (1ull << op.nN) - 1ull;
  float mx = 0.f;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nC; c += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t m = (uint64_t)c >> op.nN, n = (uint64_t)c & nmask;
    const uint64_t ab = dep(m, op.aM), bb = dep(n, op.bN);
    // runs of at most 2^kTabBits terms per FP32 chain, added to the total
    float re = 0.f, im = 0.f;
    for (int64_t h = 0; h < n_hi; ++h) {
      const uint64_t ah = ab | dep((uint64_t)h << lo_bits, op.aK), bh = bb | dep((uint64_t)h << lo_bits, op.bK);
      float pr = 0.f, pi = 0.f;
      for (int k = 0; k < n_lo; ++k) {
        const float2 x = to_f2(A[ah | atab[k]]);
        const float2 y = to_f2(B[bh | btab[k]]);
        pr = fmaf(x.x, y.x, pr);
        pr = fmaf(-x.y, y.y, pr);
        pi = fmaf(x.x, y.y, pi);
        pi = fmaf(x.y, y.x, pi);
      }
      re += pr;
      im += pi;
    }
    mx = mag_max(mx, re, im);
    C[c] = from_f2<E>(re * op.out_scale, im * op.out_scale);
  }
  record_max(maxslot, mx);
}

// Short sums into many outputs (2^nM, 2^nN >= 64, 2^nK <= 16): a workgroup
// owns a 64 x 64 output tile, gathers the tile's A rows (64 x 2^nK) and B
// rows once into LDS in FP32, and each thread accumulates a 4 x 4 block of
// outputs from LDS; 16 consecutive threads write 16 consecutive n of a row.
template <typename E>
__global__ __launch_bounds__(256) void k_generic_tiled(const E* __restrict__ A, const E* __restrict__ B,
                                                      E* __restrict__ C, const IndexOp op, float* maxslot) {
  __shared__ float2 As[16][65], Bs[16][65];  // [k][m], [k][n]
  const int nk = 1 << op.nK;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t tiles_n = (int64_t)1 << (op.nN - 6), tiles = (int64_t)1 << (op.nM + op.nN - 12);
  float mx = 0.f;
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int64_t m0 = (t / tiles_n) << 6, n0 = (t % tiles_n) << 6;
    for (int i = tid; i < 64 * nk; i += 256) {
      const int k = i >> 6, r = i & 63;
      const uint64_t ak = dep((uint64_t)k, op.aK), bk = dep((uint64_t)k, op.bK);
      As[k][r] = to_f2(A[dep((uint64_t)(m0 + r), op.aM) | ak]);
      Bs[k][r] = to_f2(B[dep((uint64_t)(n0 + r), op.bN) | bk]);
    }
    __syncthreads();
    float re[4][4], im[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) re[i][j] = im[i][j] = 0.f;
    for (int k = 0; k < nk; ++k) {
      float2 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          re[i][j] = fmaf(a[i].x, b[j].x, re[i][j]);
          re[i][j] = fmaf(-a[i].y, b[j].y, re[i][j]);
          im[i][j] = fmaf(a[i].x, b[j].y, im[i][j]);
          im[i][j] = fmaf(a[i].y, b[j].x, im[i][j]);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        mx = mag_max(mx, re[i][j], im[i][j]);
        const int64_t c = ((m0 + ty + 16 * i) << op.nN) | (n0 + tx + 16 * j);
        C[c] = from_f2<E>(re[i][j] * op.out_scale, im[i][j] * op.out_scale);
      }
    __syncthreads();
  }
  record_max(maxslot, mx);
}

hipError_t launch_generic(int dtype, const void* A, const void* B, void* C, const IndexOp& op, float* maxslot,
                          hipStream_t s) {
  if (op.nM >= 6 && op.nN >= 6 && op.nK <= 4) {
    const dim3 g((unsigned)std::min<int64_t>((int64_t)1 << (op.nM + op.nN - 12), 16384));
    if (dtype == TN_DTYPE_F16S)
      hipLaunchKernelGGL(k_generic_tiled<cf16>, g, dim3(256), 0, s, (const cf16*)A, (const cf16*)B, (cf16*)C, op,
                         maxslot);
    else if (dtype == TN_DTYPE_BF16S)
      hipLaunchKernelGGL(k_generic_tiled<cbf16>, g, dim3(256), 0, s, (const cbf16*)A, (const cbf16*)B, (cbf16*)C, op,
                         maxslot);
    else
      hipLaunchKernelGGL(k_generic_tiled<float2>, g, dim3(256), 0, s, (const float2*)A, (const float2*)B,
                         (float2*)C, op, maxslot);
    return hipGetLastError();
  }
  const int64_t nC = (int64_t)1 << (op.nM + op.nN);
  const int64_t grid = std::min<int64_t>((nC + 255) / 256, 16384);
  const dim3 g((unsigned)grid);
  if (dtype == TN_DTYPE_F16S)
    hipLaunchKernelGGL(k_generic<cf16>, g, dim3(256), 0, s, (const cf16*)A, (const cf16*)B, (cf16*)C, op, maxslot);
  else if (dtype == TN_DTYPE_BF16S)
    hipLaunchKernelGGL(k_generic<cbf16>, g, dim3(256), 0, s, (const cbf16*)A, (const cbf16*)B, (cbf16*)C, op,
                       maxslot);
  else
    hipLaunchKernelGGL(k_generic<float2>, g, dim3(256), 0, s, (const float2*)A, (const float2*)B, (float2*)C, op,
                       maxslot);
  return hipGetLastError();
}

// ----------------------------------------------------------------- skinny --
// Skewed contraction (M large, N and K small; Supplement, CPU-architecture
// section: the small operand stays in fast local memory and the large one is
// read once): B (2^(nK+nN) <= 2048 entries) and A's K offsets are kept in
// LDS; each thread owns whole rows m (2^nN outputs in registers), A is read
// once and C written once, both through coalesced accesses where the layout
// allows.

typedef unsigned int row_u32x4 __attribute__((ext_vector_type(4)));

// Each pass of a workgroup covers 256 R consecutive m (R per thread, at
// stride 256), whose C rows form one contiguous run of 256 R NN entries: the
// outputs are staged in LDS and written back in coalesced 16-byte
// nontemporal stores.  NK > 0: A's layout is [M bits, K bits] in order
// (nK = log2(NK)), so the pass's A rows are one contiguous run as well,
// loaded the same way; NK == 0: any layout, each thread gathers its rows
// through the offset table (consecutive m are adjacent in A wherever A's
// low bits are M bits).  R > 1 keeps more loads in flight per thread.
template <int NN, int NK, int R, typename E>
__global__ __launch_bounds__(256) void k_skinny(const E* __restrict__ A, const E* __restrict__ B, E* __restrict__ C,
                                               const IndexOp op, float* maxslot) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  constexpr int PM = 256 * R;  // rows per pass
  const int nk = NK > 0 ? NK : 1 << op.nK;
  E* sC = reinterpret_cast<E*>(smem);                          // [PM][NN]
  E* sA = sC + PM * NN;                                        // [PM][NK] (NK > 0)
  float2* Bs = reinterpret_cast<float2*>(sA + PM * NK);        // [nk][NN]
  uint64_t* kofs = reinterpret_cast<uint64_t*>(Bs + nk * NN);  // [nk] (NK == 0)
  for (int i = threadIdx.x; i < nk * NN; i += blockDim.x) {
    const int k = i / NN, n = i % NN;
    Bs[i] = to_f2(B[dep((uint64_t)n, op.bN) | dep((uint64_t)k, op.bK)]);
  }
  if (NK == 0)
    for (int k = threadIdx.x; k < nk; k += blockDim.x) kofs[k] = dep((uint64_t)k, op.aK);
  __syncthreads();
  const int tid = threadIdx.x;
  const int64_t nm = (int64_t)1 << op.nM;  // a multiple of PM
  // row offsets dep(m0 + r 256 + tid) = dep(m0) | dep(r 256 + tid): the
  // first part advanced in the deposited domain per pass, the second fixed
  uint64_t am_t[R];
#pragma unroll
  for (int r = 0; r < R; ++r) am_t[r] = dep((uint64_t)(r * 256 + tid), op.aM);
  const uint64_t mask_m = dep((uint64_t)(nm - PM), op.aM);
  const uint64_t inc_m = dep((uint64_t)gridDim.x * PM, op.aM);
  uint64_t am0 = dep((uint64_t)blockIdx.x * PM, op.aM);
  float mx = 0.f;
  for (int64_t m0 = (int64_t)blockIdx.x * PM; m0 < nm;
       m0 += (int64_t)gridDim.x * PM, am0 = ((am0 | ~mask_m) + inc_m) & mask_m) {
    float re[R][NN], im[R][NN];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int n = 0; n < NN; ++n) re[r][n] = im[r][n] = 0.f;
    auto madd = [&](int r, const float2 x, int k) {
      const float2* b = Bs + k * NN;
#pragma unroll
      for (int n = 0; n < NN; ++n) {
        const float2 y = b[n];
        re[r][n] = fmaf(x.x, y.x, re[r][n]);
        re[r][n] = fmaf(-x.y, y.y, re[r][n]);
        im[r][n] = fmaf(x.x, y.y, im[r][n]);
        im[r][n] = fmaf(x.y, y.x, im[r][n]);
      }
    };
    if constexpr (NK > 0) {
      constexpr int CH = PM * NK * (int)sizeof(E) / 16;  // 16-byte chunks of the pass's A rows
      const row_u32x4* src = reinterpret_cast<const row_u32x4*>(A + (m0 << op.nK));
      row_u32x4 v[(CH + 255) / 256];
#pragma unroll
      for (int i = 0; i < (CH + 255) / 256; ++i) {
        const int c = i * 256 + tid;
        if (CH % 256 == 0 || c < CH) v[i] = src[c];
      }
#pragma unroll
      for (int i = 0; i < (CH + 255) / 256; ++i) {
        const int c = i * 256 + tid;
        if (CH % 256 == 0 || c < CH) reinterpret_cast<row_u32x4*>(sA)[c] = v[i];
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < NK; ++k) madd(r, to_f2(sA[(r * 256 + tid) * NK + k]), k);
    } else {
      uint64_t am[R];
#pragma unroll
      for (int r = 0; r < R; ++r) am[r] = am0 | am_t[r];
      for (int k = 0; k < nk; ++k) {
        float2 x[R];
#pragma unroll
        for (int r = 0; r < R; ++r) x[r] = to_f2(A[am[r] | kofs[k]]);
#pragma unroll
        for (int r = 0; r < R; ++r) madd(r, x[r], k);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int n = 0; n < NN; ++n) {
        mx = mag_max(mx, re[r][n], im[r][n]);
        sC[(r * 256 + tid) * NN + n] = from_f2<E>(re[r][n] * op.out_scale, im[r][n] * op.out_scale);
      }
    __syncthreads();
    constexpr int CC = PM * NN * (int)sizeof(E) / 16;  // 16-byte chunks of the pass's C rows
    row_u32x4* dst = reinterpret_cast<row_u32x4*>(C + m0 * NN);
#pragma unroll
    for (int i = 0; i < (CC + 255) / 256; ++i) {
      const int c = i * 256 + tid;
      if (CC % 256 == 0 || c < CC) __builtin_nontemporal_store(reinterpret_cast<const row_u32x4*>(sC)[c], dst + c);
    }
    __syncthreads();
  }
  record_max_in(maxslot, mx, reinterpret_cast<float*>(smem));
}

// LDS of one workgroup: staged C rows, staged A rows (a_rows: A's layout is
// [M bits, K bits]), B as FP32 pairs and A's K offsets; pm rows per pass.
size_t skinny_lds_bytes(const IndexOp& op, int elem_bytes, bool a_rows, int pm) {
  const size_t nk = (size_t)1 << op.nK, nn = (size_t)1 << op.nN;
  return pm * nn * elem_bytes + (a_rows ? pm * nk * elem_bytes : 0) + nk * nn * sizeof(float2) +
         (a_rows ? 0 : nk * sizeof(uint64_t));
}

// Rows per thread and pass: the most of 4, 2, 1 whose staged rows fit in
// 32 KB, so that with B and the offset table (at most 32 KB) a workgroup
// stays within 64 KB of LDS.  A tensor with fewer rows than one such pass
// uses 1.
template <int NN, int NK, typename E>
constexpr int skinny_rows() {
  constexpr int row = (NN + NK) * (int)sizeof(E);
  return 1024 * row <= 32768 ? 4 : (512 * row <= 32768 ? 2 : 1);
}

template <int NN, int NK, typename E>
static void launch_skinny_k(const E* A, const E* B, E* C, const IndexOp& op, float* maxslot, hipStream_t s) {
  constexpr int RX = skinny_rows<NN, NK, E>();
  const int64_t nm = (int64_t)1 << op.nM;
  const bool wide = RX > 1 && nm >= 256 * RX;
  const int pm = wide ? 256 * RX : 256;
  const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>(nm / pm, 8192)));
  const size_t lds = skinny_lds_bytes(op, (int)sizeof(E), NK > 0, pm);
  if (wide)
    hipLaunchKernelGGL((k_skinny<NN, NK, RX, E>), g, dim3(256), lds, s, A, B, C, op, maxslot);
  else
    hipLaunchKernelGGL((k_skinny<NN, NK, 1, E>), g, dim3(256), lds, s, A, B, C, op, maxslot);
}

template <int NN, typename E>
static void launch_skinny_nn(const E* A, const E* B, E* C, const IndexOp& op, float* maxslot, hipStream_t s) {
  // A's layout is [M bits, K bits], both in order: contiguous rows
  const bool rows = op.aK.n == 1 && op.aK.src[0] == 0 && op.aK.dst[0] == 0 && op.aK.len[0] == op.nK &&
                    op.aM.n == 1 && op.aM.src[0] == 0 && op.aM.dst[0] == op.nK && op.aM.len[0] == op.nM;
  if (rows && op.nK == 1)
    launch_skinny_k<NN, 2>(A, B, C, op, maxslot, s);
  else if (rows && op.nK == 2)
    launch_skinny_k<NN, 4>(A, B, C, op, maxslot, s);
  else if (rows && op.nK == 3)
    launch_skinny_k<NN, 8>(A, B, C, op, maxslot, s);
  else
    launch_skinny_k<NN, 0>(A, B, C, op, maxslot, s);
}

template <typename E>
static hipError_t launch_skinny_t(const E* A, const E* B, E* C, const IndexOp& op, float* maxslot, hipStream_t s) {
  if (op.nM < 8) return hipErrorInvalidValue;  // whole 256-row passes
  switch (op.nN) {
    case 0: launch_skinny_nn<1>(A, B, C, op, maxslot, s); break;
    case 1: launch_skinny_nn<2>(A, B, C, op, maxslot, s); break;
    case 2: launch_skinny_nn<4>(A, B, C, op, maxslot, s); break;
    case 3: launch_skinny_nn<8>(A, B, C, op, maxslot, s); break;
    case 4: launch_skinny_nn<16>(A, B, C, op, maxslot, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_skinny(int dtype, const void* A, const void* B, void* C, const IndexOp& op, float* maxslot,
                         hipStream_t s) {
  if (op.nN > 4 || op.nK + op.nN > kSkinnyMaxLog2) return hipErrorInvalidValue;
  if (dtype == TN_DTYPE_F16S) return launch_skinny_t<cf16>((const cf16*)A, (const cf16*)B, (cf16*)C, op, maxslot, s);
  if (dtype == TN_DTYPE_BF16S)
    return launch_skinny_t<cbf16>((const cbf16*)A, (const cbf16*)B, (cbf16*)C, op, maxslot, s);
  return launch_skinny_t<float2>((const float2*)A, (const float2*)B, (float2*)C, op, maxslot, s);
}

// ---------------------------------------------------------------- split-K --
// Few outputs (<= 64) and a long contraction: the K range is split over a
// fixed grid; each thread accumulates all outputs over its k's (consecutive
// threads take consecutive k, so the gathers are coalesced wherever the low
// K bits are the operands' low bits), the block reduces in LDS, and one
// block sums the FP32 per-block partials in a fixed order.

// VK consecutive entries starting at p (VK > 1: one 16-byte load).
template <int VK, typename E>
__device__ __forceinline__ void load_run(const E* p, float2 (&out)[VK]) {
  if constexpr (VK == 1) {
    out[0] = to_f2(*p);
  } else {
    static_assert(VK * sizeof(E) == 16, "one 16-byte load");
    const row_u32x4 w = *reinterpret_cast<const row_u32x4*>(p);
    E v[VK];
    __builtin_memcpy(v, &w, 16);
#pragma unroll
    for (int i = 0; i < VK; ++i) out[i] = to_f2(v[i]);
  }
}

// VK > 1: each thread takes VK consecutive k per step (both operands' lowest
// log2(VK) k bits are their lowest bits, in order), read in 16-byte loads.
// Groups (more than 64 outputs): blockIdx.y = group (im, in) of 2^op.nM x
// 2^op.nN outputs, whose A and B start at dep(im << op.nM, gA) and
// dep(in << op.nN, gB) (the full maps); 2^gn_bits groups along n.  Block
// partials go to part[(group * gridDim.x + block) * nout + output].
struct SplitGroups {
  Runs gA, gB;
  int32_t gn_bits = 0;
};

template <int NN, int VK, typename E>
__global__ __launch_bounds__(256) void k_splitk_part(const E* __restrict__ A, const E* __restrict__ B,
                                                    float2* __restrict__ part, const IndexOp op,
                                                    const SplitGroups gr) {
  // outputs (m, n): m < nm = 2^nM <= 64 / NN, n < NN = 2^nN; each k loads
  // every A entry (one per m) and every B entry (one per n) once
  constexpr int NM = 64 / NN;
  __shared__ uint64_t am[NM], bn[NN];
  __shared__ float red[2][256];
  const int nm = 1 << op.nM;
  const int tid = threadIdx.x;
  {
    const uint64_t grp = blockIdx.y;
    A += dep((grp >> gr.gn_bits) << op.nM, gr.gA);
    B += dep((grp & ((1ull << gr.gn_bits) - 1)) << op.nN, gr.gB);
    part += (int64_t)blockIdx.y * gridDim.x * (nm * NN);
  }
  if (tid < nm) am[tid] = dep((uint64_t)tid, op.aM);
  if (tid < NN) bn[tid] = dep((uint64_t)tid, op.bN);
  __syncthreads();
  float acc_r[NM][NN], acc_i[NM][NN];
#pragma unroll
  for (int i = 0; i < NM; ++i)
#pragma unroll
    for (int j = 0; j < NN; ++j) acc_r[i][j] = acc_i[i][j] = 0.f;
  auto madd = [&](int i, int j, const float2 x, const float2 y) {
    acc_r[i][j] = fmaf(x.x, y.x, acc_r[i][j]);
    acc_r[i][j] = fmaf(-x.y, y.y, acc_r[i][j]);
    acc_i[i][j] = fmaf(x.x, y.y, acc_i[i][j]);
    acc_i[i][j] = fmaf(x.y, y.x, acc_i[i][j]);
  };
  const int64_t nK = (int64_t)1 << op.nK;
  for (int64_t k = ((int64_t)blockIdx.x * 256 + tid) * VK; k < nK; k += (int64_t)gridDim.x * 256 * VK) {
    const uint64_t ak = dep((uint64_t)k, op.aK), bk = dep((uint64_t)k, op.bK);
    if constexpr (NN <= 8) {  // keep the B entries, stream the A entries
      float2 y[NN][VK];
#pragma unroll
      for (int j = 0; j < NN; ++j) load_run<VK>(B + (bn[j] | bk), y[j]);
#pragma unroll
      for (int i = 0; i < NM; ++i) {
        if (i < nm) {  // uniform across the grid
          float2 x[VK];
          load_run<VK>(A + (am[i] | ak), x);
#pragma unroll
          for (int v = 0; v < VK; ++v)
#pragma unroll
            for (int j = 0; j < NN; ++j) madd(i, j, x[v], y[j][v]);
        }
      }
    } else {  // few m (NM <= 4): keep the A entries, stream the B entries
      float2 x[NM][VK];
#pragma unroll
      for (int i = 0; i < NM; ++i) {
        if (i < nm) {
          load_run<VK>(A + (am[i] | ak), x[i]);
        } else {
#pragma unroll
          for (int v = 0; v < VK; ++v) x[i][v] = make_float2(0.f, 0.f);
        }
      }
#pragma unroll
      for (int j = 0; j < NN; ++j) {
        float2 y[VK];
        load_run<VK>(B + (bn[j] | bk), y);
#pragma unroll
        for (int v = 0; v < VK; ++v)
#pragma unroll
          for (int i = 0; i < NM; ++i) madd(i, j, x[i][v], y[v]);
      }
    }
  }
  // block sum in a fixed order: butterfly within each wave, then the four
  // wave sums in wave order (one barrier for all outputs)
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    if (i < nm) {
#pragma unroll
      for (int j = 0; j < NN; ++j) {
        float r = acc_r[i][j], q = acc_i[i][j];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          r += __shfl_xor(r, o);
          q += __shfl_xor(q, o);
        }
        if (lane == 0) {
          red[0][wave * 64 + i * NN + j] = r;
          red[1][wave * 64 + i * NN + j] = q;
        }
      }
    }
  }
  __syncthreads();
  const int nout = nm * NN;
  if (tid < nout) {
    float r = 0.f, q = 0.f;
    for (int w = 0; w < 4; ++w) {
      r += red[0][w * 64 + tid];
      q += red[1][w * 64 + tid];
    }
    part[(int64_t)blockIdx.x * nout + tid] = make_float2(r, q);
  }
}

template <typename E>
__global__ __launch_bounds__(256) void k_splitk_final(const float2* __restrict__ part, int nblk, int nout,
                                                     E* __restrict__ C, float out_scale, float* maxslot, int ln_sub,
                                                     int ln_row, int lm_sub, int gn_bits) {
  __shared__ float red[2][256];
  const int tid = threadIdx.x;
  float mx = 0.f;
  {
    // group blockIdx.x = (im, in): its block partials, and its outputs'
    // first row and column in C
    const int64_t grp = blockIdx.x;
    part += grp * nblk * nout;
    const int64_t im = grp >> gn_bits, in = grp & ((1 << gn_bits) - 1);
    C += ((im << lm_sub) << ln_row) | (in << ln_sub);
  }
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
    if (tid == 0) {
      mx = mag_max(mx, red[0][0], red[1][0]);
      // output o = (i, j) of the group (j < 2^ln_sub) sits at row i, column j
      // of C, whose rows hold 2^ln_row entries
      C[((int64_t)(o >> ln_sub) << ln_row) | (o & ((1 << ln_sub) - 1))] =
          from_f2<E>(red[0][0] * out_scale, red[1][0] * out_scale);
    }
    __syncthreads();
  }
  record_max(maxslot, mx);
}

int64_t splitk_blocks(const IndexOp& op) { return splitk_grid(op.nK); }

template <int VK, typename E>
static void launch_splitk_v(const E* A, const E* B, float2* part, const IndexOp& op, const SplitGroups& gr,
                            dim3 grid, hipStream_t s) {
  const dim3 blk(256);
  switch (op.nN) {
    case 0: hipLaunchKernelGGL((k_splitk_part<1, VK, E>), grid, blk, 0, s, A, B, part, op, gr); break;
    case 1: hipLaunchKernelGGL((k_splitk_part<2, VK, E>), grid, blk, 0, s, A, B, part, op, gr); break;
    case 2: hipLaunchKernelGGL((k_splitk_part<4, VK, E>), grid, blk, 0, s, A, B, part, op, gr); break;
    case 3: hipLaunchKernelGGL((k_splitk_part<8, VK, E>), grid, blk, 0, s, A, B, part, op, gr); break;
    case 4: hipLaunchKernelGGL((k_splitk_part<16, VK, E>), grid, blk, 0, s, A, B, part, op, gr); break;
    case 5: hipLaunchKernelGGL((k_splitk_part<32, VK, E>), grid, blk, 0, s, A, B, part, op, gr); break;
    default: hipLaunchKernelGGL((k_splitk_part<64, VK, E>), grid, blk, 0, s, A, B, part, op, gr); break;
  }
}

// The map of value bits 0 .. bits-1 only.
static Runs low_runs(const Runs& r, int bits) {
  Runs o{};
  for (int i = 0; i < r.n; ++i) {
    if (r.src[i] >= bits) continue;
    o.src[o.n] = r.src[i];
    o.dst[o.n] = r.dst[i];
    o.len[o.n] = (int8_t)std::min<int>(r.len[i], bits - r.src[i]);
    ++o.n;
  }
  return o;
}

template <typename E>
static hipError_t launch_splitk_t(int dtype, const E* A, const E* B, E* C, float2* part, const IndexOp& op,
                                  float* maxslot, hipStream_t s) {
  // at most 8 x 8 outputs and an operand whose low k bits are not its low
  // bits: both operands are read in place, chunk by chunk
  if (splitk_chunk_ok(op.nM, op.nN, op.nK) && !splitk_chunk_aligned(op)) {
    int64_t nb = 0;
    const hipError_t e = launch_splitk_chunk(dtype, A, B, part, op, &nb, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_splitk_final<E>, dim3(1), dim3(256), 0, s, part, (int)nb, 1 << (op.nM + op.nN), C,
                       op.out_scale, maxslot, op.nN, op.nN, op.nM, 0);
    return hipSuccess;
  }
  const int64_t g = splitk_blocks(op);
  // 16-byte runs of k when both operands hold their lowest k bits lowest
  constexpr int VK = 16 / (int)sizeof(E), LV = VK == 4 ? 2 : 1;
  auto low = [&](const Runs& r) { return r.n >= 1 && r.src[0] == 0 && r.dst[0] == 0 && r.len[0] >= LV; };
  const bool vec = op.nK >= LV && low(op.aK) && low(op.bK);
  // more than 64 outputs: groups of 2^gm x 2^gn2 = 64 outputs (rows m and
  // columns n of C), all in one launch (blockIdx.y), each re-reading its
  // rows of A and B
  const int gn = std::min(op.nN, 3), gm = std::min(op.nM, 6 - gn);
  const int gn2 = std::min(op.nN, 6 - gm);
  IndexOp sub = op;
  sub.nM = gm;
  sub.nN = gn2;
  sub.aM = low_runs(op.aM, gm);
  sub.bN = low_runs(op.bN, gn2);
  SplitGroups gr;
  gr.gA = op.aM;
  gr.gB = op.bN;
  gr.gn_bits = op.nN - gn2;
  const int nout = 1 << (gm + gn2);
  const unsigned groups = 1u << (op.nM - gm + op.nN - gn2);
  const dim3 grid((unsigned)g, groups);
  if (vec)
    launch_splitk_v<VK>(A, B, part, sub, gr, grid, s);
  else
    launch_splitk_v<1>(A, B, part, sub, gr, grid, s);
  hipLaunchKernelGGL(k_splitk_final<E>, dim3(groups), dim3(256), 0, s, part, (int)g, nout, C, op.out_scale, maxslot,
                     gn2, op.nN, gm, gr.gn_bits);
  return hipSuccess;
}

hipError_t launch_splitk(int dtype, const void* A, const void* B, void* C, float2* part, const IndexOp& op,
                         float* maxslot, hipStream_t s) {
  if (op.nM + op.nN > kSplitKMaxOutLog2) return hipErrorInvalidValue;
  hipError_t e;
  if (dtype == TN_DTYPE_F16S)
    e = launch_splitk_t<cf16>(dtype, (const cf16*)A, (const cf16*)B, (cf16*)C, part, op, maxslot, s);
  else if (dtype == TN_DTYPE_BF16S)
    e = launch_splitk_t<cbf16>(dtype, (const cbf16*)A, (const cbf16*)B, (cbf16*)C, part, op, maxslot, s);
  else
    e = launch_splitk_t<float2>(dtype, (const float2*)A, (const float2*)B, (float2*)C, part, op, maxslot, s);
  return e != hipSuccess ? e : hipGetLastError();
}

// ------------------------------------------------------------ accumulate --
// amp[y] += root[dep(y)] * 2^e_root in FP64 for the current slice; raises the
// non-finite flag; evaluates and clears the per-op magnitude records of
// scaled storage (overflow: a stored magnitude reached the format's maximum;
// underflow: an op's largest stored magnitude fell below `under`); advances
// the slice cursor.

template <typename E>
__global__ __launch_bounds__(256) void k_accum(const E* __restrict__ root, const Runs y2root, int n_open,
                                              double root_scale, Ctrl* ctrl, float* maxslots,
                                              const float* __restrict__ out_scales, int n_slots, float over,
                                              float under, double k0re, double k0im, int sliced_factors) {
  double* amp = ctrl->amp;
  const int64_t n = (int64_t)1 << n_open;
  // factor of this slice: 2^e_root, the unsliced leaves' rounding factor and
  // (left by the bind kernel) the sliced leaves' factor for this slice
  double kr = k0re * root_scale, ki = k0im * root_scale;
  if (sliced_factors) {
    const double sr = ctrl->kap_re, si = ctrl->kap_im;
    const double t = kr * sr - ki * si;
    ki = kr * si + ki * sr;
    kr = t;
  }
  bool bad = false;
  for (int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; y < n; y += (int64_t)gridDim.x * blockDim.x) {
    const float2 v = to_f2(root[dep((uint64_t)y, y2root)]);
    bad |= !(isfinite(v.x) && isfinite(v.y));
    amp[2 * y] += (double)v.x * kr - (double)v.y * ki;
    amp[2 * y + 1] += (double)v.x * ki + (double)v.y * kr;
  }
  if (bad) atomicOr(&ctrl->flags, (unsigned)TN_FLAG_NONFINITE);
  if (blockIdx.x == 0) {
    unsigned f = 0;
    for (int i = threadIdx.x; i < n_slots; i += blockDim.x) {
      const float m = maxslots[i] * out_scales[i];
      if (!(m < over)) f |= TN_FLAG_OVERFLOW;
      if (m < under) f |= TN_FLAG_UNDERFLOW;
      maxslots[i] = 0.f;
    }
    if (f) atomicOr(&ctrl->flags, f);
    if (threadIdx.x == 0) ctrl->cursor += 1;
  }
}

hipError_t launch_accum(int dtype, const void* root, const AccumDesc& d, Ctrl* ctrl, float* maxslots,
                        const float* out_scales, int n_slots, bool sliced_factors, hipStream_t s) {
  const int64_t n = (int64_t)1 << d.n_open;
  const int64_t grid = std::min<int64_t>((n + 255) / 256, 4096);
  const dim3 g((unsigned)grid);
  const float under = 0.25f;
  const int sf = sliced_factors ? 1 : 0;
  if (dtype == TN_DTYPE_F16S)
    hipLaunchKernelGGL(k_accum<cf16>, g, dim3(256), 0, s, (const cf16*)root, d.y2root, d.n_open, d.root_scale, ctrl,
                       maxslots, out_scales, n_slots, 65504.f, under, d.kappa0_re, d.kappa0_im, sf);
  else if (dtype == TN_DTYPE_BF16S)
    hipLaunchKernelGGL(k_accum<cbf16>, g, dim3(256), 0, s, (const cbf16*)root, d.y2root, d.n_open, d.root_scale,
                       ctrl, maxslots, out_scales, n_slots, 3.0e38f, under, d.kappa0_re, d.kappa0_im, sf);
  else
    hipLaunchKernelGGL(k_accum<float2>, g, dim3(256), 0, s, (const float2*)root, d.y2root, d.n_open, d.root_scale,
                       ctrl, maxslots, out_scales, 0, 3.0e38f, 0.f, 1.0, 0.0, 0);
  return hipGetLastError();
}

// ----------------------------------------------------------------- frugal --
// Frugal rejection sampling: candidate j (amplitude idx[j], or j) is kept
// when u[j] * m < scale * (re*re + im*im), evaluated in FP64 with every
// operation rounded on its own (no fused multiply-add), so the decision is
// the same as a plain FP64 evaluation of that expression.  Kept indices are
// appended through an atomic counter (order unspecified).

__global__ void k_zero_count(unsigned long long* count) { *count = 0ull; }

__global__ __launch_bounds__(256) void k_frugal(const double* __restrict__ amp, int64_t n,
                                               const int64_t* __restrict__ idx, int64_t n_cand,
                                               const double* __restrict__ u, double scale, double m,
                                               int64_t* __restrict__ out, unsigned long long* count) {
#pragma clang fp contract(off)
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_cand;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx ? idx[j] : j;
    if (i < 0 || i >= n) continue;  // out-of-range candidates are never kept
    const double re = amp[2 * i], im = amp[2 * i + 1];
    const double rr = re * re;
    const double ii = im * im;
    const double x = (rr + ii) * scale;
    const double t = u[j] * m;
    if (t < x) out[atomicAdd(count, 1ull)] = i;
  }
}

hipError_t launch_frugal(const double* amp, int64_t n, const int64_t* idx, int64_t n_cand, const double* u,
                         double scale, double m, int64_t* out, unsigned long long* count, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, count);
  if (n_cand > 0) {
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((n_cand + 255) / 256, 8192));
    hipLaunchKernelGGL(k_frugal, dim3((unsigned)grid), dim3(256), 0, s, amp, n, idx, n_cand, u, scale, m, out, count);
  }
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
  const int64_t grid = std::min<int64_t>((n + 255) / 256, 4096);
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hist, dim3((unsigned)grid), dim3(256), 0, s, amp, n, scale, xmax, n_bins, counts);
  return hipGetLastError();
}

}  // namespace tnrcs
