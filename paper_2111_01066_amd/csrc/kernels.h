// Host-side launchers of the tnrcs gfx950 kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace tnrcs {

// Per-plan device control block read and written by the per-slice kernels.
struct Ctrl {
  int64_t cursor;   // slice id of the slice being contracted
  double* amp;      // caller's complex128 accumulator (re, im pairs)
  uint32_t flags;   // TN_FLAG_* (sticky)
  uint32_t pad;
  double kap_re, kap_im;  // scaled storage: product of the sliced leaves' rounding factors for this slice
};

inline int elem_bytes_of(int dtype) { return dtype == TN_DTYPE_C64 ? 8 : 4; }

hipError_t launch_set_ctrl(Ctrl* ctrl, int64_t cursor, void* amp, hipStream_t s, bool clear_flags = false);
// dst += src over n complex128 entries.
hipError_t launch_add_amp(const double* src, double* dst, int64_t n, hipStream_t s);
// bytes / 4 words of pseudo-random values of the storage format (tuning data)
hipError_t launch_fill_random(void* p, int64_t bytes, int dtype, hipStream_t s);
// Copies every sliced leaf's sub-block of the current slice; with kappa
// (scaled storage) also stores the product of their rounding factors in ctrl.
hipError_t launch_bind(int elem_bytes, const void* leaves, void* bound, const BindDesc* descs, int n_desc,
                       int64_t max_elems, Ctrl* ctrl, const double2* kappa, hipStream_t s);
hipError_t launch_permute(int elem_bytes, const void* in, void* out, int rank, const int32_t* perm, int64_t batch,
                          hipStream_t s);
// complex64 GEMM on FP32 MFMA; splits > 1: K split into slabs summed in order
// through `work` (splits*M*N complex64).
hipError_t launch_gemm_c64(const float2* A, const float2* B, float2* C, int64_t M, int64_t N, int64_t K,
                           int64_t batch, int form, hipStream_t s, float2* work = nullptr, int splits = 1,
                           int tile = 0);
// complex64 GEMM whose A is read in its stored layout through idx.aM / idx.aK
// (B is [N][K], C is [M][N]; 128x128 tiles, no K split): the planner's
// alternative to permuting A first (gemm_gather_ok must hold).
hipError_t launch_gemm_c64_ga(const float2* A, const float2* B, float2* C, const IndexOp& idx, int form,
                              hipStream_t s);
// the same for scaled FP16/BF16 (4M, 128x128 tiles, stages of 32 k; nK >= 5):
// C = A B^T * out_scale, max |A B^T| recorded in *maxslot
hipError_t launch_gemm_half_ga(int dtype, const void* A, const void* B, void* C, const IndexOp& idx, float out_scale,
                               float* maxslot, hipStream_t s);
// scaled FP16/BF16 GEMM on half MFMA; C = A B^T * out_scale; max |A B^T| recorded in *maxslot.
// tile: 0 auto, 64 or 128; occ (128 tiles): 0 auto, 1 or 2 waves per SIMD, 3 the
// ping-pong 256x128 kernel (4M, M % 256 == 0, K per split % 32 == 0).
hipError_t launch_gemm_half(int dtype, const void* A, const void* B, void* C, int64_t M, int64_t N, int64_t K,
                            int64_t batch, int form, hipStream_t s, float2* work, int splits, float out_scale,
                            float* maxslot, int tile = 0, int occ = 0);
hipError_t launch_generic(int dtype, const void* A, const void* B, void* C, const IndexOp& op, float* maxslot,
                          hipStream_t s);
// skewed contraction with B and A's K offsets in LDS (nN <= 4, nK + nN <= kSkinnyMaxLog2)
hipError_t launch_skinny(int dtype, const void* A, const void* B, void* C, const IndexOp& op, float* maxslot,
                         hipStream_t s);
// skewed contraction on FP32 matrix cores (nN <= 6, 1 <= nK <= 10, nM >= 7)
hipError_t launch_skew(int dtype, const void* A, const void* B, void* C, const IndexOp& op, float* maxslot,
                       hipStream_t s);
bool skew_ok(const IndexOp& op);
hipError_t launch_splitk(int dtype, const void* A, const void* B, void* C, float2* part, const IndexOp& op,
                         float* maxslot, hipStream_t s);
int64_t splitk_blocks(const IndexOp& op);
// split-K with both operands read in place (splitk_chunk_ok); *nblk = the
// blocks whose partial sums it leaves in part
hipError_t launch_splitk_chunk(int dtype, const void* A, const void* B, float2* part, const IndexOp& op,
                               int64_t* nblk, hipStream_t s);
// both operands hold their lowest k bits (up to 2^kSplitChunkLog2) lowest, in order
bool splitk_chunk_aligned(const IndexOp& op);
// The slice result is multiplied by d.root_scale, d.kappa0 and, if
// sliced_factors, by the per-slice factor that the bind kernel left in ctrl.
hipError_t launch_accum(int dtype, const void* root, const AccumDesc& d, Ctrl* ctrl, float* maxslots,
                        const float* out_scales, int n_slots, bool sliced_factors, hipStream_t s);
hipError_t launch_frugal(const double* amp, int64_t n, const int64_t* idx, int64_t n_cand, const double* u,
                         double scale, double m, int64_t* out, unsigned long long* count, hipStream_t s);
hipError_t launch_norm2(const double* amp, int64_t n, double* out, hipStream_t s);
hipError_t launch_xeb(const double* amp, int64_t n, const int64_t* idx, int64_t n_idx, double* out,
                      hipStream_t s);
hipError_t launch_hist(const double* amp, int64_t n, double scale, double xmax, int n_bins,
                       unsigned long long* counts, hipStream_t s);

// probes: MFMA issue loop (kind 0 FP32, 1 FP16, 2 BF16; *flops = flops issued),
// streaming copy of n16 16-byte units
hipError_t launch_mfma_peak(int kind, int64_t iters, float* out, double* flops, hipStream_t s);
int64_t mfma_peak_out_floats();
hipError_t launch_stream_copy(const void* src, void* dst, int64_t n16, hipStream_t s);

bool gemm_shape_ok(int64_t M, int64_t N, int64_t K);
bool hgemm_shape_ok(int64_t M, int64_t N, int64_t K);

}  // namespace tnrcs
