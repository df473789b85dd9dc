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
};

hipError_t launch_set_ctrl(Ctrl* ctrl, int64_t cursor, void* amp, hipStream_t s);
hipError_t launch_bind(const float2* leaves, float2* bound, const BindDesc* descs, int n_desc,
                       int64_t max_elems, const Ctrl* ctrl, hipStream_t s);
hipError_t launch_permute_c64(const float2* in, float2* out, int rank, const int32_t* perm, int64_t batch,
                              hipStream_t s);
// splits > 1: K split into slabs summed in order through `work` (splits*M*N entries).
hipError_t launch_gemm_c64(const float2* A, const float2* B, float2* C, int64_t M, int64_t N, int64_t K,
                           int64_t batch, int form, hipStream_t s, float2* work = nullptr, int splits = 1);
hipError_t launch_generic_c64(const float2* A, const float2* B, float2* C, const IndexOp& op,
                              hipStream_t s);
hipError_t launch_splitk_c64(const float2* A, const float2* B, float2* C, float2* part, const IndexOp& op,
                             hipStream_t s);
int64_t splitk_blocks(const IndexOp& op);
hipError_t launch_accum(const float2* root, const AccumDesc& d, Ctrl* ctrl, hipStream_t s);
hipError_t launch_norm2(const double* amp, int64_t n, double* out, hipStream_t s);
hipError_t launch_xeb(const double* amp, int64_t n, const int64_t* idx, int64_t n_idx, double* out,
                      hipStream_t s);
hipError_t launch_hist(const double* amp, int64_t n, double scale, double xmax, int n_bins,
                       unsigned long long* counts, hipStream_t s);

bool gemm_shape_ok(int64_t M, int64_t N, int64_t K);

}  // namespace tnrcs
