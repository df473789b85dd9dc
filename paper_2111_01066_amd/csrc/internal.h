// Internal data structures shared by the planner (host C++) and the HIP
// runtime of the tnrcs library.  Not part of the C ABI.
#pragma once

#include <complex>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/tnrcs.h"

namespace tnrcs {

constexpr int kMaxRank = 48;  // bits of a device tensor index
constexpr int kMaxRuns = 48;  // runs of a bit-deposit map
constexpr int kSkinnyMaxLog2 = 11;  // the skewed kernel keeps 2^(nK+nN) <= 2^11 B entries in LDS
// Longest run of terms that one FP32 accumulator of the complex64 GEMM sums
// before the run is added to the output: sequential FP32 accumulation of n
// products of random sign has a relative error growing like u sqrt(n/2)
// (u = 2^-24), about 6e-6 for n = 2^17, so long contractions are summed in
// runs of this length (about 8e-7 at n = 2^17).
constexpr int kAccChain = 2048;

// Bit-deposit map: value bit (src + i) goes to target bit (dst + i) for
// i < len, for each run.  Built from "value bit j -> target position pos[j]".
struct Runs {
  int32_t n = 0;
  int8_t src[kMaxRuns] = {};
  int8_t dst[kMaxRuns] = {};
  int8_t len[kMaxRuns] = {};
};

bool make_runs(const std::vector<int>& pos, Runs* r);  // false if too many runs

enum Region : int32_t { kArena = 0, kLeaves = 1, kBound = 2, kExtA = 3, kExtB = 4, kExtC = 5 };

struct TRef {
  int32_t region = kArena;
  int64_t off = 0;  // element offset (complex elements) within the region
};

enum OpKind : int32_t { kOpPermute = 0, kOpGemm = 1, kOpGeneric = 2, kOpSkinny = 3, kOpSplitK = 4, kOpSkew = 5 };

// Permute: output position q takes input position perm[q].
struct PermuteOp {
  int32_t rank = 0;
  int32_t perm[kMaxRank] = {};
};

// GEMM: C[M][N] = sum_k A[M][K] * B[N][K]   (row-major, complex)
struct GemmOp {
  int64_t M = 0, N = 0, K = 0;
  int32_t form = TN_GEMM_4M;
  int32_t split_k = 1;  // K split into this many partial products (summed in a second pass)
  float out_scale = 1.f;  // scaled storage: 2^-s applied before rounding
  int32_t tile = 0;       // workgroup tile edge: 0 = chosen by shape, 64 or 128 (autotuner)
  int32_t split_max = 1;  // split-K workspace capacity in slabs
  int32_t occ = 0;        // FP16/BF16 128x128 kernel: waves per SIMD (0 = chosen by K, 1 or 2; autotuner)
  int32_t gather_a = 0;   // 1: A is read in its stored layout through the op's idx.aM / idx.aK
};

// Generic / skinny: C[m, n] = sum_k A[dep(m,aM) | dep(k,aK)] * B[dep(n,bN) | dep(k,bK)],
// C index = (m << nN) | n.
struct IndexOp {
  int32_t nM = 0, nN = 0, nK = 0;
  Runs aM, aK, bN, bK;
  // skinny tiling (planner-chosen): the tile holds the low tM M-bits and the
  // low tK K-bits of the chunk; the remaining bits index tiles / chunks.
  int32_t tM = 0, tK = 0;
  float out_scale = 1.f;  // scaled storage: 2^-s applied before rounding
};

struct Op {
  int32_t kind = kOpGeneric;
  int32_t step = -1;  // SSA step this op belongs to
  TRef a, b, c;       // permute: a = in, c = out
  TRef w;             // workspace (split-K partial sums)
  PermuteOp perm;
  GemmOp gemm;
  IndexOp idx;
  double flops = 0;   // algorithmic (8 per complex MAC)
  double bytes = 0;   // bytes moved by this kernel
  // scaled storage: producing ops record max |accumulator| in slot max_slot
  // and store accumulator * 2^-s_out; their result's exponent is
  // e(ssa_a) + e(ssa_b) + s_out.
  int32_t max_slot = -1;
  int32_t s_out = 0;
  int32_t ssa_a = -1, ssa_b = -1, ssa_c = -1;
};

// A device leaf: stored once for all slices with its sliced wires as the top
// bits; per slice the bind kernel copies the selected sub-tensor to `bound`.
struct DevLeaf {
  int32_t ssa = -1;
  std::vector<int> layout;   // stored layout, most significant first (sliced wires first)
  int32_t n_sliced = 0;      // leading entries of layout that are sliced wires
  std::vector<int> slice_bit;  // per leading sliced wire: its index j in the sliced list
  int64_t stored_off = 0;    // element offset in the leaves region
  int64_t bound_off = 0;     // element offset in the bound region (if n_sliced > 0)
  std::vector<std::complex<double>> data;  // FP64 values in the stored layout
  int32_t e = 0;  // scaled storage: stored = value * 2^-e
};

struct BindDesc {  // device-side descriptor of one sliced leaf
  int64_t src_off, dst_off, n_elems;
  int32_t n_sl;
  int32_t sbit[8];
  int32_t pos[8];
  int64_t kappa_off;  // scaled storage: first entry of this leaf's rounding factors (one per sub-block)
};

struct AccumDesc {
  int32_t n_open = 0;
  Runs y2root;  // amplitude index bits -> root layout positions
  TRef root;
  int32_t root_ssa = -1;
  double root_scale = 1.0;  // 2^e_root for scaled storage
  // scaled storage: product over the unsliced device leaves of <L, L>/<L, round(L)>
  double kappa0_re = 1.0, kappa0_im = 0.0;
};

struct HostTensor {
  std::vector<int> wires;  // most significant first
  std::vector<std::complex<double>> data;
};

struct PlanCore {
  // inputs (copied)
  int32_t n_qubits = 0;
  std::vector<tn_gate> gates;
  std::vector<uint8_t> out_bits;
  std::vector<int32_t> pairs;
  std::vector<int32_t> sliced;
  std::vector<int32_t> open_q;
  tn_plan_opts opts{};

  // network
  int32_t n_leaves = 0, n_wires = 0;
  std::vector<std::vector<int>> leaf_wires;
  std::vector<int> open_wires;
  std::vector<int> wire_slice_idx;  // wire -> j or -1

  // host part
  std::vector<bool> on_host;   // per SSA id
  int32_t n_host_steps = 0;
  std::vector<DevLeaf> dev_leaves;
  std::vector<BindDesc> binds;
  int64_t leaves_elems = 0, bound_elems = 0;

  // device part
  std::vector<Op> ops;
  AccumDesc accum;
  int64_t arena_elems = 0;
  int32_t root_is_leaf = 0;
  std::vector<int> root_layout;  // layout of the final tensor (wires, most significant first)
  int32_t n_slots = 0;  // producing ops with a magnitude record (scaled storage)
  tn_plan_stats stats{};
  std::string json;

  // kernel class per device step: the planner's rule unless the autotuner
  // measured another valid class to be faster (step -> OpKind)
  std::map<int, int> class_override;
  struct StepInfo {
    int32_t t = 0;
    // operand and result layouts, most significant first, with the wires
    // relabelled by first appearance (A's, then B's new ones): steps with
    // the same labels run the same kernels on the same index maps
    std::vector<int> la, lb, lc;
    std::string key;  // the three label lists as text ("0.1.2/3.1/0.2.3")
    int32_t nM = 0, nN = 0, nK = 0, cls = 0;
  };
  std::vector<StepInfo> steps;  // device steps as planned

  // pairwise-contraction mode (one step A x B -> C over caller buffers)
  bool pair_mode = false;
  std::vector<int> pair_a, pair_b, pair_out;  // index labels, most significant first
};

// Plans one pairwise contraction of caller tensors with the given index
// labels (most significant first); the result is left in kExtC in the order
// of `out` (a permute is appended when the step's natural layout differs).
int build_pair_plan(PlanCore& P, std::string& err);
// (Re)writes P.json from the current plan.
void make_json(PlanCore& P);

// Kernel classes of a step with 2^nM x 2^nN outputs over 2^nK terms.  dense
// (permutes + MFMA GEMM): both free extents at least 64 (the smallest GEMM
// tile) and K at least 16; split-K: at most 64 outputs, or up to
// 2^kSplitKMaxOutLog2 outputs (run as groups of 64) over at least 2^12
// terms; skewed (Supplement,
// CPU-architecture section): few outputs per row of the large operand, in
// two kernels: on the vector units with the small operand in LDS (at most
// 16 outputs per row, 2^(nK+nN) <= 2^kSkinnyMaxLog2 entries), and on the
// matrix cores (at most 64 outputs per row, 2 <= K <= 2^10, at least 128
// rows); gathered: always valid.  Bit mask over OpKind.
constexpr int kSplitKMaxOutLog2 = 12;
inline unsigned step_classes(int nM, int nN, int nK) {
  unsigned m = 1u << kOpGeneric;
  if (nM >= 6 && nN >= 6 && nK >= 4) m |= 1u << kOpGemm;
  if ((nM + nN <= 6 && nK >= 4) || (nM + nN <= kSplitKMaxOutLog2 && nK >= 12)) m |= 1u << kOpSplitK;
  if (nN <= 4 && nK + nN <= kSkinnyMaxLog2 && nM >= 8) m |= 1u << kOpSkinny;
  if (nN <= 6 && nK >= 1 && nK <= 10 && nM >= 7) m |= 1u << kOpSkew;
  return m;
}
// The planner's rule among them: dense where valid and the contraction is
// long (K >= 128) or the output wide (N >= 128), split-K for long sums into
// few outputs, the vector skewed kernel for at most 2^4 terms x outputs,
// then the matrix-core skewed kernel, then the vector one, then gathered.
inline int default_class(int nM, int nN, int nK) {
  const unsigned m = step_classes(nM, nN, nK);
  if ((m & (1u << kOpGemm)) && (nK >= 7 || nN >= 7 || !(m & (1u << kOpSkew)))) return kOpGemm;
  if ((m & (1u << kOpSplitK)) && nK >= 10) return kOpSplitK;
  // the fewest terms and outputs (a gate on a state): the vector-unit kernel
  if ((m & (1u << kOpSkinny)) && nK + nN <= 4) return kOpSkinny;
  if (m & (1u << kOpSkew)) return kOpSkew;
  if (m & (1u << kOpSkinny)) return kOpSkinny;
  return kOpGeneric;
}
// Position in the target of bit j of a value deposited by runs r (-1: none).
inline int run_pos(const Runs& r, int j) {
  for (int i = 0; i < r.n; ++i)
    if (j >= r.src[i] && j < r.src[i] + r.len[i]) return r.dst[i] + (j - r.src[i]);
  return -1;
}
// GEMM steps whose large operand A (at least 2^kGatherMinLog2
// entries) is not stored as [M bits, K bits] and whose sum has at least
// 2^kGatherMinK terms read A in place instead of permuting it first, when
// its layout admits that: 128 x 128 output tiles and chunks of 16 k (nM, nN
// >= 7, nK >= 4), the chunk's 11 bits within A's low 32 positions, and the k
// bits above 3 in increasing positions.  (The planner also requires at least
// 512 output tiles when the sum has 2^11 terms or more, since the in-place
// kernels do not split K.)
constexpr int kGatherMinLog2 = 20;
constexpr int kGatherMinK = 5;
inline bool gemm_gather_ok(const IndexOp& idx) {
  if (idx.nM < 7 || idx.nN < 7 || idx.nK < 4) return false;
  for (int j = 0; j < 7; ++j) {
    const int p = run_pos(idx.aM, j);
    if (p < 0 || p >= 32) return false;
  }
  int prev = -1;
  for (int j = 0; j < idx.nK; ++j) {
    const int p = run_pos(idx.aK, j);
    if (p < 0 || (j < 4 && p >= 32) || (j >= 4 && p <= prev)) return false;
    if (j >= 4) prev = p;
  }
  return true;
}
// Split-K steps with at most 2^3 x 2^3 outputs read both operands in place
// whatever their layout (chunks of 2^kSplitChunkLog2 k loaded in address
// order), so the planner permutes neither operand for them.
constexpr int kSplitChunkLog2 = 8;
inline bool splitk_chunk_ok(int nM, int nN, int nK) { return nM <= 3 && nN <= 3 && nK >= 12 && nK <= 40; }
// Planner entry (host only).  Returns TN_OK or an error code with a message.
int build_plan(PlanCore& P, std::string& err);
// Blocks of the split-K reduction over 2^nK terms (its workspace holds
// blocks x outputs entries).
inline int64_t splitk_grid(int nK) {
  const int64_t k = (int64_t)1 << nK;
  const int64_t g = k / 1024;
  return g < 1 ? 1 : (g > 1024 ? 1024 : g);
}
// Re-folds the leaves after an output-bit change (same structure).
int refold_leaves(PlanCore& P, std::string& err);
// Scaled storage: leaf exponents from the leaf data (largest |component|
// brought to 2^kTargetLog2), then every tensor's exponent along the ops and
// the root scale of the accumulation.
constexpr int kTargetLog2 = 12;
void leaf_exponents(PlanCore& P);
void propagate_exponents(PlanCore& P);
// Sets op.s_out (and its out_scale) from a recorded max |accumulator|.
void set_output_shift(Op& op, float max_acc);

}  // namespace tnrcs
