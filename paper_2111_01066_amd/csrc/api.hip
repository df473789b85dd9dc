// C ABI of the tnrcs library: plan objects, the per-slice scheduler (one HIP
// graph replay per slice, FP64 accumulation into the caller's buffer), the
// exponent calibration of scaled half-precision plans, and the standalone
// kernel entry points.  See include/tnrcs.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <string>

#include "internal.h"
#include "kernels.h"
#include "tune.h"

using namespace tnrcs;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// Progress lines of the plan-time tuners on stderr when TNRCS_VERBOSE is set
// (tuning a large plan runs for minutes).
bool verbose() {
  static const bool v = std::getenv("TNRCS_VERBOSE") != nullptr;
  return v;
}

int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return TN_E_HIP;
}

#define HIP_TRY(expr, what)                 \
  do {                                      \
    hipError_t _e = (expr);                 \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

// Round-to-nearest-even encodings of a double in IEEE binary16 and bfloat16.
uint16_t encode_small_float(double v, int mant_bits, int exp_bias, int exp_max_field) {
  uint16_t sign = std::signbit(v) ? 0x8000u : 0u;
  double a = std::fabs(v);
  if (a == 0) return sign;
  if (!std::isfinite(a)) return sign | (uint16_t)(exp_max_field << mant_bits);
  int e;
  std::frexp(a, &e);  // a = m 2^e, m in [0.5, 1)
  int ef = e - 1 + exp_bias;  // biased exponent of the normal encoding
  if (ef <= 0) {
    // subnormal: unit 2^(1 - bias - mant_bits)
    double q = std::nearbyint(std::ldexp(a, exp_bias - 1 + mant_bits));
    return sign | (uint16_t)q;  // q == 2^mant_bits carries into the smallest normal
  }
  double q = std::nearbyint(std::ldexp(a, mant_bits + 1 - e));  // in [2^mant, 2^(mant+1)]
  if (q >= std::ldexp(1.0, mant_bits + 1)) {
    q /= 2;
    ++ef;
  }
  if (ef >= exp_max_field) return sign | (uint16_t)(exp_max_field << mant_bits);
  return sign | (uint16_t)((ef << mant_bits) | ((uint32_t)q - (1u << mant_bits)));
}
uint16_t to_f16_bits(double v) { return encode_small_float(v, 10, 15, 31); }
uint16_t to_bf16_bits(double v) { return encode_small_float(v, 7, 127, 255); }

// Value of a finite binary16 / bfloat16 encoding.
double decode_small_float(uint16_t b, int mant_bits, int exp_bias) {
  const int ef = (b & 0x7FFF) >> mant_bits;
  const double m = (double)(b & ((1u << mant_bits) - 1u));
  const double a = ef == 0 ? std::ldexp(m, 1 - exp_bias - mant_bits)
                           : std::ldexp(1.0 + std::ldexp(m, -mant_bits), ef - exp_bias);
  return (b & 0x8000u) ? -a : a;
}

}  // namespace

struct tn_plan_s {
  PlanCore core;
  int device = 0;
  int eb = 8;  // element bytes
  char* d_leaves = nullptr;
  char* d_bound = nullptr;
  char* d_arena = nullptr;
  bool own_arena = true;  // false: the caller's workspace (opts.arena)
  BindDesc* d_binds = nullptr;
  Ctrl* d_ctrl = nullptr;
  float* d_maxslots = nullptr;
  float* d_outscales = nullptr;
  double2* d_kappa = nullptr;  // scaled storage: per sub-block rounding factors of the sliced leaves
  double* d_stage = nullptr;   // checked runs: one slice's bunch before it joins the sum
  int64_t bind_max = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t last_stream = nullptr;
  bool ran = false;
  // pairwise mode: caller buffers of the current run
  const char* ext_a = nullptr;
  const char* ext_b = nullptr;
  char* ext_c = nullptr;
};

// Independent lanes of a batch (plans on separate arenas); at most this
// many run side by side.
constexpr int kBatchMaxLanes = 4;

// One captured graph per lane.  A run launches each lane's graph on a lane
// stream of the batch, between a fork event recorded on the caller's stream
// and join events the caller's stream waits for.  (One graph with a branch
// per lane measured no faster than the lanes in sequence: its branches did
// not overlap.)
struct tn_batch_s {
  int device = 0;
  std::vector<tn_plan_s*> plans;
  std::vector<int64_t> ranges;            // [begin, end) of plan i at 2i, 2i + 1
  std::vector<void*> amps;
  std::vector<std::vector<int>> lanes;    // plan indices of each lane, in the order given
  std::vector<hipStream_t> lane_streams;  // one per lane
  std::vector<hipEvent_t> fork, join;     // fork[k] / join[k] for lane k
};

static void batch_release(tn_batch_s* b) {
  for (hipStream_t st : b->lane_streams)
    if (st) hipStreamDestroy(st);
  for (hipEvent_t ev : b->fork)
    if (ev) hipEventDestroy(ev);
  for (hipEvent_t ev : b->join)
    if (ev) hipEventDestroy(ev);
  b->lane_streams.clear();
  b->fork.clear();
  b->join.clear();
}

static char* resolve(const tn_plan_s* p, const TRef& r) {
  char* base;
  switch (r.region) {
    case kLeaves:
      base = p->d_leaves;
      break;
    case kBound:
      base = p->d_bound;
      break;
    case kExtA:
      base = const_cast<char*>(p->ext_a);
      break;
    case kExtB:
      base = const_cast<char*>(p->ext_b);
      break;
    case kExtC:
      base = p->ext_c;
      break;
    default:
      base = p->d_arena;
  }
  return base + r.off * (int64_t)p->eb;
}

static int upload_leaves(tn_plan_s* p) {
  PlanCore& P = p->core;
  const int dt = P.opts.dtype;
  if (dt != TN_DTYPE_C64) leaf_exponents(P);
  std::vector<uint32_t> h32;
  std::vector<float2> h64;
  if (dt == TN_DTYPE_C64)
    h64.assign((size_t)P.leaves_elems, make_float2(0.f, 0.f));
  else
    h32.assign((size_t)P.leaves_elems, 0u);
  const bool f16 = dt == TN_DTYPE_F16S;
  const int mant = f16 ? 10 : 7, bias = f16 ? 15 : 127;
  std::complex<double> kappa0 = 1.0;
  std::vector<std::complex<double>> kappa;  // sliced leaves' sub-block factors, in bind order
  for (const DevLeaf& d : P.dev_leaves) {
    if (dt == TN_DTYPE_C64) {
      for (size_t i = 0; i < d.data.size(); ++i)
        h64[d.stored_off + i] = make_float2((float)d.data[i].real(), (float)d.data[i].imag());
      continue;
    }
    // Round to nearest even, then measure what rounding did to the leaf as
    // a whole.  Write round(L) = rho L + D with D orthogonal to L, per
    // sub-block that one slice uses (rho = <L, round(L)> / <L, L>).  The
    // amplitude is linear in every leaf, so the rho part scales it exactly by
    // rho; the same gate tensors recur throughout a circuit, so these
    // factors do not average out but compound with depth (a bias of the
    // amplitudes' magnitude, visible in the cross-entropy estimate).  The
    // accumulation divides them out in FP64; only D, which averages out,
    // remains.
    const double sc = std::ldexp(1.0, -d.e);
    const size_t nb = d.data.size() >> d.n_sliced;
    for (size_t blk = 0; blk < ((size_t)1 << d.n_sliced); ++blk) {
      std::complex<double> dot = 0;
      double ssq = 0;
      for (size_t i = blk * nb; i < (blk + 1) * nb; ++i) {
        const double re = d.data[i].real() * sc, im = d.data[i].imag() * sc;
        const uint16_t r = f16 ? to_f16_bits(re) : to_bf16_bits(re);
        const uint16_t m = f16 ? to_f16_bits(im) : to_bf16_bits(im);
        h32[d.stored_off + i] = (uint32_t)r | ((uint32_t)m << 16);
        const std::complex<double> x(re, im), xr(decode_small_float(r, mant, bias), decode_small_float(m, mant, bias));
        dot += std::conj(x) * xr;
        ssq += std::norm(x);
      }
      const std::complex<double> kap = (ssq > 0 && std::abs(dot) > 0) ? ssq / dot : std::complex<double>(1.0);
      if (d.n_sliced == 0)
        kappa0 *= kap;
      else
        kappa.push_back(kap);
    }
  }
  const void* src = dt == TN_DTYPE_C64 ? (const void*)h64.data() : (const void*)h32.data();
  if (P.leaves_elems > 0)
    HIP_TRY(hipMemcpy(p->d_leaves, src, (size_t)P.leaves_elems * p->eb, hipMemcpyHostToDevice), "upload leaves");
  P.accum.kappa0_re = kappa0.real();
  P.accum.kappa0_im = kappa0.imag();
  if (dt != TN_DTYPE_C64 && !kappa.empty()) {
    int64_t off = 0;
    size_t j = 0;
    for (const DevLeaf& d : P.dev_leaves)
      if (d.n_sliced > 0) {
        P.binds[j++].kappa_off = off;
        off += (int64_t)1 << d.n_sliced;
      }
    if (!p->d_kappa)
      HIP_TRY(hipMalloc((void**)&p->d_kappa, kappa.size() * sizeof(double2)), "alloc rounding factors");
    HIP_TRY(hipMemcpy(p->d_kappa, kappa.data(), kappa.size() * sizeof(double2), hipMemcpyHostToDevice),
            "upload rounding factors");
  }
  return TN_OK;
}

static int upload_scales(tn_plan_s* p) {
  PlanCore& P = p->core;
  if (P.n_slots == 0) return TN_OK;
  std::vector<float> sc(P.n_slots, 1.f), zero(P.n_slots, 0.f);
  for (const Op& op : P.ops)
    if (op.max_slot >= 0) sc[op.max_slot] = (float)std::ldexp(1.0, -op.s_out);
  HIP_TRY(hipMemcpy(p->d_outscales, sc.data(), sc.size() * sizeof(float), hipMemcpyHostToDevice), "upload scales");
  HIP_TRY(hipMemcpy(p->d_maxslots, zero.data(), zero.size() * sizeof(float), hipMemcpyHostToDevice),
          "clear magnitude records");
  return TN_OK;
}

// Launches the kernel(s) of one planned op.
static int launch_op(tn_plan_s* p, const Op& op, hipStream_t s) {
  const int dt = p->core.opts.dtype;
  const char* a = resolve(p, op.a);
  const char* b = resolve(p, op.b);
  char* c = resolve(p, op.c);
  float* slot = op.max_slot >= 0 ? p->d_maxslots + op.max_slot : nullptr;
  float2* w = reinterpret_cast<float2*>(resolve(p, op.w));
  switch (op.kind) {
    case kOpPermute:
      HIP_TRY(launch_permute(p->eb, a, c, op.perm.rank, op.perm.perm, 1, s), "permute kernel");
      break;
    case kOpGemm:
      if (op.gemm.gather_a && dt == TN_DTYPE_C64)
        HIP_TRY(launch_gemm_c64_ga((const float2*)a, (const float2*)b, (float2*)c, op.idx, op.gemm.form, s),
                "gemm kernel (A in place)");
      else if (op.gemm.gather_a)
        HIP_TRY(launch_gemm_half_ga(dt, a, b, c, op.idx, op.gemm.out_scale, slot, s), "half gemm kernel (A in place)");
      else if (dt == TN_DTYPE_C64)
        HIP_TRY(launch_gemm_c64((const float2*)a, (const float2*)b, (float2*)c, op.gemm.M, op.gemm.N, op.gemm.K, 1,
                                op.gemm.form, s, op.gemm.split_k > 1 ? w : nullptr, op.gemm.split_k, op.gemm.tile),
                "gemm kernel");
      else
        HIP_TRY(launch_gemm_half(dt, a, b, c, op.gemm.M, op.gemm.N, op.gemm.K, 1, op.gemm.form, s,
                                 op.gemm.split_k > 1 ? w : nullptr, op.gemm.split_k, op.gemm.out_scale, slot,
                                 op.gemm.tile, op.gemm.occ),
                "half gemm kernel");
      break;
    case kOpSplitK:
      HIP_TRY(launch_splitk(dt, a, b, c, w, op.idx, slot, s), "split-K kernel");
      break;
    case kOpSkinny:
      HIP_TRY(launch_skinny(dt, a, b, c, op.idx, slot, s), "skewed contraction kernel");
      break;
    case kOpSkew:
      HIP_TRY(launch_skew(dt, a, b, c, op.idx, slot, s), "skewed matrix-core contraction kernel");
      break;
    default:
      HIP_TRY(launch_generic(dt, a, b, c, op.idx, slot, s), "contraction kernel");
      break;
  }
  return TN_OK;
}

static int launch_bind_slice(tn_plan_s* p, hipStream_t s) {
  const PlanCore& P = p->core;
  if (!P.binds.empty())
    HIP_TRY(launch_bind(p->eb, p->d_leaves, p->d_bound, p->d_binds, (int)P.binds.size(), p->bind_max, p->d_ctrl,
                        p->d_kappa, s),
            "bind kernel");
  return TN_OK;
}

static int launch_accum_slice(tn_plan_s* p, hipStream_t s) {
  const PlanCore& P = p->core;
  HIP_TRY(launch_accum(P.opts.dtype, resolve(p, P.accum.root), P.accum, p->d_ctrl, p->d_maxslots, p->d_outscales,
                       P.n_slots, p->d_kappa != nullptr, s),
          "accumulate kernel");
  return TN_OK;
}

// Enqueues one slice: bind, the per-step kernels, FP64 accumulation.
static int enqueue_slice(tn_plan_s* p, hipStream_t s) {
  int rc = launch_bind_slice(p, s);
  if (rc) return rc;
  for (const Op& op : p->core.ops) {
    rc = launch_op(p, op, s);
    if (rc) return rc;
  }
  return launch_accum_slice(p, s);
}

// Scaled storage: choose every producing op's output shift from slice 0.  Op
// by op in plan order: run it with shift 0 (its FP32 accumulator magnitude is
// recorded before any rounding), derive the shift that brings the largest
// magnitude to 2^kTargetLog2, run it again so its stored output uses that
// shift, and go on to the next op (whose inputs are now final).
static int calibrate(tn_plan_s* p, int64_t slice = 0) {
  PlanCore& P = p->core;
  if (P.opts.dtype == TN_DTYPE_C64 || P.n_slots == 0) {
    propagate_exponents(P);
    return TN_OK;
  }
  hipStream_t s = nullptr;
  HIP_TRY(launch_set_ctrl(p->d_ctrl, slice, nullptr, s), "control kernel");
  int rc = launch_bind_slice(p, s);
  if (rc) return rc;
  const float zero = 0.f;
  for (Op& op : P.ops) {
    if (op.max_slot < 0) {
      if ((rc = launch_op(p, op, s))) return rc;
      continue;
    }
    float* slot = p->d_maxslots + op.max_slot;
    set_output_shift(op, 0.f);
    HIP_TRY(hipMemcpy(slot, &zero, sizeof(float), hipMemcpyHostToDevice), "clear record");
    if ((rc = launch_op(p, op, s))) return rc;
    float mx = 0.f;
    HIP_TRY(hipMemcpy(&mx, slot, sizeof(float), hipMemcpyDeviceToHost), "read record");
    if (!std::isfinite(mx)) return fail(TN_E_NUMERIC, "calibration: non-finite accumulator in step " +
                                                         std::to_string(op.step));
    set_output_shift(op, mx);
    if ((rc = launch_op(p, op, s))) return rc;
  }
  HIP_TRY(hipDeviceSynchronize(), "calibration synchronize");
  propagate_exponents(P);
  make_json(P);
  return upload_scales(p);
}

// Autotuning: fill the arena with random values of the storage format, then
// time each dense GEMM step's variants on its own buffers (shapes seen before
// are answered from the cache).
static int tune_plan(tn_plan_s* p) {
  PlanCore& P = p->core;
  bool any = false;
  for (const Op& op : P.ops) any |= op.kind == kOpGemm;
  if (!any) return TN_OK;
  if (P.arena_elems > 0)
    HIP_TRY(launch_fill_random(p->d_arena, P.arena_elems * p->eb, P.opts.dtype, nullptr), "fill arena");
  HIP_TRY(hipDeviceSynchronize(), "tuner synchronize");
  for (Op& op : P.ops) {
    if (op.kind != kOpGemm || op.gemm.gather_a) continue;
    std::string err;
    float* slot = op.max_slot >= 0 ? p->d_maxslots + op.max_slot : nullptr;
    float2* w = op.gemm.split_max > 1 ? reinterpret_cast<float2*>(resolve(p, op.w)) : nullptr;
    int rc = tune_gemm(P.opts.dtype, op.gemm, resolve(p, op.a), resolve(p, op.b), resolve(p, op.c), w, slot,
                       P.opts.tune_db, err);
    if (rc) return fail(rc, err);
    if (verbose())
      std::fprintf(stderr, "tnrcs: tuned GEMM %lld x %lld x %lld: tile %d split %d variant %d\n",
                   (long long)op.gemm.M, (long long)op.gemm.N, (long long)op.gemm.K, op.gemm.tile, op.gemm.split_k,
                   op.gemm.occ);
  }
  make_json(P);
  return TN_OK;
}

// Kernel-class autotuning (the permute/GEMM fusion choice).  A step whose
// shape admits more than one kernel class is run in each candidate class on
// a one-step plan with the same operand layouts over buffers of its own
// filled with random values; the fastest class overrides the planner's rule.
// Candidates: the gathered kernel (and the matrix-core skewed kernel where
// valid) against permutes + GEMM when the contraction is short (2^nK <=
// 2^kFuseMaxK terms), and gathered, split-K and the two skewed kernels
// against each other for steps too narrow for the GEMM.  Steps whose buffers would exceed
// the tuning budget (a third of the free device memory, at most
// kClassTuneMaxBytes) keep the rule.  Choices are cached per process and in
// the tuning database by dtype and the step's relabelled layouts.
constexpr int kFuseMaxK = 6;
constexpr int64_t kClassTuneMaxBytes = (int64_t)48 << 30;
constexpr int kGatherTuneLog2 = 22;
constexpr int kGatherTuneMaxK = 16;  // nor on sums of 2^16 terms or more (one output per thread)

// Average time of one run of a one-step plan's ops in class `cls` (INFINITY
// when the step does not fit the budget); builds, runs and frees the plan.
static int time_class(const PlanCore& P, const std::vector<int>& a, const std::vector<int>& b,
                      const std::vector<int>& c, int cls, int64_t budget, float* ms) {
  *ms = INFINITY;
  tn_plan_s q;
  PlanCore& Q = q.core;
  Q.pair_a = a;
  Q.pair_b = b;
  Q.pair_out = c;
  Q.opts = P.opts;
  Q.opts.tune = 0;
  Q.opts.arena = nullptr;
  Q.opts.arena_bytes = 0;
  Q.class_override[0] = cls;
  std::string err;
  int rc = build_pair_plan(Q, err);
  if (rc) return fail(rc, "class tuner: " + err);
  if (Q.steps.size() != 1 || Q.steps[0].cls != cls) return fail(TN_E_UNSUPPORTED, "class tuner: class not applied");
  q.eb = elem_bytes_of(Q.opts.dtype);
  q.device = P.opts.device;
  const int64_t na = (int64_t)1 << a.size(), nb = (int64_t)1 << b.size(), nc = (int64_t)1 << c.size();
  const int64_t bytes = (na + nb + nc + Q.arena_elems) * q.eb;
  if (bytes > budget) return TN_OK;
  char *A = nullptr, *B = nullptr, *C = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    hipFree(A);
    hipFree(B);
    hipFree(C);
    hipFree(q.d_arena);
    hipFree(q.d_maxslots);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  };
  hipError_t e = hipSuccess;
  const std::pair<char**, int64_t> bufs[] = {{&A, na}, {&B, nb}, {&C, nc}, {&q.d_arena, Q.arena_elems}};
  for (const auto& [ptr, n] : bufs)
    if (e == hipSuccess && (e = hipMalloc((void**)ptr, (size_t)std::max<int64_t>(n * q.eb, 256))) == hipSuccess)
      e = launch_fill_random(*ptr, std::max<int64_t>(n * q.eb, 256), Q.opts.dtype, nullptr);
  if (e == hipSuccess) e = hipMalloc((void**)&q.d_maxslots, (size_t)std::max(Q.n_slots, 1) * 4);
  if (e == hipSuccess) e = hipMemset(q.d_maxslots, 0, (size_t)std::max(Q.n_slots, 1) * 4);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "class tuner: allocate");
  }
  q.ext_a = A;
  q.ext_b = B;
  q.ext_c = C;
  // the GEMM of the dense class runs its own tuned variant
  for (Op& op : Q.ops)
    if (op.kind == kOpGemm && !op.gemm.gather_a && (rc = tune_gemm(Q.opts.dtype, op.gemm, resolve(&q, op.a), resolve(&q, op.b),
                                                resolve(&q, op.c),
                                                op.gemm.split_max > 1 ? (float2*)resolve(&q, op.w) : nullptr,
                                                op.max_slot >= 0 ? q.d_maxslots + op.max_slot : nullptr,
                                                P.opts.tune_db, err))) {
      cleanup();
      return fail(rc, err);
    }
  auto run = [&](int reps, float* out) -> int {
    HIP_TRY(hipEventRecord(e0, nullptr), "class tuner: event");
    for (int r = 0; r < reps; ++r)
      for (const Op& op : Q.ops) {
        int rc2 = launch_op(&q, op, nullptr);
        if (rc2) return rc2;
      }
    HIP_TRY(hipEventRecord(e1, nullptr), "class tuner: event");
    HIP_TRY(hipEventSynchronize(e1), "class tuner: synchronize");
    HIP_TRY(hipEventElapsedTime(out, e0, e1), "class tuner: elapsed time");
    return TN_OK;
  };
  float t1 = 0.f, tr = 0.f;
  rc = run(1, &t1);
  // repeat to about 2 ms of work (at most 20 runs)
  const int reps = std::max(1, std::min(20, (int)std::ceil(2.0 / std::max(t1, 1e-3f))));
  if (!rc) rc = run(reps, &tr);
  cleanup();
  if (!rc) *ms = tr / reps;
  return rc;
}

// measure = false (plans without device state): only the choices already in
// the process cache or the database apply.
static int tune_classes(PlanCore& P, bool measure) {
  size_t free_b = 0, total_b = 0;
  if (measure) HIP_TRY(hipMemGetInfo(&free_b, &total_b), "class tuner: hipMemGetInfo");
  const int64_t budget = std::min<int64_t>((int64_t)(free_b / 3), kClassTuneMaxBytes);
  bool changed = false;
  for (const PlanCore::StepInfo& st : P.steps) {
    const unsigned valid = step_classes(st.nM, st.nN, st.nK);
    std::vector<int> cand;
    // the gathered kernel (one output per thread, operands re-read per
    // output) is a candidate only for steps of at most 2^kGatherTuneLog2
    // outputs and sums shorter than 2^kGatherTuneMaxK: beyond that it loses
    // to every other class by far, and timing it would dominate the tuning
    // time
    const bool big = st.nM + st.nN > kGatherTuneLog2 || st.nK >= kGatherTuneMaxK;
    if (valid & (1u << kOpGemm)) {
      if (st.nK > kFuseMaxK) continue;
      cand = {kOpGemm};
      if (!big) cand.push_back(kOpGeneric);
      if (valid & (1u << kOpSkew)) cand.push_back(kOpSkew);
    } else {
      for (int k : {kOpGeneric, kOpSplitK, kOpSkinny, kOpSkew})
        if ((valid & (1u << k)) && !(k == kOpGeneric && big && valid != (1u << kOpGeneric))) cand.push_back(k);
    }
    if (cand.size() < 2) continue;
    const std::string& key = st.key;
    int best = -1;
    if (!class_lookup(P.opts.dtype, key, P.opts.tune_db, &best)) {
      if (!measure) continue;
      float best_ms = INFINITY;
      for (int k : cand) {
        float ms = INFINITY;
        int rc = time_class(P, st.la, st.lb, st.lc, k, budget, &ms);
        if (rc) return rc;
        if (ms < best_ms) {
          best_ms = ms;
          best = k;
        }
      }
      if (best < 0) continue;  // above the tuning budget: the rule stands
      class_store(P.opts.dtype, key, P.opts.tune_db, best, best_ms);
      if (verbose())
        std::fprintf(stderr, "tnrcs: class tuner: step %d (%d x %d x %d bits): class %d, %.3f ms\n", st.t, st.nM,
                     st.nN, st.nK, best, best_ms);
    }
    if (!(valid & (1u << best))) continue;
    P.class_override[st.t] = best;
    changed |= best != st.cls;
  }
  if (!changed) return TN_OK;
  std::string err;
  int rc = build_plan(P, err);
  return rc ? fail(rc, "rebuild after class tuning: " + err) : TN_OK;
}

static void drop_graph(tn_plan_s* p) {
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->graph) hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
}

static void release(tn_plan_s* p) {
  if (!p) return;
  if (p->core.opts.dry_run) return;
  hipSetDevice(p->device);
  drop_graph(p);
  if (p->cap_stream) hipStreamDestroy(p->cap_stream);
  hipFree(p->d_leaves);
  hipFree(p->d_bound);
  if (p->own_arena) hipFree(p->d_arena);
  hipFree(p->d_binds);
  hipFree(p->d_ctrl);
  hipFree(p->d_maxslots);
  hipFree(p->d_outscales);
  if (p->d_kappa) hipFree(p->d_kappa);
  if (p->d_stage) hipFree(p->d_stage);
}

extern "C" {

void tn_plan_opts_default(tn_plan_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->dtype = TN_DTYPE_C64;
  o->gemm_form = TN_GEMM_AUTO;
  o->max_log2 = 0;
  o->use_graph = 1;
  o->dry_run = 0;
  o->device = 0;
  o->host_fold_log2 = 12;
  o->arena_bytes = 0;
}

const char* tn_last_error(void) { return g_err.c_str(); }

int tn_plan(const tn_circuit* c, const int32_t* order_pairs, int32_t n_steps, const int32_t* sliced_wires,
            int32_t k, const int32_t* open_qubits, int32_t n_open, const tn_plan_opts* opts, tn_plan_t* out) {
  if (!out) return fail(TN_E_ARG, "out is NULL");
  *out = nullptr;
  if (!c) return fail(TN_E_ARG, "circuit is NULL");
  if (c->n_qubits < 1 || c->n_qubits > 4096) return fail(TN_E_ARG, "n_qubits out of range");
  if (c->n_gates < 0 || (c->n_gates > 0 && !c->gates)) return fail(TN_E_ARG, "bad gate list");
  if (n_steps < 0 || (n_steps > 0 && !order_pairs)) return fail(TN_E_ARG, "bad order");
  if (k < 0 || k > 62 || (k > 0 && !sliced_wires)) return fail(TN_E_ARG, "bad sliced-wire list");
  if (n_open < 0 || n_open > 40 || (n_open > 0 && !open_qubits)) return fail(TN_E_ARG, "bad open-qubit list");
  tn_plan_opts o;
  if (opts)
    o = *opts;
  else
    tn_plan_opts_default(&o);
  if (o.dtype != TN_DTYPE_C64 && o.dtype != TN_DTYPE_F16S && o.dtype != TN_DTYPE_BF16S)
    return fail(TN_E_ARG, "unknown dtype");
  if (o.host_fold_log2 < 0 || o.host_fold_log2 > 20) return fail(TN_E_ARG, "host_fold_log2 out of range");
  for (int g = 0; g < c->n_gates; ++g) {
    const tn_gate& G = c->gates[g];
    if (G.nq != 1 && G.nq != 2) return fail(TN_E_ARG, "gate " + std::to_string(g) + ": nq must be 1 or 2");
    for (int j = 0; j < G.nq; ++j)
      if (G.q[j] < 0 || G.q[j] >= c->n_qubits)
        return fail(TN_E_ARG, "gate " + std::to_string(g) + ": qubit out of range");
    if (G.nq == 2 && G.q[0] == G.q[1]) return fail(TN_E_ARG, "gate " + std::to_string(g) + ": repeated qubit");
  }
  std::vector<bool> seen(c->n_qubits, false);
  for (int i = 0; i < n_open; ++i) {
    int q = open_qubits[i];
    if (q < 0 || q >= c->n_qubits) return fail(TN_E_ARG, "open qubit out of range");
    if (seen[q]) return fail(TN_E_ARG, "open qubit listed twice");
    seen[q] = true;
  }
  if (n_open < c->n_qubits && !c->out_bits) return fail(TN_E_ARG, "out_bits is NULL but some qubits are closed");

  tn_plan_s* p = new (std::nothrow) tn_plan_s();
  if (!p) return fail(TN_E_MEM, "host allocation failed");
  PlanCore& P = p->core;
  P.n_qubits = c->n_qubits;
  P.gates.assign(c->gates, c->gates + c->n_gates);
  if (c->out_bits) P.out_bits.assign(c->out_bits, c->out_bits + c->n_qubits);
  P.pairs.assign(order_pairs, order_pairs + 2 * n_steps);
  P.sliced.assign(sliced_wires, sliced_wires + k);
  P.open_q.assign(open_qubits, open_qubits + n_open);
  P.opts = o;
  std::string err;
  int rc = build_plan(P, err);
  if (rc) {
    delete p;
    return fail(rc, err);
  }
  p->device = o.device;
  p->eb = elem_bytes_of(o.dtype);
  if (o.dry_run) {
    if (o.tune && (rc = tune_classes(P, false))) {
      delete p;
      return rc;
    }
    if (o.dtype != TN_DTYPE_C64) leaf_exponents(P);
    propagate_exponents(P);
    *out = p;
    return TN_OK;
  }
  // device side
  auto bail = [&](int code) {
    release(p);
    delete p;
    return code;
  };
  hipError_t e = hipSetDevice(o.device);
  if (e != hipSuccess) return bail(hip_fail(e, "hipSetDevice"));
  if (o.tune && (rc = tune_classes(P, true))) return bail(rc);
  size_t free_b = 0, total_b = 0;
  e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) return bail(hip_fail(e, "hipMemGetInfo"));
  const bool ext_arena = o.arena != nullptr;
  if (ext_arena) {
    if ((reinterpret_cast<uintptr_t>(o.arena) & 255) != 0) return bail(fail(TN_E_ARG, "arena not 256-byte aligned"));
    if (P.arena_elems * (int64_t)p->eb > o.arena_bytes)
      return bail(fail(TN_E_MEM, "plan needs an arena of " + std::to_string(P.arena_elems * (int64_t)p->eb) +
                                     " bytes, workspace has " + std::to_string(o.arena_bytes)));
  }
  const int64_t need = ((ext_arena ? 0 : P.arena_elems) + P.leaves_elems + P.bound_elems) * (int64_t)p->eb;
  const int64_t budget =
      (!ext_arena && o.arena_bytes > 0) ? o.arena_bytes : (int64_t)(0.92 * (double)free_b);
  if (need > budget)
    return bail(fail(TN_E_MEM, "plan needs " + std::to_string(need) + " device bytes, budget " + std::to_string(budget)));
  auto dmalloc = [&](void** ptr, int64_t bytes, const char* what) -> int {
    if (bytes <= 0) bytes = 256;
    hipError_t e2 = hipMalloc(ptr, (size_t)bytes);
    if (e2 != hipSuccess) return hip_fail(e2, what);
    return TN_OK;
  };
  if ((rc = dmalloc((void**)&p->d_leaves, P.leaves_elems * p->eb, "alloc leaves")) ||
      (rc = dmalloc((void**)&p->d_bound, P.bound_elems * p->eb, "alloc bound leaves")) ||
      (!ext_arena && (rc = dmalloc((void**)&p->d_arena, P.arena_elems * p->eb, "alloc arena"))) ||
      (rc = dmalloc((void**)&p->d_maxslots, (int64_t)std::max(P.n_slots, 1) * 4, "alloc records")) ||
      (rc = dmalloc((void**)&p->d_outscales, (int64_t)std::max(P.n_slots, 1) * 4, "alloc scales")) ||
      (rc = dmalloc((void**)&p->d_binds, (int64_t)P.binds.size() * (int64_t)sizeof(BindDesc), "alloc binds")) ||
      (rc = dmalloc((void**)&p->d_ctrl, sizeof(Ctrl), "alloc control")))
    return bail(rc);
  if (ext_arena) {
    p->d_arena = static_cast<char*>(o.arena);
    p->own_arena = false;
  }
  if ((rc = upload_leaves(p))) return bail(rc);
  if (!P.binds.empty()) {
    e = hipMemcpy(p->d_binds, P.binds.data(), P.binds.size() * sizeof(BindDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(hip_fail(e, "upload binds"));
    for (auto& b : P.binds) p->bind_max = std::max(p->bind_max, b.n_elems);
  }
  Ctrl zero{};
  e = hipMemcpy(p->d_ctrl, &zero, sizeof(Ctrl), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bail(hip_fail(e, "init control"));
  if (o.tune && (rc = tune_plan(p))) return bail(rc);
  if ((rc = calibrate(p))) return bail(rc);
  e = hipMemcpy(p->d_ctrl, &zero, sizeof(Ctrl), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bail(hip_fail(e, "init control"));
  *out = p;
  return TN_OK;
}

int tn_pair_plan(int32_t rank_a, const int32_t* labels_a, int32_t rank_b, const int32_t* labels_b, int32_t rank_c,
                 const int32_t* labels_c, const tn_plan_opts* opts, tn_plan_t* out) {
  if (!out) return fail(TN_E_ARG, "out is NULL");
  *out = nullptr;
  if (rank_a < 0 || rank_b < 0 || rank_c < 0 || rank_a > 40 || rank_b > 40 || rank_c > 40 ||
      (rank_a && !labels_a) || (rank_b && !labels_b) || (rank_c && !labels_c))
    return fail(TN_E_ARG, "bad label list");
  tn_plan_opts o;
  if (opts)
    o = *opts;
  else
    tn_plan_opts_default(&o);
  if (o.dtype != TN_DTYPE_C64 && o.dtype != TN_DTYPE_F16S && o.dtype != TN_DTYPE_BF16S)
    return fail(TN_E_ARG, "unknown dtype");
  tn_plan_s* p = new (std::nothrow) tn_plan_s();
  if (!p) return fail(TN_E_MEM, "host allocation failed");
  PlanCore& P = p->core;
  P.pair_a.assign(labels_a, labels_a + rank_a);
  P.pair_b.assign(labels_b, labels_b + rank_b);
  P.pair_out.assign(labels_c, labels_c + rank_c);
  o.tune = 0;
  o.arena = nullptr;
  o.tune_db = nullptr;
  P.opts = o;
  std::string err;
  int rc = build_pair_plan(P, err);
  if (rc) {
    delete p;
    return fail(rc, err);
  }
  p->device = o.device;
  p->eb = elem_bytes_of(o.dtype);
  if (o.dry_run) {
    *out = p;
    return TN_OK;
  }
  auto bail = [&](int code) {
    release(p);
    delete p;
    return code;
  };
  hipError_t e = hipSetDevice(o.device);
  if (e != hipSuccess) return bail(hip_fail(e, "hipSetDevice"));
  if ((e = hipMalloc((void**)&p->d_arena, (size_t)std::max<int64_t>(P.arena_elems * p->eb, 256))) != hipSuccess ||
      (e = hipMalloc((void**)&p->d_maxslots, (size_t)std::max(P.n_slots, 1) * 4)) != hipSuccess)
    return bail(hip_fail(e, "alloc pair workspace"));
  std::vector<float> zero(std::max(P.n_slots, 1), 0.f);
  if ((e = hipMemcpy(p->d_maxslots, zero.data(), zero.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return bail(hip_fail(e, "clear records"));
  *out = p;
  return TN_OK;
}

int tn_pair_run(tn_plan_t p, const void* A, const void* B, void* C, int64_t batch, float out_scale, void* stream) {
  if (!p || !A || !B || !C) return fail(TN_E_ARG, "NULL argument");
  if (!p->core.pair_mode) return fail(TN_E_ARG, "not a pairwise plan");
  if (p->core.opts.dry_run) return fail(TN_E_UNSUPPORTED, "dry-run plan has no device state");
  if (batch < 0) return fail(TN_E_ARG, "batch < 0");
  if (p->core.opts.dtype == TN_DTYPE_C64 && out_scale != 1.f) return fail(TN_E_ARG, "out_scale must be 1 for complex64");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(p->device), "hipSetDevice");
  PlanCore& P = p->core;
  for (Op& op : P.ops) {
    op.gemm.out_scale = out_scale;
    op.idx.out_scale = out_scale;
  }
  const int64_t sa = ((int64_t)1 << P.pair_a.size()) * p->eb, sb = ((int64_t)1 << P.pair_b.size()) * p->eb,
                sc = ((int64_t)1 << P.pair_out.size()) * p->eb;
  for (int64_t i = 0; i < batch; ++i) {
    p->ext_a = (const char*)A + i * sa;
    p->ext_b = (const char*)B + i * sb;
    p->ext_c = (char*)C + i * sc;
    for (const Op& op : P.ops) {
      int rc = launch_op(p, op, s);
      if (rc) return rc;
    }
  }
  p->last_stream = s;
  p->ran = true;
  return TN_OK;
}

// Runs `count` slices from the cursor on, replaying the per-slice graph
// (captured on first use) or enqueueing the kernels directly.
// Captures the plan's per-slice graph once (plans with opts.use_graph).
static int ensure_graph(tn_plan_s* p) {
  if (!p->core.opts.use_graph || p->exec) return TN_OK;
  if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking), "create capture stream");
  HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  int rc = enqueue_slice(p, p->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
  if (rc) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  p->graph = g;
  HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0), "instantiate graph");
  return TN_OK;
}

static int run_slices(tn_plan_s* p, int64_t count, hipStream_t s) {
  if (p->core.opts.use_graph) {
    if (int rc = ensure_graph(p)) return rc;
    for (int64_t i = 0; i < count; ++i) HIP_TRY(hipGraphLaunch(p->exec, s), "graph launch");
  } else {
    for (int64_t i = 0; i < count; ++i) {
      int rc = enqueue_slice(p, s);
      if (rc) return rc;
    }
  }
  return TN_OK;
}

int tn_contract_slices(tn_plan_t p, int64_t s_begin, int64_t s_end, void* amp, void* stream) {
  if (!p) return fail(TN_E_ARG, "plan is NULL");
  if (p->core.pair_mode) return fail(TN_E_ARG, "pairwise plan: use tn_pair_run");
  if (p->core.opts.dry_run) return fail(TN_E_UNSUPPORTED, "dry-run plan has no device state");
  if (!amp) return fail(TN_E_ARG, "amp is NULL");
  const int64_t ns = p->core.stats.n_slices;
  if (s_begin < 0 || s_end < s_begin || s_end > ns)
    return fail(TN_E_ARG, "slice range [" + std::to_string(s_begin) + ", " + std::to_string(s_end) +
                              ") outside [0, " + std::to_string(ns) + ")");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(p->device), "hipSetDevice");
  p->last_stream = s;
  p->ran = true;
  if (s_end == s_begin) return TN_OK;
  HIP_TRY(launch_set_ctrl(p->d_ctrl, s_begin, amp, s), "control kernel");
  return run_slices(p, s_end - s_begin, s);
}

int tn_contract_slices_checked(tn_plan_t p, int64_t s_begin, int64_t s_end, void* amp, void* stream,
                               int32_t* retries) {
  if (!p) return fail(TN_E_ARG, "plan is NULL");
  if (p->core.pair_mode) return fail(TN_E_ARG, "pairwise plan: use tn_pair_run");
  if (p->core.opts.dry_run) return fail(TN_E_UNSUPPORTED, "dry-run plan has no device state");
  if (!amp) return fail(TN_E_ARG, "amp is NULL");
  const int64_t ns = p->core.stats.n_slices;
  if (s_begin < 0 || s_end < s_begin || s_end > ns)
    return fail(TN_E_ARG, "slice range [" + std::to_string(s_begin) + ", " + std::to_string(s_end) +
                              ") outside [0, " + std::to_string(ns) + ")");
  if (retries) *retries = 0;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(p->device), "hipSetDevice");
  const int64_t n_amp = (int64_t)1 << p->core.accum.n_open;
  if (!p->d_stage) HIP_TRY(hipMalloc((void**)&p->d_stage, (size_t)n_amp * 16), "alloc staging bunch");
  HIP_TRY(hipStreamSynchronize(s), "stream synchronize");
  if (p->ran && p->last_stream != s) HIP_TRY(hipStreamSynchronize(p->last_stream), "stream synchronize");
  p->last_stream = s;
  p->ran = true;
  Ctrl c{};
  HIP_TRY(hipMemcpy(&c, p->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost), "read control");
  uint32_t sticky = c.flags;
  const bool scaled = p->core.opts.dtype != TN_DTYPE_C64;
  int rc = TN_OK;
  for (int64_t sl = s_begin; sl < s_end && rc == TN_OK; ++sl) {
    for (int attempt = 0;; ++attempt) {
      HIP_TRY(hipMemsetAsync(p->d_stage, 0, (size_t)n_amp * 16, s), "clear staging bunch");
      HIP_TRY(launch_set_ctrl(p->d_ctrl, sl, p->d_stage, s, true), "control kernel");
      if ((rc = run_slices(p, 1, s))) break;
      HIP_TRY(hipStreamSynchronize(s), "stream synchronize");
      HIP_TRY(hipMemcpy(&c, p->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost), "read control");
      const uint32_t range = c.flags & (TN_FLAG_OVERFLOW | TN_FLAG_UNDERFLOW);
      if (c.flags == 0) {
        HIP_TRY(launch_add_amp(p->d_stage, (double*)amp, n_amp, s), "add slice");
        break;
      }
      if (scaled && range && attempt == 0) {
        // the shifts calibrated on slice 0 do not fit this slice: calibrate
        // on it (every later slice keeps the new shifts) and run it again
        if ((rc = calibrate(p, sl))) break;
        drop_graph(p);  // the captured kernels hold the old output scales
        if (retries) ++*retries;
        continue;
      }
      sticky |= c.flags;
      rc = fail(TN_E_NUMERIC, "slice " + std::to_string(sl) + ": numeric flags " + std::to_string(c.flags) +
                                  (attempt ? " persist after recalibration" : ""));
      break;
    }
  }
  HIP_TRY(hipStreamSynchronize(s), "stream synchronize");
  HIP_TRY(hipMemcpy(reinterpret_cast<char*>(p->d_ctrl) + offsetof(Ctrl, flags), &sticky, sizeof(uint32_t),
                    hipMemcpyHostToDevice),
          "restore flags");
  return rc;
}

int tn_plan_shift_outputs(tn_plan_t p, int32_t op_index, int32_t delta) {
  if (!p) return fail(TN_E_ARG, "plan is NULL");
  PlanCore& P = p->core;
  if (P.pair_mode) return fail(TN_E_ARG, "pairwise plan");
  if (P.opts.dtype == TN_DTYPE_C64) return fail(TN_E_ARG, "complex64 plans have no output shifts");
  if (delta < -64 || delta > 64) return fail(TN_E_ARG, "delta out of range");
  if (op_index >= (int32_t)P.ops.size()) return fail(TN_E_ARG, "kernel index out of range");
  if (op_index >= 0 && P.ops[op_index].max_slot < 0) return fail(TN_E_ARG, "kernel has no output shift");
  for (size_t i = 0; i < P.ops.size(); ++i) {
    Op& op = P.ops[i];
    if (op.max_slot < 0 || (op_index >= 0 && (int32_t)i != op_index)) continue;
    op.s_out += delta;
    const float sc = (float)std::ldexp(1.0, -op.s_out);
    op.gemm.out_scale = sc;
    op.idx.out_scale = sc;
  }
  propagate_exponents(P);
  make_json(P);
  if (P.opts.dry_run) return TN_OK;
  HIP_TRY(hipSetDevice(p->device), "hipSetDevice");
  if (p->ran) HIP_TRY(hipStreamSynchronize(p->last_stream), "stream synchronize");
  drop_graph(p);
  return upload_scales(p);
}

int tn_batch_create(const tn_plan_t* plans, int32_t n, const int64_t* ranges, void* const* amps, tn_batch_t* out) {
  if (!out) return fail(TN_E_ARG, "out is NULL");
  *out = nullptr;
  if (n < 0 || (n > 0 && (!plans || !ranges || !amps))) return fail(TN_E_ARG, "bad batch lists");
  int device = -1;
  bool work = false;
  for (int i = 0; i < n; ++i) {
    const tn_plan_s* p = plans[i];
    const std::string at = "batch entry " + std::to_string(i) + ": ";
    if (!p) return fail(TN_E_ARG, at + "plan is NULL");
    if (p->core.pair_mode) return fail(TN_E_ARG, at + "pairwise plan");
    if (p->core.opts.dry_run) return fail(TN_E_UNSUPPORTED, at + "dry-run plan has no device state");
    if (device >= 0 && p->device != device) return fail(TN_E_ARG, at + "plans on different devices");
    device = p->device;
    const int64_t b = ranges[2 * i], e = ranges[2 * i + 1];
    if (b < 0 || e < b || e > p->core.stats.n_slices)
      return fail(TN_E_ARG, at + "slice range outside [0, " + std::to_string(p->core.stats.n_slices) + ")");
    if (e > b && !amps[i]) return fail(TN_E_ARG, at + "amp is NULL");
    work |= e > b;
  }
  tn_batch_s* b = new (std::nothrow) tn_batch_s();
  if (!b) return fail(TN_E_MEM, "host allocation failed");
  b->plans.assign(plans, plans + n);
  b->ranges.assign(ranges, ranges + 2 * (int64_t)n);
  b->amps.assign(amps, amps + n);
  b->device = device < 0 ? 0 : device;
  if (!work) {
    *out = b;
    return TN_OK;
  }
  auto bail = [&](int code) {
    batch_release(b);
    delete b;
    return code;
  };
  // lanes: plans whose arenas overlap (or that share a plan or an output
  // buffer) run one after another in one lane; different lanes are
  // independent and may run side by side
  std::vector<int> lane(n);
  for (int i = 0; i < n; ++i) lane[i] = i;
  std::function<int(int)> root = [&](int i) { return lane[i] == i ? i : (lane[i] = root(lane[i])); };
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      const tn_plan_s *p = plans[i], *q = plans[j];
      const char *pa = p->d_arena, *qa = q->d_arena;
      const int64_t pn = p->core.arena_elems * p->eb, qn = q->core.arena_elems * q->eb;
      const bool overlap = pn > 0 && qn > 0 && pa < qa + qn && qa < pa + pn;
      if (overlap || p == q || amps[i] == amps[j]) lane[root(i)] = root(j);
    }
  std::vector<int> lane_of(n), first_of;  // dense lane ids in order of first appearance
  for (int i = 0; i < n; ++i) {
    const int r = root(i);
    int id = -1;
    for (size_t k = 0; k < first_of.size(); ++k)
      if (first_of[k] == r) id = (int)k;
    if (id < 0) {
      id = (int)first_of.size();
      first_of.push_back(r);
    }
    lane_of[i] = id;
  }
  const int n_lanes = std::max<int>(1, std::min<int>((int)first_of.size(), kBatchMaxLanes));
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return bail(hip_fail(e, "hipSetDevice"));
  for (int k = 0; k < n_lanes; ++k) {
    std::vector<int> mine;
    for (int i = 0; i < n; ++i)
      if (lane_of[i] % n_lanes == k && ranges[2 * i + 1] > ranges[2 * i]) mine.push_back(i);
    if (!mine.empty()) b->lanes.push_back(mine);
  }
  // every plan's per-slice graph is captured now, so that a run only replays
  for (int i = 0; i < n; ++i)
    if (ranges[2 * i + 1] > ranges[2 * i])
      if (int rc = ensure_graph(plans[i])) return bail(rc);
  // each lane gets a stream of its own, created one after the other so that
  // the runtime spreads them over its hardware queues
  for (size_t k = 0; k < b->lanes.size(); ++k) {
    hipStream_t st = nullptr;
    hipEvent_t f = nullptr, j = nullptr;
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) == hipSuccess) b->lane_streams.push_back(st);
    if (e == hipSuccess && (e = hipEventCreateWithFlags(&f, hipEventDisableTiming)) == hipSuccess)
      b->fork.push_back(f);
    if (e == hipSuccess && (e = hipEventCreateWithFlags(&j, hipEventDisableTiming)) == hipSuccess)
      b->join.push_back(j);
    if (e != hipSuccess) return bail(hip_fail(e, "create lane stream"));
  }
  *out = b;
  return TN_OK;
}

int tn_batch_run(tn_batch_t b, void* stream) {
  if (!b) return fail(TN_E_ARG, "batch is NULL");
  hipStream_t s = (hipStream_t)stream;
  for (tn_plan_s* p : b->plans) {
    p->last_stream = s;
    p->ran = true;
  }
  if (b->lanes.empty()) return TN_OK;
  HIP_TRY(hipSetDevice(b->device), "hipSetDevice");
  // the lanes start after the work already on the caller's stream, and the
  // caller's stream then waits for every lane; in a lane, each plan sets its
  // slice cursor and replays its per-slice graph
  for (size_t k = 0; k < b->lanes.size(); ++k) {
    HIP_TRY(hipEventRecord(b->fork[k], s), "batch fork");
    HIP_TRY(hipStreamWaitEvent(b->lane_streams[k], b->fork[k], 0), "batch fork");
  }
  // plans are issued to the lanes in turn (the j-th plan of every lane, then
  // the (j+1)-th), so that every lane has work queued from the start
  size_t longest = 0;
  for (const std::vector<int>& l : b->lanes) longest = std::max(longest, l.size());
  for (size_t j = 0; j < longest; ++j)
    for (size_t k = 0; k < b->lanes.size(); ++k) {
      if (j >= b->lanes[k].size()) continue;
      const int i = b->lanes[k][j];
      tn_plan_s* p = b->plans[i];
      const int64_t s0 = b->ranges[2 * i], s1 = b->ranges[2 * i + 1];
      HIP_TRY(launch_set_ctrl(p->d_ctrl, s0, b->amps[i], b->lane_streams[k]), "control kernel");
      if (int rc = run_slices(p, s1 - s0, b->lane_streams[k])) return rc;
    }
  for (size_t k = 0; k < b->lanes.size(); ++k) {
    HIP_TRY(hipEventRecord(b->join[k], b->lane_streams[k]), "batch join");
    HIP_TRY(hipStreamWaitEvent(s, b->join[k], 0), "batch join");
  }
  return TN_OK;
}

int tn_batch_destroy(tn_batch_t b) {
  if (!b) return TN_OK;
  hipSetDevice(b->device);
  batch_release(b);
  delete b;
  return TN_OK;
}

int tn_contract_batch(const tn_plan_t* plans, const int64_t* ranges, void* const* amps, int32_t n, void* stream) {
  tn_batch_t b = nullptr;
  int rc = tn_batch_create(plans, n, ranges, amps, &b);
  if (rc) return rc;
  rc = tn_batch_run(b, stream);
  if (rc == TN_OK) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) rc = hip_fail(e, "batch synchronize");
  }
  tn_batch_destroy(b);
  return rc;
}

int tn_plan_profile(tn_plan_t p, int64_t slice, void* amp, void* stream, float* op_ms, int32_t cap,
                    int32_t* n_ops) {
  if (!p || !amp || !n_ops) return fail(TN_E_ARG, "NULL argument");
  if (p->core.opts.dry_run) return fail(TN_E_UNSUPPORTED, "dry-run plan has no device state");
  const PlanCore& P = p->core;
  const int nk = (int)P.ops.size() + 1;
  *n_ops = nk;
  if (!op_ms || cap < nk) return fail(TN_E_ARG, "op_ms capacity below the kernel count");
  if (slice < 0 || slice >= P.stats.n_slices) return fail(TN_E_ARG, "slice out of range");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(p->device), "hipSetDevice");
  p->last_stream = s;
  p->ran = true;
  std::vector<hipEvent_t> ev(nk + 1, nullptr);
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e), "event create");
  int rc = TN_OK;
  auto body = [&]() -> int {
    HIP_TRY(launch_set_ctrl(p->d_ctrl, slice, amp, s), "control kernel");
    int rc1 = launch_bind_slice(p, s);
    if (rc1) return rc1;
    for (int i = 0; i < (int)P.ops.size(); ++i) {
      HIP_TRY(hipEventRecord(ev[i], s), "event record");
      int rc2 = launch_op(p, P.ops[i], s);
      if (rc2) return rc2;
    }
    HIP_TRY(hipEventRecord(ev[nk - 1], s), "event record");
    int rc3 = launch_accum_slice(p, s);
    if (rc3) return rc3;
    HIP_TRY(hipEventRecord(ev[nk], s), "event record");
    HIP_TRY(hipEventSynchronize(ev[nk]), "event synchronize");
    for (int i = 0; i < nk; ++i) HIP_TRY(hipEventElapsedTime(&op_ms[i], ev[i], ev[i + 1]), "event elapsed");
    return TN_OK;
  };
  rc = body();
  for (auto& e : ev)
    if (e) hipEventDestroy(e);
  return rc;
}

int tn_plan_info(tn_plan_t p, tn_plan_stats* s) {
  if (!p || !s) return fail(TN_E_ARG, "NULL argument");
  *s = p->core.stats;
  return TN_OK;
}

int tn_plan_json(tn_plan_t p, char* buf, int64_t cap, int64_t* needed) {
  if (!p) return fail(TN_E_ARG, "plan is NULL");
  const std::string& j = p->core.json;
  if (needed) *needed = (int64_t)j.size() + 1;
  if (buf) {
    if (cap < (int64_t)j.size() + 1) return fail(TN_E_ARG, "buffer too small");
    std::memcpy(buf, j.c_str(), j.size() + 1);
  }
  return TN_OK;
}

int tn_plan_leaf(tn_plan_t p, int32_t i, double* out, int64_t cap) {
  if (!p || !out) return fail(TN_E_ARG, "NULL argument");
  if (i < 0 || i >= (int32_t)p->core.dev_leaves.size()) return fail(TN_E_ARG, "leaf index out of range");
  const DevLeaf& d = p->core.dev_leaves[i];
  if (cap < 2 * (int64_t)d.data.size()) return fail(TN_E_ARG, "buffer too small");
  for (size_t j = 0; j < d.data.size(); ++j) {
    out[2 * j] = d.data[j].real();
    out[2 * j + 1] = d.data[j].imag();
  }
  return TN_OK;
}

int tn_plan_status(tn_plan_t p, uint32_t* flags) {
  if (!p || !flags) return fail(TN_E_ARG, "NULL argument");
  *flags = 0;
  if (p->core.opts.dry_run || !p->ran) return TN_OK;
  HIP_TRY(hipSetDevice(p->device), "hipSetDevice");
  HIP_TRY(hipStreamSynchronize(p->last_stream), "stream synchronize");
  Ctrl c{};
  HIP_TRY(hipMemcpy(&c, p->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost), "read control");
  *flags = c.flags;
  return TN_OK;
}

int tn_plan_set_output_bits(tn_plan_t p, const uint8_t* out_bits) {
  if (!p || !out_bits) return fail(TN_E_ARG, "NULL argument");
  PlanCore& P = p->core;
  P.out_bits.assign(out_bits, out_bits + P.n_qubits);
  std::string err;
  int rc = refold_leaves(P, err);
  if (rc) return fail(rc, err);
  if (P.opts.dry_run) return TN_OK;
  HIP_TRY(hipSetDevice(p->device), "hipSetDevice");
  if (p->ran) HIP_TRY(hipStreamSynchronize(p->last_stream), "stream synchronize");
  rc = upload_leaves(p);
  if (rc) return rc;
  propagate_exponents(P);  // leaf exponents may have moved: new root scale
  drop_graph(p);           // the captured accumulation holds the old scale
  return TN_OK;
}

int tn_plan_destroy(tn_plan_t p) {
  if (!p) return TN_OK;
  if (!p->core.opts.dry_run && p->ran) {
    hipSetDevice(p->device);
    hipStreamSynchronize(p->last_stream);
  }
  release(p);
  delete p;
  return TN_OK;
}

int tn_permute(const void* in, void* out, int32_t elem_bytes, int32_t rank, const int32_t* perm, int64_t batch,
               void* stream) {
  if (!in || !out || !perm) return fail(TN_E_ARG, "NULL argument");
  if (elem_bytes != 4 && elem_bytes != 8) return fail(TN_E_ARG, "elem_bytes must be 4 or 8");
  if (rank < 0 || rank > 40 || batch < 0 || batch > 65535) return fail(TN_E_ARG, "rank or batch out of range");
  hipError_t e = launch_permute(elem_bytes, in, out, rank, perm, batch, (hipStream_t)stream);
  if (e == hipErrorInvalidValue) return fail(TN_E_ARG, "perm is not a permutation of 0..rank-1");
  if (e != hipSuccess) return hip_fail(e, "permute kernel");
  return TN_OK;
}

int tn_cgemm_half(int32_t dtype, const void* A, const void* B, void* C, int64_t M, int64_t N, int64_t K,
                  int64_t batch, int32_t form, float out_scale, void* work, int32_t splits, void* max_out,
                  void* stream) {
  if (!A || !B || !C) return fail(TN_E_ARG, "NULL argument");
  if (dtype != TN_DTYPE_F16S && dtype != TN_DTYPE_BF16S) return fail(TN_E_ARG, "dtype must be F16S or BF16S");
  if (form != TN_GEMM_4M && form != TN_GEMM_3M) return fail(TN_E_ARG, "form must be TN_GEMM_4M or TN_GEMM_3M");
  if (!hgemm_shape_ok(M, N, K) || batch < 0 || batch > 65535)
    return fail(TN_E_ARG, "shape not supported: M, N multiples of 64, K a multiple of 16");
  if (splits > 1 && (!work || batch != 1 || K % (16 * (int64_t)splits)))
    return fail(TN_E_ARG, "split-K needs work, batch 1 and K a multiple of 16*splits");
  hipError_t e = launch_gemm_half(dtype, A, B, C, M, N, K, batch, form, (hipStream_t)stream, (float2*)work,
                                  splits < 1 ? 1 : splits, out_scale, (float*)max_out);
  if (e != hipSuccess) return hip_fail(e, "half gemm kernel");
  return TN_OK;
}

}  // extern "C"

// ---- allocation-free split-K GEMM: the slab workspace is a static device array ----

namespace {

constexpr int64_t kScratchBytes = TN_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Split-K slabs of tn_cgemm_c64_noalloc.  Each device holds its own copy for
// the life of the process.  In host code this name is only a handle for
// hipGetSymbolAddress; kernels get the per-device address below.
static __device__ __align__(256) float2 scratch[kScratchBytes / sizeof(float2)];

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int scratch_address(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(TN_E_UNSUPPORTED, "device ordinal above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(TN_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return TN_OK;
}

}  // namespace

extern "C" {

int tn_cgemm_c64_noalloc(const void* A, const void* B, void* C, int64_t M, int64_t N, int64_t K, int32_t form,
                         int32_t splits, void* stream) {
  if (!A || !B || !C) return fail(TN_E_ARG, "NULL argument");
  if (form != TN_GEMM_4M && form != TN_GEMM_3M) return fail(TN_E_ARG, "form must be TN_GEMM_4M or TN_GEMM_3M");
  if (!gemm_shape_ok(M, N, K)) return fail(TN_E_ARG, "shape not supported: M, N multiples of 64, K a multiple of 16");
  if (splits < 1) splits = 1;
  void* work = nullptr;
  if (splits > 1) {
    if (M % 128 || N % 128 || K % (16 * (int64_t)splits))
      return fail(TN_E_ARG, "split-K needs M and N multiples of 128 and K a multiple of 16*splits");
    const int64_t need = (int64_t)splits * M * N * (int64_t)sizeof(float2);
    if (need > kScratchBytes)
      return fail(TN_E_ARG, "split-K slabs need " + std::to_string(need) + " bytes; the static scratch holds " +
                                std::to_string(kScratchBytes) + " (splits * M * N <= " +
                                std::to_string(kScratchBytes / 8) + ")");
    int rc = scratch_address(&work);
    if (rc) return rc;
  }
  hipError_t e = launch_gemm_c64((const float2*)A, (const float2*)B, (float2*)C, M, N, K, 1, form,
                                 (hipStream_t)stream, (float2*)work, splits);
  if (e != hipSuccess) return hip_fail(e, "gemm kernel");
  return TN_OK;
}

int tn_cgemm_c64(const void* A, const void* B, void* C, int64_t M, int64_t N, int64_t K, int64_t batch,
                 int32_t form, void* work, int32_t splits, void* stream) {
  if (!A || !B || !C) return fail(TN_E_ARG, "NULL argument");
  if (form != TN_GEMM_4M && form != TN_GEMM_3M) return fail(TN_E_ARG, "form must be TN_GEMM_4M or TN_GEMM_3M");
  if (!gemm_shape_ok(M, N, K) || batch < 0)
    return fail(TN_E_ARG, "shape not supported: M, N multiples of 64, K a multiple of 16");
  if (splits > 1 && (!work || batch != 1 || K % (16 * (int64_t)splits)))
    return fail(TN_E_ARG, "split-K needs work, batch 1 and K a multiple of 16*splits");
  hipError_t e = launch_gemm_c64((const float2*)A, (const float2*)B, (float2*)C, M, N, K, batch, form,
                                 (hipStream_t)stream, (float2*)work, splits < 1 ? 1 : splits);
  if (e != hipSuccess) return hip_fail(e, "gemm kernel");
  return TN_OK;
}

int64_t tn_probe_mfma_out_floats(void) { return mfma_peak_out_floats(); }

int tn_probe_mfma(int32_t kind, int64_t iters, void* out_dev, double* flops, void* stream) {
  if (kind < 0 || kind > 2) return fail(TN_E_ARG, "kind must be 0, 1 or 2");
  if (iters < 1 || iters > ((int64_t)1 << 24)) return fail(TN_E_ARG, "iters out of range");
  if (!out_dev || !flops) return fail(TN_E_ARG, "NULL argument");
  HIP_TRY(launch_mfma_peak(kind, iters, (float*)out_dev, flops, (hipStream_t)stream), "MFMA probe");
  return TN_OK;
}

int tn_probe_copy(const void* src, void* dst, int64_t bytes, void* stream) {
  if (!src || !dst) return fail(TN_E_ARG, "NULL argument");
  if (bytes < 0 || bytes % 16) return fail(TN_E_ARG, "bytes must be a non-negative multiple of 16");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
    return fail(TN_E_ARG, "buffers must be 16-byte aligned");
  HIP_TRY(launch_stream_copy(src, dst, bytes / 16, (hipStream_t)stream), "copy probe");
  return TN_OK;
}

int tn_amp_norm2(const void* amp, int64_t n, void* out_dev, void* stream) {
  if (!amp || !out_dev || n < 0) return fail(TN_E_ARG, "bad argument");
  hipError_t e = launch_norm2((const double*)amp, n, (double*)out_dev, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "norm kernel");
  return TN_OK;
}

int tn_amp_xeb(const void* amp, int64_t n, const void* idx_dev, int64_t n_idx, void* out_dev, void* stream) {
  if (!amp || !out_dev || (n_idx > 0 && !idx_dev) || n < 0 || n_idx < 0) return fail(TN_E_ARG, "bad argument");
  hipError_t e = launch_xeb((const double*)amp, n, (const int64_t*)idx_dev, n_idx, (double*)out_dev,
                            (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "xeb kernel");
  return TN_OK;
}

int tn_amp_frugal(const void* amp, int64_t n, const void* idx_dev, int64_t n_cand, const void* u_dev, double scale,
                  double m, void* out_idx_dev, void* count_dev, void* stream) {
  if (!amp || n < 0 || n_cand < 0 || (n_cand > 0 && (!u_dev || !out_idx_dev)) || !count_dev)
    return fail(TN_E_ARG, "bad argument");
  if (!(m > 0) || !(scale > 0)) return fail(TN_E_ARG, "scale and m must be positive");
  hipError_t e = launch_frugal((const double*)amp, n, (const int64_t*)idx_dev, n_cand, (const double*)u_dev, scale, m,
                               (int64_t*)out_idx_dev, (unsigned long long*)count_dev, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "frugal sampling kernel");
  return TN_OK;
}

int tn_amp_hist(const void* amp, int64_t n, double scale, double xmax, int32_t n_bins, void* counts_dev,
                void* stream) {
  if (!amp || !counts_dev || n < 0 || n_bins < 1 || !(xmax > 0)) return fail(TN_E_ARG, "bad argument");
  hipError_t e = launch_hist((const double*)amp, n, scale, xmax, n_bins, (unsigned long long*)counts_dev,
                             (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "histogram kernel");
  return TN_OK;
}

}  // extern "C"
