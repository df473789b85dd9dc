/*
 * tnrcs.h - C ABI of the MI355X (gfx950) sliced tensor-network contraction
 * library for random-quantum-circuit amplitudes.
 *
 * What is computed.  For a circuit U = G_m ... G_1 on n qubits, a set O of
 * open qubits and bit values x_C on the closed qubits, the library returns the
 * bunch of amplitudes a[y] = <x_C, y_O | U | 0^n> for all y in {0,1}^|O|
 * (main text, "Establishing quantum supremacy baseline": leaving qubits open
 * yields a correlated bunch at little extra cost).  The amplitude is the
 * contraction of the circuit's tensor network (main text, section on the
 * customized TNC algorithm; Supplement Fig. S2), done pairwise in a caller-given
 * order (Supplement, "Tensor network contraction algorithm": an order is a
 * list of two-tuples) with a caller-given set of sliced bonds (main text: the
 * network equals the sum of the smaller networks obtained by fixing the sliced
 * indices).  Each pairwise contraction is an index permutation followed by a
 * complex matrix product (Supplement Eq. (matmul)), or the fused form of the
 * two for skewed shapes (Supplement, CPU-architecture section, Fig. S7a).
 *
 * Conventions (all plain data, no ownership transfer unless stated):
 *  - Qubits 0..n-1.  Bit strings: qubit j is character j; a basis index is
 *    sum_j x_j 2^(n-1-j).
 *  - Gate matrices are row-major complex128, re/im interleaved; a two-qubit
 *    gate acts on |q[0] q[1]> with q[0] the more significant bit.
 *  - Canonical leaves: ids 0..n-1 are the |0> input vectors; then one leaf per
 *    gate in circuit order; then one output vector per CLOSED qubit in qubit
 *    order.  Canonical wires: wire q < n leaves input vector q; every gate
 *    appends one new wire per entry of its qubit list, in that order.
 *  - Order (SSA): step t contracts ids order_pairs[2t], order_pairs[2t+1] and
 *    creates id n_leaves + t; n_steps must be n_leaves - 1 (a full tree).
 *  - Slice s in [0, 2^k) fixes sliced_wires[j] to bit j of s.
 *  - Amplitude buffer: complex128 (re, im doubles), 2^|O| entries; entry y
 *    holds the open qubits (increasing qubit order) as sum_j y_j 2^(|O|-1-j).
 *
 * Errors: every function returns TN_OK (0) or a negative TN_E_* code and
 * never throws; tn_last_error() returns a thread-local message describing the
 * last failure on the calling thread.
 */
#ifndef TNRCS_H
#define TNRCS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TN_OK 0
#define TN_E_ARG (-1)         /* bad argument (null pointer, range, size) */
#define TN_E_TOPOLOGY (-2)    /* order is not a full tree / unknown wire */
#define TN_E_MEM (-3)         /* arena exceeds the budget or device memory */
#define TN_E_HIP (-4)         /* a HIP runtime call failed */
#define TN_E_UNSUPPORTED (-5) /* valid request this library does not handle */
#define TN_E_NUMERIC (-6)     /* non-finite or out-of-range values seen */

#define TN_DTYPE_C64 0   /* complex64 storage, FP32 arithmetic */
#define TN_DTYPE_F16S 1  /* FP16 storage + per-tensor power-of-two exponent, FP32 accumulation */
#define TN_DTYPE_BF16S 2 /* BF16 storage + per-tensor power-of-two exponent, FP32 accumulation */

#define TN_GEMM_AUTO 0
#define TN_GEMM_4M 1 /* Cr = ArBr - AiBi, Ci = ArBi + AiBr: four real products */
#define TN_GEMM_3M 2 /* three real products: ArBr, AiBi, (Ar+Ai)(Br+Bi) */

/* Numeric status bits reported by tn_plan_status. */
#define TN_FLAG_NONFINITE 1u  /* a NaN/Inf reached the final tensor */
#define TN_FLAG_OVERFLOW 2u   /* scaled storage: a value exceeded the format range */
#define TN_FLAG_UNDERFLOW 4u  /* scaled storage: a tensor's maximum fell below the target range */

typedef struct tn_plan_s* tn_plan_t;

typedef struct {
  int32_t nq;   /* 1 or 2 */
  int32_t q[2]; /* qubits; q[1] unused when nq == 1 */
  double m[32]; /* row-major complex128 matrix, re/im interleaved: 8 doubles (2x2) or 32 (4x4) */
} tn_gate;

typedef struct {
  int32_t n_qubits;
  int32_t n_gates;
  const tn_gate* gates;    /* n_gates entries, circuit order */
  const uint8_t* out_bits; /* n_qubits entries (0/1); read only for closed qubits; may be NULL if all open */
} tn_circuit;

typedef struct {
  int32_t dtype;          /* TN_DTYPE_* */
  int32_t gemm_form;      /* TN_GEMM_* */
  int32_t max_log2;       /* reject plans with a per-slice tensor above 2^max_log2 elements (0: no bound) */
  int32_t use_graph;      /* 1: run each slice as one replay of a captured HIP graph */
  int32_t dry_run;        /* 1: plan on the host only; no device calls, no device memory */
  int32_t device;         /* HIP device ordinal */
  int32_t host_fold_log2; /* steps whose result has at most 2^host_fold_log2 entries and whose operands
                             are leaves or folded leaves are evaluated once on the host in FP64 */
  int32_t tune;           /* 1: at tn_plan time, choose each step's kernel class (permutes + GEMM or a
                             fused kernel) and every dense GEMM step's tile size (64 or 128) and
                             K-split count by timing them on the device (see below) */
  int64_t arena_bytes;    /* arena == NULL: device memory budget for intermediates (0: 92% of free
                             memory); arena != NULL: the size of that workspace in bytes */
  void* arena;            /* NULL: the plan allocates and owns its intermediate arena.  Otherwise a
                             caller-owned device workspace of arena_bytes bytes (256-byte aligned)
                             used for every intermediate; several plans may share one workspace as
                             long as their runs are ordered (one stream, or a batch below).  It must
                             outlive the plan.  tn_plan fails with TN_E_MEM if it is too small. */
  const char* tune_db;    /* with tune: a text file caching tuning results across processes (read
                             at the first use of a path, new results appended); NULL: the results
                             are kept for the life of the process only */
} tn_plan_opts;

/* Per-plan totals for one slice (flop convention: one complex multiply-add = 8 flops). */
typedef struct {
  int64_t n_slices;        /* 2^k */
  int32_t n_leaves;        /* canonical leaves */
  int32_t n_host_steps;    /* steps folded on the host at plan time */
  int32_t n_device_steps;  /* steps run per slice */
  int32_t n_kernels;       /* kernel launches per slice */
  int32_t max_log2;        /* largest per-slice device tensor, log2 elements */
  int32_t n_open;
  double flops_per_slice;  /* sum over device steps of 8*M*N*K */
  double bytes_per_slice;  /* algorithmic bytes: each step reads A and B once and writes C once */
  double moved_per_slice;  /* bytes the chosen kernels move, extra permute traffic included */
  int64_t arena_bytes;     /* device arena for intermediates and permute scratch */
  int64_t leaf_bytes;      /* device leaves (all slices) */
  int32_t n_dense, n_skinny, n_generic, n_permute; /* kernel-class counts per slice */
  int32_t k_hist[64];      /* histogram of contracted-index count |K| over device steps */
} tn_plan_stats;

/* Fills *o with the defaults (complex64, auto GEMM form, graph on, device 0,
 * host folding up to 2^12 entries, automatic arena budget).
 *
 * Scaled storage (dtype TN_DTYPE_F16S / TN_DTYPE_BF16S; the main text names
 * mixed precision without a scheme, this is this library's): every device
 * tensor T holds value * 2^-e_T in the 16-bit format; leaves get e from their
 * largest component; every contraction accumulates in FP32 and stores its
 * result shifted by a per-step power of two chosen once, at tn_plan time, by
 * running slice 0 step by step and bringing each step's largest accumulator
 * magnitude to 2^12; the slice result is widened to FP64 with its exponent
 * before the cross-slice sum.  Later slices reuse the shifts; each slice
 * checks every step's largest stored magnitude and raises TN_FLAG_OVERFLOW
 * (the format's maximum reached) or TN_FLAG_UNDERFLOW (a step's largest
 * magnitude fell below 2^-2), read with tn_plan_status.
 *
 * Tuning (opts->tune), two stages.  Kernel class: a step with more than
 * one valid kernel class (permutes + MFMA GEMM against the fused gathered
 * kernel and the matrix-core skewed kernel when the contraction has at most
 * 2^6 terms; gathered, the two skewed kernels and split-K against each
 * other for steps with too few outputs for the GEMM)
 * is run in each on a one-step plan of the same operand layouts over
 * scratch buffers of random values (at most 48 GiB and a third of the free
 * device memory; larger steps keep the default rule; the gathered kernel is
 * timed only on steps of at most 2^22 outputs and sums shorter than 2^16
 * terms), and the fastest is planned.  With the environment variable
 * TNRCS_VERBOSE set, each tuned step prints a line on stderr.  Tile: for
 * each distinct dense-GEMM shape of the plan (dtype, M, N, K, form) every
 * valid tile size, K-split count and kernel variant is timed with HIP events
 * on the plan's own buffers (the arena is filled with random values first:
 * the matrix cores run faster on zeros) and the fastest kept.  Dense steps
 * that read a large A in place (no permute of A; at least 2^5 terms and,
 * for sums of 2^11 terms or more, at least 512 output tiles of 128x128)
 * have one fixed kernel and are not timed.
 * Results are cached per process and, with tune_db, in a file (lines
 * "tnrcs-class dtype key class ms" and "tnrcs-gemm dtype M N K form cap tile
 * split occ ms"; the key is the step's operand and result layouts with the
 * wires relabelled, as in tn_plan_json's "steps").  A dry-run plan with tune
 * set measures nothing but applies the class lines already cached or in
 * tune_db.  The split count and the class change the summation order inside
 * a step, so two processes that tune differently may differ in the last
 * bits; a shared tune_db file makes the choice reproducible. */
void tn_plan_opts_default(tn_plan_opts* o);

/* Plans the contraction (main text TNC section; Supplement Fig. S2 and the
 * TNC section).  Copies every input.  Validates the circuit, the order (full
 * SSA tree over the canonical leaves), the sliced wires (in range, distinct,
 * not open) and the open qubits (distinct, in range); folds small slice-local
 * subtrees on the host in FP64; chooses tensor layouts and kernels; assigns
 * device-arena offsets by liveness; unless opts->dry_run, allocates device
 * memory on opts->device, uploads the leaves and, with use_graph, prepares the
 * per-slice graph lazily.  opts may be NULL (defaults).  On success *out owns
 * all of this until tn_plan_destroy. */
int tn_plan(const tn_circuit* c, const int32_t* order_pairs, int32_t n_steps,
            const int32_t* sliced_wires, int32_t k, const int32_t* open_qubits, int32_t n_open,
            const tn_plan_opts* opts, tn_plan_t* out);

/* The sliced network is the sum of the networks with the sliced bonds fixed
 * (main text, customized-TNC section), and slices are independent units of
 * work (the outer level of the paper's two-level parallel scheme, main text).
 * Contracts slices s_begin <= s < s_end and ACCUMULATES (+=) their sum into
 * amp (device memory, complex128[2^n_open]), in increasing slice order, on
 * `stream` (a hipStream_t; NULL = the null stream).  Asynchronous: returns
 * after enqueueing.  The per-slice result is widened to FP64 before it is
 * added, so the cross-slice sum is FP64 and its order is fixed by the slice
 * ids; splitting a range over several calls gives the identical sum.  A plan
 * must be used by one stream at a time.  TN_E_UNSUPPORTED for dry-run plans. */
int tn_contract_slices(tn_plan_t p, int64_t s_begin, int64_t s_end, void* amp, void* stream);

/* Checked form of tn_contract_slices for scaled storage (the retry of the
 * mixed-precision scheme): every slice is first contracted into plan-owned
 * staging, the stream is synchronized and the slice's numeric flags are
 * read.  A clean slice is then added to amp.  A slice that raised
 * TN_FLAG_OVERFLOW or TN_FLAG_UNDERFLOW makes the plan recalibrate its output
 * shifts on that slice (later slices keep the new shifts) and run it again
 * once; if flags persist, or a NaN/Inf appears without a range flag (or in
 * complex64), nothing of that slice is added, the flags stay set and the
 * call returns TN_E_NUMERIC (slices before it are in amp).  *retries
 * (may be NULL) receives the number of re-run slices.  Synchronous. */
int tn_contract_slices_checked(tn_plan_t p, int64_t s_begin, int64_t s_end, void* amp, void* stream,
                               int32_t* retries);

/* Scaled storage: adds delta (|delta| <= 64) to the calibrated output shift
 * of kernel `op` (its index in the plan's kernel list, see tn_plan_json), or
 * of every producing kernel if op < 0.  The kernel's stored result is scaled
 * by 2^-delta relative to its stored inputs, so the change carries along the
 * contraction tree (with op < 0 it compounds with depth); the exponents are
 * updated so the results are unchanged, exactly so while every value stays in
 * the format's normal range.  A manual adjustment of the calibration, also
 * used to test the range checks.  TN_E_ARG for complex64 plans, for a kernel
 * without an output shift (a permute) or an index out of range. */
int tn_plan_shift_outputs(tn_plan_t p, int32_t op, int32_t delta);

/* ---- batches of plans (many circuits in one call) ----
 * An extension with no counterpart in the paper: slices of several
 * independent networks (different circuits) run from one call, in lanes
 * that may run side by side.  Each network's value is still the sum over its
 * slices (main text, customized-TNC section). */

typedef struct tn_batch_s* tn_batch_t;

/* Prepares a batch that runs plans[0..n): for plan i the
 * slices ranges[2i] <= s < ranges[2i+1], accumulated (+=) into amps[i]
 * (device complex128[2^n_open of plan i]) exactly as tn_contract_slices
 * would (same kernels, same order, same sums).  Plans may be of different
 * circuits, sizes and dtypes, and may share one arena workspace
 * (opts.arena); the same plan may appear more than once.  Plans whose
 * arenas overlap, that are the same plan or that share an amplitude buffer
 * run one after the other, in the order given, in one lane; plans on
 * separate arenas may go to separate lanes (at most 4).  In a lane, each
 * plan sets its slice cursor and replays its per-slice HIP graph (captured
 * here for every plan with opts.use_graph) once per slice.  Each lane runs
 * on a stream of the batch (default priority) that starts after the
 * caller's stream's earlier work and that the caller's stream waits for, so
 * lanes run side by side.  The plans and amplitude buffers must
 * outlive the batch, and a plan must not be run elsewhere while the batch
 * runs. */
int tn_batch_create(const tn_plan_t* plans, int32_t n, const int64_t* ranges, void* const* amps, tn_batch_t* out);

/* Enqueues the batch on `stream`: every lane's plans in order, the lanes
 * joined back into `stream`.  Asynchronous. */
int tn_batch_run(tn_batch_t b, void* stream);

/* Releases the batch's streams and events (not the plans or their graphs).
 * NULL is accepted. */
int tn_batch_destroy(tn_batch_t b);

/* One-shot form: tn_batch_create, tn_batch_run on `stream`, wait for the
 * stream, tn_batch_destroy. */
int tn_contract_batch(const tn_plan_t* plans, const int64_t* ranges, void* const* amps, int32_t n, void* stream);

/* Copies the plan's statistics into *s: the per-slice contraction cost of
 * the order (the complexity measure of Table I and of the Supplement's
 * "Tensor network contraction algorithm" section, counted as 8 flops per
 * complex multiply-add), the bytes of its tensors, and the slice count 2^k. */
int tn_plan_info(tn_plan_t p, tn_plan_stats* s);

/* Writes the plan as JSON (host folds, device leaves, per-step kernels with
 * layouts and arena offsets, and per device step its extents nM nN nK, its
 * kernel class (1 GEMM, 2 gathered, 3 skewed, 4 split-K), its
 * relabelled layout key and whether the class tuner chose it) into buf (capacity cap bytes, NUL-terminated);
 * *needed receives the full length + 1.  buf may be NULL to query the size. */
int tn_plan_json(tn_plan_t p, char* buf, int64_t cap, int64_t* needed);

/* Copies device leaf i (host-folded, FP64, in its stored layout, all slices)
 * into out (host memory, 2 * 2^rank doubles).  For tests of the planner. */
int tn_plan_leaf(tn_plan_t p, int32_t i, double* out, int64_t cap_doubles);

/* Numeric state of the mixed-precision mode that the main text names (the
 * range checks are this library's scheme, see tn_plan_opts_default).
 * Sticky numeric flags (TN_FLAG_*) of the plan's runs so far.  Synchronizes
 * the stream of the plan's last tn_contract_slices call. */
int tn_plan_status(tn_plan_t p, uint32_t* flags);

/* The target basis state enters the network only through the rank-1 output
 * vectors of the closed qubits (main text, customized-TNC section: the
 * network with a given target basis yields that basis's amplitude), so the
 * same plan serves every bit string.
 * Rebinds the closed-qubit output bits without re-planning (re-folds and
 * re-uploads the affected leaves).  Synchronous. */
int tn_plan_set_output_bits(tn_plan_t p, const uint8_t* out_bits);

/* Runs slice `slice` once without a graph, accumulating into amp like
 * tn_contract_slices, with a pair of HIP events on `stream` around every
 * kernel; synchronizes and writes each kernel's duration in milliseconds to
 * op_ms[0..n) in plan order (the per-step kernels, then the accumulation).
 * *n_ops receives the kernel count; cap is op_ms's capacity.  Measurement
 * support for benchmarks; the slice result is the same as in the graph path. */
int tn_plan_profile(tn_plan_t p, int64_t slice, void* amp, void* stream, float* op_ms, int32_t cap,
                    int32_t* n_ops);

/* Releases the plan, its device memory and its graph.  NULL is accepted. */
int tn_plan_destroy(tn_plan_t p);

const char* tn_last_error(void);

/* ---- one pairwise contraction (Supplement Eq. (matmul)) ---- */

/* Plans C = sum over shared labels of A * B for caller tensors whose indices
 * carry integer labels (0..4095, most significant first; every dimension 2):
 * labels shared by A and B are contracted, and C's labels must be exactly
 * the unshared ones, in the caller's order.  The planner picks the same
 * kernels as for a network step (permute + MFMA GEMM, the skewed kernels,
 * split-K or a gathered contraction) and adds a final permute when its natural
 * output order differs.  opts as for tn_plan (dtype, gemm_form, device;
 * host folding and graphs are not used).  Release with tn_plan_destroy. */
int tn_pair_plan(int32_t rank_a, const int32_t* labels_a, int32_t rank_b, const int32_t* labels_b, int32_t rank_c,
                 const int32_t* labels_c, const tn_plan_opts* opts, tn_plan_t* out);

/* Runs the pairwise plan on `batch` independent (A, B, C) triples stored
 * consecutively (strides 2^rank_a, 2^rank_b, 2^rank_c elements of the plan's
 * dtype; device memory, C must not overlap A or B), asynchronously on
 * `stream`.  out_scale: for F16S/BF16S the FP32 product is multiplied by it
 * before rounding (it must be 1 for complex64). */
int tn_pair_run(tn_plan_t p, const void* A, const void* B, void* C, int64_t batch, float out_scale, void* stream);

/* ---- standalone kernels of the hot path (same kernels the plans run) ---- */

/* Binary-index tensor permutation (the index permutation of Supplement
 * Eq. (matmul)): a rank-r tensor with every dimension 2, row-major (position
 * p = bit p of the linear index, position 0 fastest), elements of elem_bytes
 * = 8 (complex64) or 4 (FP16/BF16 pair).  Output position q takes input
 * position perm[q]:  out[sum_q b_{perm[q]} 2^q] = in[sum_p b_p 2^p].
 * `batch` (<= 65535) tensors at strides of 2^r elements.  in/out are device
 * pointers and must not overlap.  0 <= r <= 40. */
int tn_permute(const void* in, void* out, int32_t elem_bytes, int32_t rank, const int32_t* perm, int64_t batch,
               void* stream);

/* Complex GEMM from real MFMA products with FP32 accumulation (the matrix
 * product of Supplement Eq. (matmul)):
 * C[m][n] = sum_k A[m][k] * B[n][k] for `batch` independent problems
 * (complex64, row-major, A: M x K, B: N x K, C: M x N, batch strides
 * M*K, N*K, M*N elements).  form = TN_GEMM_4M or TN_GEMM_3M.  M, N multiples
 * of 64 and K a multiple of 16 (the planner only emits such shapes; other
 * shapes are routed to the other kernels).  splits > 1 (batch 1, K a
 * multiple of 16*splits; 128x128 tiles when M and N are multiples of 128,
 * else 64x64) splits K into slabs written to `work` (device, splits*M*N
 * complex64, caller-owned) and summed in slab order in FP64; work may be
 * NULL when splits <= 1. */
int tn_cgemm_c64(const void* A, const void* B, void* C, int64_t M, int64_t N, int64_t K,
                 int64_t batch, int32_t form, void* work, int32_t splits, void* stream);

/* Complex GEMM on FP16 (dtype TN_DTYPE_F16S) or BF16 (TN_DTYPE_BF16S) matrix
 * cores with FP32 accumulation, for scaled storage: A, B, C hold (re, im)
 * pairs of the 16-bit format; C = round(out_scale * A B^T) with the same
 * shapes, layouts and batch convention as tn_cgemm_c64; M, N multiples of
 * 64, K a multiple of 16.  If max_out (device float, non-NULL) is given, the
 * largest |component| of A B^T (before scaling) is folded into it with an
 * atomic maximum (it must start at 0 or a smaller value).  splits > 1 as in
 * tn_cgemm_c64 (work: splits*M*N complex64 entries). */
int tn_cgemm_half(int32_t dtype, const void* A, const void* B, void* C, int64_t M, int64_t N, int64_t K,
                  int64_t batch, int32_t form, float out_scale, void* work, int32_t splits, void* max_out,
                  void* stream);

/* Allocation-free form of tn_cgemm_c64 with batch 1, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  With splits > 1 the K slabs go to a
 * static device array of TN_NOALLOC_SCRATCH_BYTES that the library holds on
 * each device it runs on until the process ends (its address is looked up
 * once per device with hipGetSymbolAddress); nothing is allocated or freed.
 * The result is bitwise that of tn_cgemm_c64 with the same arguments (same
 * kernels, same summation order).  Every slab is written before it is read,
 * so nothing needs clearing between calls.  Runs on the calling thread's
 * current device.  Errors: TN_E_ARG for the shapes tn_cgemm_c64 rejects and
 * when splits * M * N * 8 bytes exceed the scratch (8 Mi complex64 entries,
 * e.g. M = N = 1024 with up to 8 slabs).  Calls that overlap in time on one
 * device share the array and race: order them on one stream. */
#define TN_NOALLOC_SCRATCH_BYTES (64ll << 20)
int tn_cgemm_c64_noalloc(const void* A, const void* B, void* C, int64_t M, int64_t N, int64_t K, int32_t form,
                         int32_t splits, void* stream);

/* ---- measurement probes (the machine ceilings the kernels are compared with) ---- */

/* MFMA issue loop with no memory traffic: kind 0 = v_mfma_f32_32x32x2_f32,
 * 1 = v_mfma_f32_32x32x16_f16, 2 = v_mfma_f32_32x32x16_bf16; every wave of a
 * fixed grid issues `iters` (1..2^24) rounds of 4 independent MFMAs.  *flops
 * (host) receives the flops issued; out_dev (device float[
 * tn_probe_mfma_out_floats()]) receives per-thread sums.  Asynchronous on
 * `stream`; time it with events. */
int tn_probe_mfma(int32_t kind, int64_t iters, void* out_dev, double* flops, void* stream);
int64_t tn_probe_mfma_out_floats(void);

/* Streaming device copy (16-byte nontemporal loads and stores, 16384
 * blocks) of `bytes` (a multiple of 16; both pointers 16-byte aligned, not
 * overlapping): the practical HBM ceiling of the data-movement kernels,
 * which read and write about as much as a copy does.  Asynchronous on
 * `stream`. */
int tn_probe_copy(const void* src, void* dst, int64_t bytes, void* stream);

/* FP64 reductions over an amplitude buffer (complex128, device):
 *  out[0] = sum |a|^2 over n entries (the norm of an all-open run). */
int tn_amp_norm2(const void* amp, int64_t n, void* out_dev, void* stream);
/*  XEB sums over sampled entries: out[0] = sum_i |a[idx_i]|^2,
 *  out[1] = sum_i |a[idx_i]|^4 (idx: device int64[n_idx]).  F = 2^n out[0]/n_idx - 1. */
int tn_amp_xeb(const void* amp, int64_t n, const void* idx_dev, int64_t n_idx, void* out_dev,
               void* stream);
/*  Frugal rejection sampling (main text: one perfect sample from a bunch of
 *  64 amplitudes by frugal sampling, after the works it cites): candidate j,
 *  the amplitude a[idx[j]] (idx_dev may be NULL: candidate j is a[j]), is
 *  kept when u[j] * m < scale * (re*re + im*im), evaluated in FP64 with each
 *  operation rounded separately; with scale = N = 2^n and u uniform on
 *  [0, 1) that is probability min(1, N p / m).  u_dev: device double[n_cand]
 *  (the caller draws the random numbers); kept amplitude indices go to
 *  out_idx_dev (device int64[n_cand]) in unspecified order, their number to
 *  *count_dev (device int64).  Candidates outside [0, n) are never kept.
 *  scale, m > 0. */
int tn_amp_frugal(const void* amp, int64_t n, const void* idx_dev, int64_t n_cand, const void* u_dev, double scale,
                  double m, void* out_idx_dev, void* count_dev, void* stream);
/*  Histogram of x = scale * |a|^2 into n_bins bins of width xmax/n_bins
 *  (last bin collects x >= xmax), counts as uint64 (Eq. (fxeb) check). */
int tn_amp_hist(const void* amp, int64_t n, double scale, double xmax, int32_t n_bins,
                void* counts_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TNRCS_H */
