"""Benchmark: sliced contraction of the 53-qubit, 14-cycle synthetic random
circuit network (6x9 grid with one missing site, 6 open qubits -> bunches of
64 amplitudes, every per-slice tensor <= 2^32 entries) on one MI355X.

One step = one slice: bind, every pairwise contraction of the slice
(permutes, complex GEMMs on MFMA, skewed / gathered contractions) and the
FP64 accumulation of its 64 amplitudes.  The headline line is the complex64
network; the same network in scaled FP16 / BF16, the pairwise-contraction
microbench (32 rank-27 x rank-25 pairs) and the permute / skewed-kernel
bandwidths are reported alongside.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--form auto|4m|3m]
                  [--dtype c64|f16s|bf16s] [--no-extra] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sec/slice + complex TFLOP/s (% MFMA peak), 53-qubit 14-cycle synthetic RCS"
PEAK = {"c64": 157.3, "f16s": 2500.0, "bf16s": 2500.0}  # dense MFMA TFLOP/s: FP32, FP16, BF16
PEAK_HBM = 8000.0  # GB/s
KIND_NAMES = {0: "k_permute", 1: "k_cgemm", 2: "k_generic", 3: "k_skinny", 4: "k_splitk", 5: "k_skew", 9: "k_accum"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2111_01066_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, dtype: str, alg_bytes_per_launch: float = None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources (else None).  The summary
    holds, for the dominant kernel's launches of the profiled run, the HBM
    bytes per launch and their ratio to the algorithmic bytes of the same
    launches; a tuned plan may mix its launches differently from run to run,
    so the ratio is applied to this run's algorithmic bytes per launch."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_sha") != source_sha():
        return None
    key = f"{kernel}:{dtype}"
    ratio = d.get("hbm_over_algorithmic", {}).get(key)
    if ratio is not None and alg_bytes_per_launch:
        return ratio * alg_bytes_per_launch
    return d.get("per_launch_bytes", {}).get(key)


def w_flops_per_slice(w):
    from rqcgen import network_structure, order_stats
    return order_stats(network_structure(w.circuit, w.open_qubits), w.pairs, w.sliced).flops_per_slice


def cpu_baseline(w, sub_log2: int):
    """The oracle on a bounded sample: one sub-slice of slice 0 (extra wires
    sliced until every tensor has <= 2^sub_log2 entries); rate in complex
    TFLOP/s of algorithmic work (8 flops per complex multiply-add)."""
    import oracle
    from oracle.tn import contract_network, slice_assignment
    from rqcgen import network_structure, order_stats, slice_to_fit
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    ns = network_structure(w.circuit, w.open_qubits)
    allsl = slice_to_fit(ns, w.pairs, sub_log2, initial=w.sliced)
    st = order_stats(ns, w.pairs, allsl)
    leaves, ow = oracle.build_network(w.circuit, w.open_qubits, w.out_bits)
    t0 = time.perf_counter()
    contract_network(leaves, w.pairs, ow, slice_assignment(allsl, 0))
    dt = time.perf_counter() - t0
    rate = st.flops_per_slice / dt / 1e12
    return {"value": rate, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": (f"FP64 numpy tensordot contraction of one sub-slice of slice 0 of the same network "
                       f"({len(allsl) - len(w.sliced)} extra sliced wires, tensors <= 2^{sub_log2}, "
                       f"{st.flops_per_slice:.3e} flop) in {dt:.1f} s; at this rate one slice "
                       f"({w_flops_per_slice(w):.3e} flop) takes {w_flops_per_slice(w) / (rate * 1e12):.0f} s"),
            "seconds": dt}


def run_network(tnrcs, torch, w, dtype, form, K, W, graph=True, profile=True, tune=True, tune_db=None):
    """Plans (with the autotuner unless tune is False: kernel class per step,
    GEMM tile / split / variant per shape; plan-time work, outside the timed
    region), warms up W slices, then times K slices on the GPU."""
    t0 = time.perf_counter()
    plan = tnrcs.Plan(w.circuit, w.pairs, w.sliced, w.open_qubits, w.out_bits, gemm_form=form, use_graph=graph,
                      dtype=dtype, tune=tune, tune_db=tune_db)
    t_plan = time.perf_counter() - t0
    info = plan.info()
    log(f"[bench] {dtype}: planned{' and tuned' if tune else ''} in {t_plan:.2f} s: "
        f"{info['n_device_steps']} device steps, "
        f"{info['n_kernels']} kernels/slice, arena {info['arena_bytes'] / 2**30:.1f} GiB, "
        f"{info['flops_per_slice']:.3e} flop/slice")
    stream = torch.cuda.current_stream()
    amp = torch.zeros(64, dtype=torch.complex128, device="cuda")
    for s in range(W):
        plan.contract(s, s + 1, amp)
        torch.cuda.synchronize()
        log(f"[bench] {dtype}: warmup slice {s} done")
    amp.zero_()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for s in range(K):
        plan.contract(s, s + 1, amp)
    ev1.record(stream)
    torch.cuda.synchronize()
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    flags = plan.status()
    res = {"plan": plan, "info": info, "sec_per_slice": gpu_s / K, "tflops": info["flops_per_slice"] * K / gpu_s / 1e12,
           "flags": flags, "amp": amp.cpu().numpy(), "plan_s": t_plan}
    log(f"[bench] {dtype}: {K} slices in {gpu_s:.3f} s: {gpu_s / K:.4f} s/slice, {res['tflops']:.2f} complex "
        f"TFLOP/s, flags={flags}")
    if profile:
        res["ops"] = plan.json()["ops"]
        scratch = torch.zeros(64, dtype=torch.complex128, device="cuda")
        res["ms"] = plan.profile(0, scratch)
    return res


def kernel_split(res, dtype):
    ops, ms = res["ops"], res["ms"]
    by_kind = {}
    for i, t in enumerate(ms):
        o = ops[i] if i < len(ops) else {"kind": 9, "flops": 0.0, "bytes": 0.0}
        d = by_kind.setdefault(o["kind"], {"ms": 0.0, "n": 0, "flops": 0.0, "bytes": 0.0, "issued": 0.0})
        d["ms"] += float(t)
        d["n"] += 1
        d["flops"] += o["flops"]
        d["bytes"] += o["bytes"]
        d["issued"] += o["flops"] * (0.75 if o.get("form") == 2 else 1.0)
    split = {KIND_NAMES[k]: {"ms_per_slice": v["ms"], "launches": v["n"]} for k, v in by_kind.items()}
    for k, v in by_kind.items():
        if k in (0, 2, 3, 4, 5) and v["ms"] > 0:
            split[KIND_NAMES[k]]["GB/s"] = v["bytes"] / (v["ms"] / 1e3) / 1e9
    order = sorted(range(len(ops)), key=lambda i: -ms[i])
    for i in order[:12]:
        o = ops[i]
        shape = (f"M={o['M']} N={o['N']} K={o['K']}" if o["kind"] == 1 else
                 f"rank={o['rank']}" if o["kind"] == 0 else f"nM={o['nM']} nN={o['nN']} nK={o['nK']}")
        rate = (f"{o['flops'] / (ms[i] / 1e3) / 1e12:.1f} TFLOP/s" if o["kind"] == 1 else
                f"{o['bytes'] / (ms[i] / 1e3) / 1e9:.0f} GB/s")
        log(f"[bench]   {dtype} op {i:3d} {KIND_NAMES.get(o['kind'], o['kind']):10s} {ms[i]:9.3f} ms  {shape:28s} "
            f"{rate}")
    return by_kind, split


def slice_roofline_frac(res, dtype):
    """Sum over the slice's kernels of max(flops / MFMA peak, bytes / HBM peak)
    divided by the measured time per slice (GEMM flops as issued: 6MNK in the
    3M form, 8MNK in 4M)."""
    t = 0.0
    for o in res["ops"]:
        fl = o["flops"] * (0.75 if o["kind"] == 1 and o.get("form") == 2 else 1.0)
        t += max(fl / (PEAK[dtype] * 1e12), o["bytes"] / (PEAK_HBM * 1e9))
    return t / res["sec_per_slice"]


def roofline(by_kind, dtype, copy_gbs=None):
    dom = max(by_kind, key=lambda k: by_kind[k]["ms"])
    d = by_kind[dom]
    avg_ms = d["ms"] / d["n"]
    name = KIND_NAMES[dom]
    if dom == 1:
        achieved = d["issued"] / d["n"] / (avg_ms / 1e3) / 1e12
        return {"kernel": name, "bound": "mfma", "achieved": achieved, "peak": PEAK[dtype], "unit": "TFLOP/s",
                "frac": achieved / PEAK[dtype], "traffic": measured_traffic(name, dtype, d["bytes"] / d["n"]),
                "launches_per_slice": d["n"], "avg_ms": avg_ms, "flop_per_launch": d["issued"] / d["n"],
                "bytes_per_launch": d["bytes"] / d["n"],
                "complex_tflops": d["flops"] / d["n"] / (avg_ms / 1e3) / 1e12,
                "note": "achieved = issued real MFMA flops per launch (6 per complex multiply-add in the 3M form, "
                        "8 in 4M) / mean launch duration (HIP events on the launch stream); traffic = this run's "
                        "algorithmic bytes per launch x the HBM/algorithmic ratio that rocprofv3 FETCH_SIZE + "
                        "WRITE_SIZE (scaled by a plain copy) measured on the same kernels (profiles/traffic.json)"}
    achieved = d["bytes"] / d["n"] / (avg_ms / 1e3) / 1e9
    r = {"kernel": name, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM, "unit": "GB/s",
         "frac": achieved / PEAK_HBM, "traffic": measured_traffic(name, dtype, d["bytes"] / d["n"]),
         "launches_per_slice": d["n"],
         "avg_ms": avg_ms, "bytes_per_launch": d["bytes"] / d["n"],
         "note": "achieved = algorithmic bytes per launch (each operand read once, the output written once) / "
                 "mean launch duration (HIP events on the launch stream); traffic = this run's algorithmic bytes "
                 "per launch x the HBM/algorithmic ratio that rocprofv3 FETCH_SIZE + WRITE_SIZE (scaled by a "
                 "plain copy) measured on the same kernel (profiles/traffic.json)"}
    if copy_gbs:
        r["copy_probe_GB/s"] = copy_gbs
        r["frac_of_copy_probe"] = achieved / copy_gbs
    return r


def copy_ceiling(tnrcs, torch, gib: int = 8, reps: int = 5):
    """The practical HBM ceiling of a kernel that reads and writes about as
    much: the streaming copy probe on two gib-GiB buffers, median of reps
    launches (HIP events on the current stream)."""
    nb = gib << 30
    src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    tnrcs.tn_probe_copy(src, dst, nb)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        tnrcs.tn_probe_copy(src, dst, nb)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nb / sorted(ts)[reps // 2] / 1e6


def config2_pairs(tnrcs, torch, timed, dtypes=("c64", "f16s")):
    """Config 2: 32 pairs of rank-27 x rank-25 complex tensors sharing 12
    indices, one pairwise-contraction launch (GEMM M = 2^15, N = 2^13,
    K = 2^12 per pair, permutes included)."""
    out = {}
    from rqcgen.workloads import config2_pair
    la, lb, lc = config2_pair(seed=2)
    n_pairs = 32
    for dtype in dtypes:
        pp = tnrcs.PairPlan(la, lb, lc, dtype=dtype)
        g = torch.Generator(device="cuda")
        g.manual_seed(2)
        if dtype == "c64":
            A = torch.randn(n_pairs, 1 << 27, dtype=torch.complex64, device="cuda", generator=g)
            B = torch.randn(n_pairs, 1 << 25, dtype=torch.complex64, device="cuda", generator=g)
            C = torch.empty(n_pairs, 1 << 28, dtype=torch.complex64, device="cuda")
        else:
            A = torch.randn(n_pairs, 1 << 27, 2, device="cuda", generator=g).half()
            B = torch.randn(n_pairs, 1 << 25, 2, device="cuda", generator=g).half()
            C = torch.empty(n_pairs, 1 << 28, 2, dtype=torch.float16, device="cuda")
        ms = timed(lambda: pp.run(A, B, C, batch=n_pairs, out_scale=1.0 if dtype == "c64" else 2.0 ** -8), n=2)
        fl = 8.0 * 2 ** 15 * 2 ** 13 * 2 ** 12 * n_pairs
        tf = fl / ms / 1e9
        out[f"pairs_rank27x25_{dtype}"] = {"ms_per_launch": ms, "complex_tflops": tf, "pairs_per_launch": n_pairs,
                                          "complex_rate_over_dtype_mfma_peak": tf / PEAK[dtype]}
        log(f"[bench] config 2 ({n_pairs} rank-27 x rank-25 pairs) {dtype}: {ms:.1f} ms/launch, {tf:.1f} complex "
            f"TFLOP/s at 8 flop per complex multiply-add, {tf / PEAK[dtype]:.2f}x the {dtype} dense MFMA peak"
            f"{' (the 3M form issues 6)' if dtype == 'c64' else ''}, permutes included)")
        pp.close()
        del A, B, C
        torch.cuda.empty_cache()
    return out


def micro(tnrcs, torch, np):
    """Standalone kernels on the shapes that matter, timed with HIP events."""
    out = {}

    def timed(fn, n=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    # machine ceilings: MFMA issue loops and a streaming copy of our own
    probe_out = torch.empty(tnrcs.tn_probe_mfma_out_floats(), dtype=torch.float32, device="cuda")
    for kind, iters, peak in (("f32", 100000, PEAK["c64"]), ("f16", 200000, PEAK["f16s"]),
                              ("bf16", 200000, PEAK["bf16s"])):
        tnrcs.tn_probe_mfma(kind, 1000, probe_out)
        fl = [0.0]
        ms = timed(lambda: fl.__setitem__(0, tnrcs.tn_probe_mfma(kind, iters, probe_out)), n=3)
        tf = fl[0] / ms / 1e9
        out[f"mfma_loop_{kind}"] = {"TFLOP/s": tf, "frac_peak": tf / peak}
        log(f"[bench] MFMA issue loop {kind}: {tf:.1f} TFLOP/s ({tf / peak:.1%} of the {peak:.1f} TFLOP/s peak)")
    del probe_out
    nb = 4 << 30
    src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    ms = timed(lambda: tnrcs.tn_probe_copy(src, dst, nb))
    assert torch.equal(src[:1024], dst[:1024])
    gbs = 2.0 * nb / ms / 1e6
    out["stream_copy_4GiB"] = {"GB/s": gbs, "frac_hbm": gbs / PEAK_HBM}
    log(f"[bench] streaming copy (16-byte accesses): {gbs:.0f} GB/s ({gbs / PEAK_HBM:.1%} of 8 TB/s)")
    del src, dst
    # FP16 subnormal inputs in MFMA: A = 2^-20 (subnormal), B = 1, K = 16
    dA = torch.zeros(128, 16, 2, dtype=torch.float16, device="cuda")
    dA[..., 0] = 2.0 ** -20
    dB = torch.zeros(128, 16, 2, dtype=torch.float16, device="cuda")
    dB[..., 0] = 1.0
    dC = torch.empty(128, 128, 2, dtype=torch.float16, device="cuda")
    tnrcs.tn_cgemm_half("f16s", dA, dB, dC, 128, 128, 16, 1, "4m", out_scale=2.0 ** 20)
    torch.cuda.synchronize()
    v = float(dC[0, 0, 0].float().item())
    out["fp16_mfma_subnormal_inputs"] = "kept" if abs(v - 16.0) < 1e-3 else f"not kept (got {v})"
    log(f"[bench] FP16 MFMA with subnormal inputs: {out['fp16_mfma_subnormal_inputs']}")

    rng = np.random.default_rng(0)
    r = 30
    perm = rng.permutation(r).tolist()
    for eb, name in ((8, "c64"), (4, "f16s")):
        x = torch.ones(1 << r, dtype=torch.float64 if eb == 8 else torch.float32, device="cuda")
        y = torch.empty_like(x)
        ms = timed(lambda: tnrcs.tn_permute(x, y, perm, elem_bytes=eb))
        ms_copy = timed(lambda: y.copy_(x))
        gbs, cps = 2.0 * x.numel() * eb / ms / 1e6, 2.0 * x.numel() * eb / ms_copy / 1e6
        out[f"permute_rank30_{name}"] = {"GB/s": gbs, "frac_hbm": gbs / PEAK_HBM, "device_copy_GB/s": cps,
                                         "frac_of_copy": gbs / cps}
        log(f"[bench] permute rank 30 {name}: {gbs:.0f} GB/s ({gbs / PEAK_HBM:.1%} of 8 TB/s; copy {cps:.0f} GB/s)")
        del x, y
    # skewed contraction: a rank-30 tensor absorbing a two-qubit gate (K=2, N=2 bits)
    la = list(range(30))
    lb = [la[29], la[28], 100, 101]
    lc = la[:28] + [100, 101]
    for dtype in ("c64", "f16s"):
        pp = tnrcs.PairPlan(la, lb, lc, dtype=dtype)
        kinds = [o["kind"] for o in pp.json()["ops"]]
        if dtype == "c64":
            A = torch.ones(1 << 30, dtype=torch.complex64, device="cuda")
            B = torch.ones(16, dtype=torch.complex64, device="cuda")
            C = torch.empty(1 << 30, dtype=torch.complex64, device="cuda")
            eb = 8
        else:
            A = torch.ones(1 << 30, 2, dtype=torch.float16, device="cuda")
            B = torch.ones(16, 2, dtype=torch.float16, device="cuda")
            C = torch.empty(1 << 30, 2, dtype=torch.float16, device="cuda")
            eb = 4
        ms = timed(lambda: pp.run(A, B, C, out_scale=1.0 if dtype == "c64" else 0.25))
        gbs = eb * ((1 << 31) + 16) / ms / 1e6
        out[f"skinny_rank30_gate_{dtype}"] = {"GB/s": gbs, "frac_hbm": gbs / PEAK_HBM, "kernels": kinds}
        log(f"[bench] skewed contraction (rank 30 x two-qubit gate) {dtype}: {gbs:.0f} GB/s ({gbs / PEAK_HBM:.1%})")
        pp.close()
        del A, B, C
    # skewed contraction with a large B (Fig. S7b's case): 2^22 rows of A
    # whose 2^9 contracted entries are interleaved with the row bits, against
    # B of 32 x 2^9 entries (staged through LDS chunk by chunk), as in the
    # 53-qubit network's largest-K skewed step
    la = [1000 + i for i in range(22)]
    kk = list(range(9))
    la = la[:6] + kk[:3] + la[6:14] + kk[3:6] + la[14:] + kk[6:]
    lb = [2000 + j for j in range(5)] + kk[::-1]
    lc = [1000 + i for i in range(22)] + [2000 + j for j in range(5)]
    for dtype in ("c64", "f16s"):
        pp = tnrcs.PairPlan(la, lb, lc, dtype=dtype)
        kinds = [o["kind"] for o in pp.json()["ops"]]
        eb = 8 if dtype == "c64" else 4
        if dtype == "c64":
            A = torch.ones(1 << 31, dtype=torch.complex64, device="cuda")
            B = torch.ones(1 << 14, dtype=torch.complex64, device="cuda")
            C = torch.empty(1 << 27, dtype=torch.complex64, device="cuda")
        else:
            A = torch.ones(1 << 31, 2, dtype=torch.float16, device="cuda")
            B = torch.ones(1 << 14, 2, dtype=torch.float16, device="cuda")
            C = torch.empty(1 << 27, 2, dtype=torch.float16, device="cuda")
        ms = timed(lambda: pp.run(A, B, C, out_scale=1.0 if dtype == "c64" else 2.0 ** -9))
        byts = eb * ((1 << 31) + (1 << 14) + (1 << 27))
        gbs, tfl = byts / ms / 1e6, 8.0 * (1 << 22) * 32 * 512 / ms / 1e9
        out[f"skew_large_b_{dtype}"] = {"GB/s": gbs, "frac_hbm": gbs / PEAK_HBM, "complex_tflops": tfl,
                                        "kernels": kinds, "ms": ms}
        log(f"[bench] skewed contraction with large B (2^22 x 32 outputs, K = 2^9) {dtype}: {ms:.2f} ms, "
            f"{gbs:.0f} GB/s ({gbs / PEAK_HBM:.1%}), {tfl:.0f} complex TFLOP/s, kernels {kinds}")
        pp.close()
        del A, B, C
    torch.cuda.empty_cache()
    out.update(config2_pairs(tnrcs, torch, timed))
    return out


def crosscheck_30q(tnrcs, torch, np):
    """Config 4 cross-check: the 30-qubit all-open network (2^30 amplitudes)
    in every storage type against the stored FP64 state-vector samples:
    normwise amplitude error on 1e4 ideal and 1e4 uniform samples, and the
    cross-entropy estimate over 1e5 samples of each kind vs FP64."""
    from rqcgen.workloads import config4, config4_uniform_indices
    path = os.path.join(ROOT, "tests", "golden", "config4_30q.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        g = {k: z[k] for k in z.files}
    w = config4()
    N = 2 ** 30
    ideal = torch.from_numpy(g["ideal_idx"].astype(np.int64)).cuda()
    uni = torch.from_numpy(config4_uniform_indices()).cuda()
    n_amp, stride = g["ideal_amp"].size, int(g["ideal_amp_stride"])
    out = {}
    for dtype in ("c64", "f16s", "bf16s"):
        plan = tnrcs.Plan(w.circuit, w.pairs, w.sliced, w.open_qubits, w.out_bits, dtype=dtype)
        amp = torch.zeros(N, dtype=torch.complex128, device="cuda")
        plan.contract(0, 1, amp)  # first run captures the graph
        torch.cuda.synchronize()
        amp.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.contract(0, 1, amp)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3
        flops = plan.info()["flops_per_slice"]
        flags = plan.status()
        plan.close()
        r = {"sec": sec, "complex_tflops": flops / sec / 1e12, "flags": flags}
        for name, idx, sub in (("ideal", ideal, ideal[::stride][:n_amp]), ("uniform", uni, uni[:n_amp])):
            got = amp[sub].cpu().numpy()
            ref = g[f"{name}_amp"]
            err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            acc = torch.zeros(2, dtype=torch.float64, device="cuda")
            tnrcs.tn_amp_xeb(amp, N, idx, idx.numel(), acc)
            s1, s2 = acc.cpu().numpy()
            m = idx.numel()
            f = N * s1 / m - 1.0
            se = float(np.sqrt(max(N * N * s2 / m - (f + 1.0) ** 2, 0.0) / m))
            r[name] = {"amp_rel_err": err, "xeb": f, "xeb_fp64": float(g[f"xeb_{name}"]),
                       "abs_delta_xeb": abs(f - float(g[f"xeb_{name}"])), "xeb_stderr": se}
        if dtype == "c64":
            # frugal rejection sampling over 1e5 random bunches of 64 amplitudes (M = 10)
            rng = np.random.default_rng(9)
            starts = rng.integers(0, N // 64, size=100_000) * 64
            cand = torch.from_numpy((starts[:, None] + np.arange(64)[None, :]).reshape(-1)).cuda()
            u = torch.from_numpy(rng.random(cand.numel())).cuda()
            kept = torch.empty(cand.numel(), dtype=torch.int64, device="cuda")
            cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
            e0.record()
            tnrcs.tn_amp_frugal(amp, N, cand, cand.numel(), u, float(N), 10.0, kept, cnt)
            e1.record()
            torch.cuda.synchronize()
            k = int(cnt.item())
            acc = torch.zeros(2, dtype=torch.float64, device="cuda")
            tnrcs.tn_amp_xeb(amp, N, kept[:k], k, acc)
            s1, s2 = acc.cpu().numpy()
            f = N * s1 / k - 1.0
            se = float(np.sqrt(max(N * N * s2 / k - (f + 1.0) ** 2, 0.0) / k))
            r["frugal"] = {"bunches": 100_000, "m": 10.0, "kept": k, "acceptance": k / cand.numel(),
                           "xeb_of_kept": f, "xeb_stderr": se, "kernel_ms": e0.elapsed_time(e1)}
            log(f"[bench] 30q frugal sampling: {k} bit strings kept of {cand.numel()} candidates "
                f"({k / cand.numel():.4f}), their XEB {f:.4f} +- {se:.4f}")
        out[dtype] = r
        log(f"[bench] 30q all-open {dtype}: {sec:.3f} s, amplitude error ideal {r['ideal']['amp_rel_err']:.2e} "
            f"uniform {r['uniform']['amp_rel_err']:.2e}, XEB ideal {r['ideal']['xeb']:.5f} (FP64 "
            f"{r['ideal']['xeb_fp64']:.5f}, s.e. {r['ideal']['xeb_stderr']:.5f}), uniform {r['uniform']['xeb']:.5f}")
        del amp
        torch.cuda.empty_cache()
    return out


def oracle_timings(tnrcs, torch, np, c2_kernels):
    """The oracle (FP64 NumPy on all host threads) on the small workloads,
    beside the GPU on the same work: config 1's state vector and its
    unsliced pairwise contraction (all 2^20 amplitudes, the GPU plan in
    complex64), and one full config-2 pair (rank 27 x rank 25, about
    8.8e12 flop; the GPU figure is one pair's share of the 32-pair launch).
    Reported baselines, not targets."""
    import oracle
    from oracle.tn import contract_network, pairwise_contract
    from rqcgen.workloads import config1, config2_pair
    out = {"cores": len(os.sched_getaffinity(0))}
    w = config1()
    t0 = time.perf_counter()
    oracle.statevector(w.circuit)
    t_sv = time.perf_counter() - t0
    leaves, ow = oracle.build_network(w.circuit, w.open_qubits, w.out_bits)
    t0 = time.perf_counter()
    contract_network(leaves, w.pairs, ow)
    t_tn = time.perf_counter() - t0
    plan = tnrcs.Plan(w.circuit, w.pairs, w.sliced, w.open_qubits, w.out_bits)
    amp = torch.zeros(1 << 20, dtype=torch.complex128, device="cuda")
    plan.contract(0, 1, amp)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        plan.contract(0, 1, amp)
    e1.record()
    torch.cuda.synchronize()
    t_gpu = e0.elapsed_time(e1) / 5e3
    plan.close()
    out["config1_20q_all_open"] = {"oracle_statevector_s": t_sv, "oracle_tn_s": t_tn, "gpu_c64_s": t_gpu,
                                   "speedup_vs_oracle_tn": t_tn / t_gpu}
    log(f"[bench] oracle, config 1: state vector {t_sv:.2f} s, pairwise contraction {t_tn:.2f} s; "
        f"GPU complex64 {t_gpu * 1e3:.2f} ms")
    la, lb, lc = config2_pair(seed=2)
    rng = np.random.default_rng(2)
    A = ((rng.standard_normal(1 << 27) + 1j * rng.standard_normal(1 << 27)) * np.sqrt(0.5)).reshape((2,) * 27)
    B = ((rng.standard_normal(1 << 25) + 1j * rng.standard_normal(1 << 25)) * np.sqrt(0.5)).reshape((2,) * 25)
    t0 = time.perf_counter()
    C, _ = pairwise_contract(A, la, B, lb)
    t_pair = time.perf_counter() - t0
    del A, B, C
    g = c2_kernels.get("pairs_rank27x25_c64", {})
    gpu_pair = g.get("ms_per_launch", float("nan")) / g.get("pairs_per_launch", 1) / 1e3
    out["config2_pair"] = {"oracle_s": t_pair, "oracle_complex_tflops": 8.0 * 2 ** 40 / t_pair / 1e12,
                           "gpu_c64_s_per_pair": gpu_pair, "speedup": t_pair / gpu_pair}
    log(f"[bench] oracle, config 2: one pair in {t_pair:.1f} s ({8.0 * 2 ** 40 / t_pair / 1e12:.2f} complex "
        f"TFLOP/s); GPU complex64 {gpu_pair * 1e3:.1f} ms per pair")
    return out


def batch_uneven(tnrcs, torch, np, cap: float, dtype: str, tune_db=None, lanes: int = 4):
    """Config 5: the frozen uneven circuits whose order costs at most `cap`
    flops over all slices, one 64-amplitude bunch each, scaled storage,
    autotuned plans, `lanes` arena workspaces dealt round-robin (plans on
    different workspaces may run side by side).  Times every plan's slices
    launched plan by plan on one stream (each plan replaying its own
    per-slice graph), plan by plan on one stream per workspace, and the same
    work as one batch call (one lane per workspace); all must
    agree bitwise."""
    from rqcgen.workloads import config5, config5_table
    t = config5_table()
    wl = config5(max_total_flops=cap, table=t)
    t0 = time.perf_counter()
    need = 0
    for w in wl:
        dry = tnrcs.Plan(w.circuit, w.pairs, w.sliced, w.open_qubits, w.out_bits, dtype=dtype, dry_run=True, tune=True)
        need = max(need, dry.info()["arena_bytes"])
        dry.close()
    arenas = [torch.empty(need, dtype=torch.uint8, device="cuda") for _ in range(lanes)]
    plans = []
    for i, w in enumerate(wl):
        plans.append(tnrcs.Plan(w.circuit, w.pairs, w.sliced, w.open_qubits, w.out_bits, dtype=dtype,
                                arena=arenas[i % lanes], tune=True, tune_db=tune_db))
        if (i + 1) % 32 == 0 or i + 1 == len(wl):
            log(f"[bench] batch: {i + 1}/{len(wl)} circuits planned, tuned and calibrated "
                f"({time.perf_counter() - t0:.1f} s)")
    t_plan = time.perf_counter() - t0
    infos = [p.info() for p in plans]
    n_sl = [i["n_slices"] for i in infos]
    flops = float(sum(i["flops_per_slice"] * i["n_slices"] for i in infos))
    kernels = int(sum((i["n_kernels"] + 1) * i["n_slices"] for i in infos))
    log(f"[bench] batch: {len(plans)} circuits of {len(t['S'])} (order cost <= {cap:.0e} flop), {sum(n_sl)} slices, "
        f"{kernels} kernels, {flops:.3e} flop, arena {need / 2**30:.2f} GiB, planned+tuned+calibrated in {t_plan:.1f} s")
    amps_seq = torch.zeros(len(plans), 64, dtype=torch.complex128, device="cuda")
    amps_b = torch.zeros_like(amps_seq)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def sequential():
        for i, p in enumerate(plans):
            p.contract(0, n_sl[i], amps_seq[i])

    sequential()  # captures each plan's per-slice graph
    torch.cuda.synchronize()
    amps_seq.zero_()
    ev0.record(stream)
    sequential()
    ev1.record(stream)
    torch.cuda.synchronize()
    t_seq = ev0.elapsed_time(ev1) / 1e3
    log(f"[bench] batch: plan-by-plan launches {t_seq:.3f} s ({flops / t_seq / 1e12:.1f} complex TFLOP/s)")
    streams = [torch.cuda.Stream() for _ in range(lanes)]  # default priority
    amps_ml = torch.zeros_like(amps_seq)

    def multi_stream():
        for i, p in enumerate(plans):
            p.contract(0, n_sl[i], amps_ml[i], stream=streams[i % lanes])

    multi_stream()
    torch.cuda.synchronize()
    amps_ml.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    multi_stream()
    torch.cuda.synchronize()
    t_ml = time.perf_counter() - t0
    log(f"[bench] batch: plan-by-plan on {lanes} streams {t_ml:.3f} s ({flops / t_ml / 1e12:.1f} complex TFLOP/s), "
        f"identical: {bool(torch.equal(amps_ml, amps_seq))}")
    t0 = time.perf_counter()
    b = tnrcs.Batch(plans, [(0, n) for n in n_sl], [amps_b[i] for i in range(len(plans))])
    t_build = time.perf_counter() - t0
    b.run()
    torch.cuda.synchronize()
    amps_b.zero_()
    ev0.record(stream)
    b.run()
    ev1.record(stream)
    torch.cuda.synchronize()
    t_b = ev0.elapsed_time(ev1) / 1e3
    same = bool(torch.equal(amps_b, amps_seq))
    flags = 0
    for p in plans:
        flags |= p.status()
    log(f"[bench] batch: one batch call {t_b:.3f} s ({flops / t_b / 1e12:.1f} complex TFLOP/s), batch created in "
        f"{t_build:.2f} s, identical to plan-by-plan: {same}, flags {flags}")
    b.close()
    # where the batch time goes: every op of every plan timed alone (HIP
    # events, slice 0) times the plan's slice count, split by the op's size
    scratch = torch.zeros(64, dtype=torch.complex128, device="cuda")
    busy = small = 0.0
    for i, p in enumerate(plans):
        ops = p.json()["ops"]
        ms = p.profile(0, scratch)
        for j, t_op in enumerate(ms):
            o = ops[j] if j < len(ops) else {}
            out_log2 = (o["rank"] if o.get("kind") == 0 else
                        (int(np.log2(o["M"] * o["N"])) if o.get("kind") == 1 else o.get("nM", 0) + o.get("nN", 0)))
            busy += float(t_op) * n_sl[i] / 1e3
            if out_log2 < 20:
                small += float(t_op) * n_sl[i] / 1e3
    log(f"[bench] batch: kernels alone {busy:.3f} s ({busy / t_b:.1%} of the batch-call time), "
        f"{small:.3f} s of it in kernels with fewer than 2^20 outputs")
    for p in plans:
        p.close()
    del arenas
    torch.cuda.empty_cache()
    return {"circuits": len(plans), "of": int(len(t["S"])), "max_order_flops": cap, "dtype": dtype,
            "workspaces": lanes, "plan_by_plan_streams_s": t_ml,
            "kernel_time_s": busy, "kernel_time_over_batch_call": busy / t_b, "small_kernel_time_s": small,
            "time_to_amplitudes_with_plan_s": t_plan + t_b,
            "slices": int(sum(n_sl)), "kernels": kernels, "flops": flops, "arena_bytes": int(need),
            "plan_tune_calibrate_s": t_plan, "batch_create_s": t_build,
            "plan_by_plan_s": t_seq, "plan_by_plan_complex_tflops": flops / t_seq / 1e12,
            "batch_call_s": t_b, "batch_call_complex_tflops": flops / t_b / 1e12, "speedup": t_seq / t_b,
            "bitwise_identical": same, "numeric_flags": flags}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="slices timed (0: every slice of the bunch)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", default="auto", choices=["auto", "4m", "3m"])
    ap.add_argument("--dtype", default="c64", choices=["c64", "f16s", "bf16s"])
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="plan with the default rules instead of the autotuner")
    ap.add_argument("--tune-db", default=None,
                    help="tuning database file (choices found there are reused, new ones appended)")
    ap.add_argument("--no-extra", action="store_true", help="skip the precision variants and microbenchmarks")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sub-log2", type=int, default=28)
    ap.add_argument("--batch-cap", type=float, default=1e14,
                    help="config 5: keep the circuits whose frozen order costs at most this many flops")
    ap.add_argument("--batch-only", action="store_true", help="run only the batched uneven workload")
    ap.add_argument("--crosscheck-only", action="store_true", help="run only the 30-qubit precision cross-check")
    ap.add_argument("--config2-only", action="store_true", help="run only the config-2 pairwise microbenchmark")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="also run a plain device copy of this size (HBM-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the slice range would be split "
                                   "across GPUs with one final 1 KiB reduction (not built)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2111_01066_amd import tnrcs
    from rqcgen.workloads import config3

    if args.crosscheck_only:
        print(json.dumps({"crosscheck_30q": crosscheck_30q(tnrcs, torch, np)}), flush=True)
        return
    if args.config2_only:
        def timed(fn, n=5):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(n):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / n
        res = config2_pairs(tnrcs, torch, timed)
        if args.copy_probe_gib > 0:  # a plain device copy of known size (HBM-counter calibration)
            n = int(args.copy_probe_gib * 2**30) // 8
            src = torch.ones(n, dtype=torch.complex64, device="cuda")
            dst = torch.empty_like(src)
            dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
        print(json.dumps({"config2": res}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batch_uneven": batch_uneven(tnrcs, torch, np, args.batch_cap, "f16s")}), flush=True)
        return
    w = config3()
    log(f"[bench] workload {w.name}: {len(w.pairs)} steps, k={len(w.sliced)} sliced wires")
    n_slices = 1 << len(w.sliced)
    K = n_slices if args.steps <= 0 else min(args.steps, n_slices)
    W = args.warmup
    main_res = run_network(tnrcs, torch, w, args.dtype, args.form, K, W, graph=not args.no_graph,
                           tune=not args.no_tune, tune_db=args.tune_db)
    by_kind, split = kernel_split(main_res, args.dtype)
    cc = copy_ceiling(tnrcs, torch)
    roof = roofline(by_kind, args.dtype, cc)
    if roof["bound"] == "hbm":
        log(f"[bench] {roof['kernel']}: {roof['achieved']:.0f} GB/s, {roof['frac']:.1%} of 8 TB/s, "
            f"{roof['achieved'] / cc:.1%} of the streaming copy probe ({cc:.0f} GB/s)")
    info = main_res["info"]
    main_res["plan"].close()
    del main_res["plan"]
    torch.cuda.empty_cache()

    if args.copy_probe_gib > 0:
        n = int(args.copy_probe_gib * 2**30) // 8
        src = torch.ones(n, dtype=torch.complex64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {n * 8} bytes read and written")
        del src, dst

    extra = {}
    if not args.no_extra:
        prec = {}
        for dt in ("f16s", "bf16s"):
            if dt == args.dtype:
                continue
            r = run_network(tnrcs, torch, w, dt, "auto", K, W, profile=(dt == "f16s"), tune=not args.no_tune,
                            tune_db=args.tune_db)
            err = float(np.linalg.norm(r["amp"] - main_res["amp"]) / np.linalg.norm(main_res["amp"]))
            prec[dt] = {"sec_per_slice": r["sec_per_slice"], "complex_tflops": r["tflops"],
                        "time_ratio_vs_" + args.dtype: main_res["sec_per_slice"] / r["sec_per_slice"],
                        "rel_err_vs_" + args.dtype: err, "flags": r["flags"]}
            if "ops" in r:
                bk, _ = kernel_split(r, dt)
                prec[dt]["roofline"] = roofline(bk, dt, cc)
            log(f"[bench] {dt}: {main_res['sec_per_slice'] / r['sec_per_slice']:.2f}x faster than {args.dtype}, "
                f"bunch relative error vs {args.dtype} over the {K} timed slices {err:.2e}")
            r["plan"].close()
            del r
            torch.cuda.empty_cache()
        extra["precision"] = prec
        extra["kernels"] = micro(tnrcs, torch, np)
        extra["oracle_timings"] = oracle_timings(tnrcs, torch, np, extra["kernels"])
        extra["batch_uneven"] = batch_uneven(tnrcs, torch, np, args.batch_cap, "f16s")
        extra["crosscheck_30q"] = crosscheck_30q(tnrcs, torch, np)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(w, args.cpu_sub_log2)
        log(f"[bench] oracle: {cpu['value']:.4f} TFLOP/s on {cpu['cores']} threads ({cpu['seconds']:.1f} s)")

    sec = main_res["sec_per_slice"]
    out = {
        "metric": METRIC,
        "value": main_res["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": "rqc-53q-6x9m1-d14: 53 qubits (6x9 grid, 1 seeded-missing site), 14 cycles, "
                        "6 open qubits (64-amplitude bunch), per-slice tensors <= 2^32 entries",
            "sec_per_slice": sec,
            "complex_tflops": main_res["tflops"],
            "complex_tflops_over_dtype_mfma_peak": main_res["tflops"] / PEAK[args.dtype],
            "n_slices_total": n_slices,
            "slices_timed": K,
            "time_to_amplitudes_s": sec * n_slices,
            "time_to_amplitudes_note": ("all slices of the bunch timed" if K == n_slices else
                                        f"{K} of {n_slices} slices timed, time per slice x slice count"),
            "time_to_amplitudes_with_plan_s": main_res["plan_s"] + sec * n_slices,
            "flops_per_slice": info["flops_per_slice"],
            "bytes_per_slice": info["bytes_per_slice"],
            "gemm_form": args.form,
            "graph": not args.no_graph,
            "tuned": not args.no_tune,
            "plan_s": main_res["plan_s"],
            "kernels_per_slice": info["n_kernels"],
            "kernel_split": split,
            "slice_roofline_frac": slice_roofline_frac(main_res, args.dtype),
            "numeric_flags": main_res["flags"],
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
