"""GPU kernels through the C ABI: permute (bit-exact vs numpy), complex GEMM
4M/3M (vs FP64 numpy), FP64 reductions."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2111_01066_amd import tnrcs  # noqa: E402

DEV = "cuda"


def _np_permute(x, perm):
    r = len(perm)
    o = np.arange(1 << r, dtype=np.int64)
    i = np.zeros_like(o)
    for q, p in enumerate(perm):
        i |= ((o >> q) & 1) << p
    return x[..., i]


# FP32 accumulation in runs of at most 2048 terms (longer contractions add
# the runs, split-K slabs are summed in FP64): the normwise relative error of
# a complex GEMM on random Gaussian operands stays near 0.4 u sqrt(1024)
# ~ 8e-7 (u = 2^-24) whatever K is; the bound leaves a factor of 3.
GEMM_C64_TOL = 2.5e-6


def _rand_c64(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)


@pytest.mark.parametrize("rank", [0, 1, 2, 3, 5, 8, 11, 12, 13, 16, 20, 23])
def test_permute_bit_exact(rank):
    rng = np.random.default_rng(rank)
    for trial in range(3):
        perm = rng.permutation(rank).tolist()
        if trial == 1:
            perm = list(range(rank))
        if trial == 2 and rank > 4:
            perm = list(range(rank))[::-1]
        x = _rand_c64(rng, 2, 1 << rank)
        xin = torch.from_numpy(x).to(DEV)
        out = torch.empty_like(xin)
        print(f"permute rank={rank} trial={trial}", flush=True)
        tnrcs.tn_permute(xin, out, perm, batch=2)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), _np_permute(x, perm))


def _gpu_source_index(rank, perm):
    """Input index of every output index, computed on the device."""
    o = torch.arange(1 << rank, dtype=torch.int64, device=DEV)
    i = torch.zeros_like(o)
    for q, p in enumerate(perm):
        i |= ((o >> q) & 1) << p
    return i


@pytest.mark.parametrize("rank,elem_bytes", [(29, 8), (30, 4)])
def test_permute_many_tiles_per_block(rank, elem_bytes):
    """Tensors with more tiles than blocks (16384 blocks, tiles of 2^12 or
    2^13 elements), so each block walks several tiles and advances its
    tile-id offsets in the loop; every element is checked bit-exact (each
    input element holds its own index)."""
    rng = np.random.default_rng(7 * rank)
    dt = torch.int64 if elem_bytes == 8 else torch.int32
    x = torch.arange(1 << rank, dtype=dt, device=DEV)
    out = torch.empty_like(x)
    for trial, perm in enumerate([rng.permutation(rank).tolist(), list(range(rank))[::-1],
                                  list(range(rank // 2, rank)) + list(range(rank // 2))]):
        print(f"permute rank={rank} elem_bytes={elem_bytes} trial={trial}", flush=True)
        out.fill_(-1)
        tnrcs.tn_permute(x, out, perm, batch=1, elem_bytes=elem_bytes)
        torch.cuda.synchronize()
        want = _gpu_source_index(rank, perm).to(dt)
        bad = int((out != want).sum())
        assert bad == 0, f"{bad} wrong elements"
        del want


def test_permute_rejects_bad_perm():
    x = torch.zeros(8, dtype=torch.complex64, device=DEV)
    with pytest.raises(tnrcs.TnError):
        tnrcs.tn_permute(x, torch.empty_like(x), [0, 0, 1])


@pytest.mark.parametrize("form", ["4m", "3m"])
@pytest.mark.parametrize("M,N,K,batch", [(64, 64, 16, 1), (128, 64, 48, 2), (256, 192, 512, 1),
                                         (64, 512, 4096, 1), (128, 128, 16, 1), (256, 384, 1024, 2),
                                         (512, 256, 4096, 1), (1280, 256, 256, 1), (384, 1152, 64, 1)])
def test_cgemm_matches_fp64(form, M, N, K, batch):
    rng = np.random.default_rng(M + N + K)
    A = _rand_c64(rng, batch, M, K)
    B = _rand_c64(rng, batch, N, K)
    ref = np.einsum("bmk,bnk->bmn", A.astype(np.complex128), B.astype(np.complex128))
    dA, dB = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    dC = torch.empty((batch, M, N), dtype=torch.complex64, device=DEV)
    print(f"cgemm {form} M={M} N={N} K={K} batch={batch}", flush=True)
    tnrcs.tn_cgemm_c64(dA, dB, dC, M, N, K, batch, form)
    torch.cuda.synchronize()
    C = dC.cpu().numpy().astype(np.complex128)
    err = np.linalg.norm(C - ref) / np.linalg.norm(ref)
    assert err < GEMM_C64_TOL, err


@pytest.mark.parametrize("form", ["4m", "3m"])
@pytest.mark.parametrize("M,N,K,splits", [(128, 128, 4096, 4), (256, 128, 65536, 16), (128, 256, 2048, 8),
                                           (192, 64, 32768, 16), (64, 320, 8192, 4)])
def test_cgemm_split_k(form, M, N, K, splits):
    """128x128-tile slabs, and 64x64-tile slabs when an extent is not a
    multiple of 128."""
    rng = np.random.default_rng(M * 7 + K)
    A = _rand_c64(rng, M, K)
    B = _rand_c64(rng, N, K)
    ref = A.astype(np.complex128) @ B.astype(np.complex128).T
    dA, dB = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    dC = torch.empty((M, N), dtype=torch.complex64, device=DEV)
    work = torch.empty((splits, M, N), dtype=torch.complex64, device=DEV)
    print(f"cgemm split-K {form} M={M} N={N} K={K} splits={splits}", flush=True)
    tnrcs.tn_cgemm_c64(dA, dB, dC, M, N, K, 1, form, work=work, splits=splits)
    torch.cuda.synchronize()
    C = dC.cpu().numpy().astype(np.complex128)
    err = np.linalg.norm(C - ref) / np.linalg.norm(ref)
    assert err < GEMM_C64_TOL, err
    with pytest.raises(tnrcs.TnError):
        tnrcs.tn_cgemm_c64(dA, dB, dC, M, N, K, 1, form, work=None, splits=splits)


@pytest.mark.parametrize("form", ["4m", "3m"])
@pytest.mark.parametrize("K,splits", [(1 << 17, 1), (1 << 17, 4), (1 << 22, 16)])
def test_cgemm_long_k_sampled(form, K, splits):
    """Contractions as long as the 53-qubit network's (K = 2^17, 2^22): 64
    sampled entries against FP64 sums of the same complex64 operands."""
    M = N = 128
    g = torch.Generator(device=DEV)
    g.manual_seed(K + splits)
    dA = torch.randn((M, K), dtype=torch.complex64, device=DEV, generator=g)
    dB = torch.randn((N, K), dtype=torch.complex64, device=DEV, generator=g)
    dC = torch.empty((M, N), dtype=torch.complex64, device=DEV)
    work = torch.empty((splits, M, N), dtype=torch.complex64, device=DEV) if splits > 1 else None
    print(f"cgemm long K {form} K={K} splits={splits}", flush=True)
    tnrcs.tn_cgemm_c64(dA, dB, dC, M, N, K, 1, form, work=work, splits=splits)
    torch.cuda.synchronize()
    rng = np.random.default_rng(K)
    rows = np.sort(rng.choice(M, 8, replace=False))
    cols = np.sort(rng.choice(N, 8, replace=False))
    a = dA[torch.from_numpy(rows).to(DEV)].cpu().numpy().astype(np.complex128)
    b = dB[torch.from_numpy(cols).to(DEV)].cpu().numpy().astype(np.complex128)
    ref = a @ b.T
    got = dC.cpu().numpy()[np.ix_(rows, cols)].astype(np.complex128)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"  normwise relative error {err:.2e}", flush=True)
    assert err < GEMM_C64_TOL, err


def test_cgemm_rejects_bad_shape():
    x = torch.zeros(64 * 64, dtype=torch.complex64, device=DEV)
    with pytest.raises(tnrcs.TnError):
        tnrcs.tn_cgemm_c64(x, x, x, 64, 64, 8, 1, "4m")


def test_reductions():
    rng = np.random.default_rng(3)
    n = 1 << 18
    a = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * 1e-3
    d = torch.from_numpy(a).to(DEV)
    out = torch.zeros(2, dtype=torch.float64, device=DEV)
    tnrcs.tn_amp_norm2(d, n, out)
    torch.cuda.synchronize()
    assert abs(out[0].item() - np.sum(np.abs(a) ** 2)) < 1e-12 * np.sum(np.abs(a) ** 2)
    idx = rng.integers(0, n, size=5000)
    didx = torch.from_numpy(idx).to(DEV)
    tnrcs.tn_amp_xeb(d, n, didx, idx.size, out)
    torch.cuda.synchronize()
    p = np.abs(a[idx]) ** 2
    np.testing.assert_allclose(out.cpu().numpy(), [p.sum(), (p * p).sum()], rtol=1e-12)
    counts = torch.zeros(16, dtype=torch.int64, device=DEV)
    scale = n / np.sum(np.abs(a) ** 2)
    tnrcs.tn_amp_hist(d, n, scale, 8.0, 16, counts)
    torch.cuda.synchronize()
    x = scale * np.abs(a) ** 2
    ref = np.minimum((x / 8.0 * 16).astype(np.int64), 15)
    np.testing.assert_array_equal(counts.cpu().numpy(), np.bincount(ref, minlength=16))


def _to_pairs(z, dtype):
    """complex array -> torch tensor of (re, im) 16-bit pairs (last dim 2)."""
    t = torch.stack([torch.from_numpy(np.ascontiguousarray(z.real)), torch.from_numpy(np.ascontiguousarray(z.imag))],
                    dim=-1)
    return t.to(torch.float16 if dtype == "f16s" else torch.bfloat16).contiguous()


def _from_pairs(t):
    x = t.float().cpu().numpy().astype(np.float64)
    return x[..., 0] + 1j * x[..., 1]


@pytest.mark.parametrize("rank", [3, 9, 12, 13, 14, 16, 21, 24])
def test_permute_4byte_bit_exact(rank):
    """Four-byte elements (FP16/BF16 pairs), tiles of up to 2^13 elements."""
    rng = np.random.default_rng(100 + rank)
    x = rng.integers(0, 2**31, size=(3, 1 << rank), dtype=np.int64).astype(np.int32)
    xin = torch.from_numpy(x).to(DEV)
    for trial in range(3):
        perm = rng.permutation(rank).tolist()
        if trial == 1:
            perm = list(range(rank))[::-1]
        if trial == 2:
            perm = list(range(rank // 2, rank)) + list(range(rank // 2))
        out = torch.empty_like(xin)
        print(f"permute 4-byte rank={rank} trial={trial}", flush=True)
        tnrcs.tn_permute(xin, out, perm, batch=3, elem_bytes=4)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), _np_permute(x, perm))


@pytest.mark.parametrize("dtype", ["f16s", "bf16s"])
@pytest.mark.parametrize("form", ["4m", "3m"])
@pytest.mark.parametrize("M,N,K,batch,splits", [(128, 128, 16, 1, 1), (256, 384, 1024, 2, 1),
                                                (128, 256, 4096, 1, 8), (512, 128, 96, 1, 1), (64, 192, 32, 1, 1),
                                                (1280, 256, 128, 1, 1), (192, 320, 1024, 1, 4),
                                                # 128x256 tiles (N a multiple of 256, K slabs >= 1024)
                                                (256, 512, 2048, 1, 1), (128, 256, 8192, 1, 2),
                                                (384, 768, 1024, 3, 1),
                                                # long K: one wave per SIMD, 64-deep stages
                                                (128, 128, 16384, 1, 1), (256, 128, 65536, 1, 2)])
def test_cgemm_half(dtype, form, M, N, K, batch, splits):
    rng = np.random.default_rng(M + 3 * N + K)
    A = rng.standard_normal((batch, M, K)) + 1j * rng.standard_normal((batch, M, K))
    B = rng.standard_normal((batch, N, K)) + 1j * rng.standard_normal((batch, N, K))
    dA, dB = _to_pairs(A, dtype).to(DEV), _to_pairs(B, dtype).to(DEV)
    Aq, Bq = _from_pairs(dA), _from_pairs(dB)  # the rounded inputs
    ref = np.einsum("bmk,bnk->bmn", Aq, Bq)
    scale = 2.0 ** -int(np.ceil(np.log2(np.abs(ref).max())) - 12)
    dC = torch.empty((batch, M, N, 2), dtype=dA.dtype, device=DEV)
    mx = torch.zeros(1, dtype=torch.float32, device=DEV)
    work = torch.empty((splits, M, N), dtype=torch.complex64, device=DEV) if splits > 1 else None
    print(f"cgemm_half {dtype} {form} M={M} N={N} K={K} batch={batch} splits={splits}", flush=True)
    tnrcs.tn_cgemm_half(dtype, dA, dB, dC, M, N, K, batch, form, out_scale=scale, work=work, splits=splits,
                        max_out=mx)
    torch.cuda.synchronize()
    C = _from_pairs(dC) / scale
    err = np.linalg.norm(C - ref) / np.linalg.norm(ref)
    u = 2.0 ** -11 if dtype == "f16s" else 2.0 ** -8
    # output rounding (and, for 3M, the rounded re+im operand sums)
    assert err < (2 if form == "4m" else 4) * u + 1e-6 * np.sqrt(K), err
    # the record is the largest |component| of the FP32 result before rounding
    comp_max = max(np.abs(C.real).max(), np.abs(C.imag).max())
    assert abs(mx.item() - comp_max) <= 2 * u * comp_max


def test_probes_copy_and_mfma_loop():
    """The ceiling probes: the streaming copy is exact (including a tail
    shorter than one grid stride) and the MFMA loops run and report their
    flop count."""
    n = (1 << 20) + 48
    src = torch.arange(n, dtype=torch.int32, device=DEV)
    dst = torch.zeros_like(src)
    tnrcs.tn_probe_copy(src, dst, n * 4)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    out = torch.empty(tnrcs.tn_probe_mfma_out_floats(), dtype=torch.float32, device=DEV)
    for kind, k in (("f32", 2), ("f16", 16), ("bf16", 16)):
        fl = tnrcs.tn_probe_mfma(kind, 10, out)
        torch.cuda.synchronize()
        assert fl == 2.0 * 32 * 32 * k * 4 * 10 * (out.numel() // 64)
        assert torch.isfinite(out).all()
