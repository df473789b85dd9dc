"""The allocation-free split-K GEMM (tn_cgemm_c64_noalloc) against
tn_cgemm_c64 with a caller-allocated slab workspace: the same kernels in the
same order, so the results must be bitwise equal.  Two calls in a row, the
second smaller, so the static scratch holds the first call's slabs when the
second one starts; then a call beyond the scratch must be refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2111_01066_amd import tnrcs  # noqa: E402

DEV = "cuda"
SCRATCH_ENTRIES = (64 << 20) // 8  # TN_NOALLOC_SCRATCH_BYTES / sizeof(complex64)


def _case(M, N, K, splits, form, seed):
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    A = torch.randn((M, K), dtype=torch.complex64, device=DEV, generator=g)
    B = torch.randn((N, K), dtype=torch.complex64, device=DEV, generator=g)
    ref = torch.empty((M, N), dtype=torch.complex64, device=DEV)
    work = torch.empty((max(splits, 1), M, N), dtype=torch.complex64, device=DEV)
    tnrcs.tn_cgemm_c64(A, B, ref, M, N, K, 1, form, work=work if splits > 1 else None, splits=splits)
    out = torch.full((M, N), float("nan"), dtype=torch.complex64, device=DEV)
    tnrcs.tn_cgemm_c64_noalloc(A, B, out, M, N, K, form, splits)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("form", ["4m", "3m"])
def test_noalloc_matches_workspace_gemm(form):
    # first call fills 16 x 512 x 512 = 4 Mi slab entries, the second a smaller 4 x 256 x 256
    for (M, N, K, splits, seed) in [(512, 512, 1 << 16, 16, 1), (256, 256, 4096, 4, 2), (384, 128, 2048, 1, 3)]:
        assert splits * M * N <= SCRATCH_ENTRIES
        print(f"noalloc gemm {form} M={M} N={N} K={K} splits={splits}", flush=True)
        ref, got = _case(M, N, K, splits, form, seed)
        np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_noalloc_rejects_oversized_split():
    M = N = 1024
    x = torch.zeros(M * 2048, dtype=torch.complex64, device=DEV)
    c = torch.zeros(M * N, dtype=torch.complex64, device=DEV)
    # 16 slabs of 1024 x 1024 need 128 MiB, twice the scratch
    with pytest.raises(tnrcs.TnError, match="static scratch"):
        tnrcs.tn_cgemm_c64_noalloc(x, x, c, M, N, 2048, "4m", 16)
    # 8 slabs fit exactly
    tnrcs.tn_cgemm_c64_noalloc(x, x, c, M, N, 2048, "4m", 8)
    torch.cuda.synchronize()
    assert float(c.abs().max()) == 0.0
