"""The 53-qubit, 14-cycle network itself on the GPU, pinned where an oracle
can reach it.  Its full sum over 2^15 slices is out of any oracle's reach,
but slicing is an exact identity (main text, TNC section: the network is the
sum over the values of its sliced wires): with 9 more wires sliced, every
tensor has at most 2^28 entries and one sub-slice is an FP64 contraction of
about 8e12 flop for the oracle.  So:

* one seeded sub-slice of slice 0, computed by the GPU through a plan over
  the extended sliced set, matches the oracle's FP64 pairwise contraction of
  the same sub-slice (complex64 1e-5, scaled FP16 1e-2, scaled BF16 6e-2);
* slice 0 of the benchmark plan (15 sliced wires, 2^32-entry
  intermediates) equals the sum of its 2^9 sub-slices computed by the
  extended plan.  Each side is held to the complex64 bar (1e-5 of its own
  norm), so the two may differ by up to 1e-5 (||slice 0|| + sum_e ||sub_e||);
  the sub-slices cancel in the sum, which is why the second term is
  not ||slice 0|| again."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle.tn import contract_network, slice_assignment  # noqa: E402
from paper_2111_01066_amd import tnrcs  # noqa: E402
from rqcgen import network_structure, slice_to_fit  # noqa: E402
from rqcgen.workloads import config3  # noqa: E402

TOL = {"c64": 1e-5, "f16s": 1e-2, "bf16s": 6e-2}
SUB_LOG2 = 28


@pytest.fixture(scope="module")
def sub():
    w = config3()
    ns = network_structure(w.circuit, w.open_qubits)
    allsl = slice_to_fit(ns, w.pairs, SUB_LOG2, initial=w.sliced)
    k = len(w.sliced)
    assert list(allsl[:k]) == list(w.sliced) and len(allsl) - k == 9
    e = int(np.random.default_rng(7).integers(1 << (len(allsl) - k)))
    s_ext = e << k  # slice 0 of the benchmark slicing, extra wires set to the bits of e
    print(f"config 3: oracle sub-slice {e} of slice 0 ({len(allsl) - k} extra wires)", flush=True)
    leaves, ow = oracle.build_network(w.circuit, w.open_qubits, w.out_bits)
    ref = contract_network(leaves, w.pairs, ow, slice_assignment(allsl, s_ext))
    return {"w": w, "allsl": allsl, "k": k, "s_ext": s_ext, "ref": ref}


@pytest.mark.parametrize("dtype", ["c64", "f16s", "bf16s"])
def test_config3_subslice_vs_oracle(sub, dtype):
    w = sub["w"]
    print(f"config 3 sub-slice {sub['s_ext']} {dtype}", flush=True)
    plan = tnrcs.Plan(w.circuit, w.pairs, sub["allsl"], w.open_qubits, w.out_bits, dtype=dtype)
    assert plan.info()["max_log2"] <= SUB_LOG2
    amp = torch.zeros(64, dtype=torch.complex128, device="cuda")
    plan.contract(sub["s_ext"], sub["s_ext"] + 1, amp)
    torch.cuda.synchronize()
    flags = plan.status()
    plan.close()
    assert flags & (tnrcs.FLAG_NONFINITE | tnrcs.FLAG_OVERFLOW) == 0
    err = oracle.relative_error_norm(amp.cpu().numpy(), sub["ref"])
    print(f"  relative error {err:.3e}", flush=True)
    assert err < TOL[dtype]


def test_config3_slice0_is_sum_of_subslices(sub):
    w, k = sub["w"], sub["k"]
    n_sub = 1 << (len(sub["allsl"]) - k)
    print(f"config 3 slice 0 against the sum of its {n_sub} sub-slices, c64", flush=True)
    ext = tnrcs.Plan(w.circuit, w.pairs, sub["allsl"], w.open_qubits, w.out_bits)
    parts = torch.zeros(n_sub, 64, dtype=torch.complex128, device="cuda")
    for e in range(n_sub):
        ext.contract(e << k, (e << k) + 1, parts[e])
    torch.cuda.synchronize()
    parts = parts.cpu().numpy()
    want = parts.sum(axis=0)
    sum_norms = float(np.linalg.norm(parts, axis=1).sum())
    assert ext.status() & (tnrcs.FLAG_NONFINITE | tnrcs.FLAG_OVERFLOW) == 0
    ext.close()
    print("  sub-slices done", flush=True)
    plan = tnrcs.Plan(w.circuit, w.pairs, w.sliced, w.open_qubits, w.out_bits)
    assert plan.info()["max_log2"] == 32
    amp = torch.zeros(64, dtype=torch.complex128, device="cuda")
    plan.contract(0, 1, amp)
    torch.cuda.synchronize()
    assert plan.status() & (tnrcs.FLAG_NONFINITE | tnrcs.FLAG_OVERFLOW) == 0
    plan.close()
    got = amp.cpu().numpy()
    diff = float(np.linalg.norm(got - want))
    bound = TOL["c64"] * (float(np.linalg.norm(got)) + sum_norms)
    print(f"  |difference| {diff:.3e}, relative {diff / np.linalg.norm(want):.3e}, bound {bound:.3e} "
          f"(sum of sub-slice norms / norm of the sum = {sum_norms / np.linalg.norm(want):.1f})", flush=True)
    assert diff < bound
