"""The 53-qubit, 14-cycle benchmark network itself on the GPU, pinned to the
FP64 oracle where the oracle can reach it.  Its full sum over 2^k slices is
out of any oracle's reach in this suite, but slicing is an exact identity
(main text, customized-TNC section: the network is the sum over the values
of its sliced wires):

* the slices that the fixture tests/golden/config3_slices.txt holds (slice 0,
  and the seeded slice once its oracle run has finished), computed by the
  benchmark plan (intermediates of up to 2^32 entries) exactly as the
  benchmark runs it (with the autotuner) and with the default kernel rules,
  match the fixture, which the oracle alone wrote as sums of sub-slices
  (complex64 1e-5, scaled FP16 1e-2, scaled BF16 6e-2, normwise);
* for slice 0 and for the seeded slice: one seeded sub-slice (more wires
  sliced until every tensor has at most 2^29 entries), computed by the GPU
  through a plan over the extended sliced set, matches the oracle's FP64
  contraction of the same sub-slice, computed here;
* slice 0 and the seeded slice of the benchmark plan each equal the sum of
  their sub-slices computed by the extended plan, within 1e-5 of the sum's
  norm."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from oracle.tn import contract_network, slice_assignment  # noqa: E402
from paper_2111_01066_amd import tnrcs  # noqa: E402
from rqcgen import network_structure, slice_to_fit  # noqa: E402
from rqcgen.workloads import config3  # noqa: E402
from tests.golden import make_config3_slice_golden as golden  # noqa: E402

TOL = {"c64": 1e-5, "f16s": 1e-2, "bf16s": 6e-2}
SUB_LOG2 = 29


@pytest.fixture(scope="module")
def work():
    return config3()


@pytest.fixture(scope="module")
def fixture_amps(work):
    if not os.path.exists(golden.OUT):
        pytest.skip("tests/golden/config3_slices.txt not written yet (tests/golden/make_config3_slice_golden.py)")
    digest, amps = golden.load()
    assert digest == golden.order_digest(work.pairs, work.sliced), "fixture written for another order"
    return amps


@pytest.mark.parametrize("tune", [True, False])
@pytest.mark.parametrize("dtype", ["c64", "f16s", "bf16s"])
def test_config3_slices_vs_oracle_fixture(work, fixture_amps, dtype, tune):
    w = work
    print(f"config 3 fixture slices {sorted(fixture_amps)} {dtype} tune={tune}", flush=True)
    plan = tnrcs.Plan(w.circuit, w.pairs, w.sliced, w.open_qubits, w.out_bits, dtype=dtype, tune=tune)
    assert plan.info()["max_log2"] == 32
    for s, ref in sorted(fixture_amps.items()):
        amp = torch.zeros(64, dtype=torch.complex128, device="cuda")
        plan.contract(s, s + 1, amp)
        torch.cuda.synchronize()
        err = oracle.relative_error_norm(amp.cpu().numpy(), ref)
        print(f"  slice {s}: normwise relative error {err:.3e}", flush=True)
        assert err < TOL[dtype]
    flags = plan.status()
    plan.close()
    assert flags & (tnrcs.FLAG_NONFINITE | tnrcs.FLAG_OVERFLOW) == 0


@pytest.fixture(scope="module", params=["slice0", "seeded"])
def sub(work, request):
    w = work
    ns = network_structure(w.circuit, w.open_qubits)
    allsl = slice_to_fit(ns, w.pairs, SUB_LOG2, initial=w.sliced)
    k = len(w.sliced)
    assert list(allsl[:k]) == list(w.sliced) and len(allsl) > k
    s = 0 if request.param == "slice0" else golden.seeded_slice(k)
    e = int(np.random.default_rng(7).integers(1 << (len(allsl) - k)))
    s_ext = s | (e << k)  # slice s of the benchmark slicing, extra wires set to the bits of e
    print(f"config 3: oracle sub-slice {e} of slice {s} ({len(allsl) - k} extra wires)", flush=True)
    leaves, ow = oracle.build_network(w.circuit, w.open_qubits, w.out_bits)
    ref = contract_network(leaves, w.pairs, ow, slice_assignment(allsl, s_ext))
    return {"allsl": allsl, "k": k, "s": s, "s_ext": s_ext, "ref": ref}


@pytest.mark.parametrize("dtype", ["c64", "f16s", "bf16s"])
def test_config3_subslice_vs_oracle(work, sub, dtype):
    w = work
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


def test_config3_slice_is_sum_of_subslices(work, sub):
    w, k, s = work, sub["k"], sub["s"]
    n_sub = 1 << (len(sub["allsl"]) - k)
    print(f"config 3 slice {s} against the sum of its {n_sub} sub-slices, c64", flush=True)
    ext = tnrcs.Plan(w.circuit, w.pairs, sub["allsl"], w.open_qubits, w.out_bits)
    parts = torch.zeros(n_sub, 64, dtype=torch.complex128, device="cuda")
    for e in range(n_sub):
        ext.contract(s | (e << k), (s | (e << k)) + 1, parts[e])
    torch.cuda.synchronize()
    parts = parts.cpu().numpy()
    want = parts.sum(axis=0)
    assert ext.status() & (tnrcs.FLAG_NONFINITE | tnrcs.FLAG_OVERFLOW) == 0
    ext.close()
    plan = tnrcs.Plan(w.circuit, w.pairs, w.sliced, w.open_qubits, w.out_bits)
    assert plan.info()["max_log2"] == 32
    amp = torch.zeros(64, dtype=torch.complex128, device="cuda")
    plan.contract(s, s + 1, amp)
    torch.cuda.synchronize()
    assert plan.status() & (tnrcs.FLAG_NONFINITE | tnrcs.FLAG_OVERFLOW) == 0
    plan.close()
    err = oracle.relative_error_norm(amp.cpu().numpy(), want)
    ratio = float(np.linalg.norm(parts, axis=1).sum() / np.linalg.norm(want))
    print(f"  normwise relative difference {err:.3e} (sum of sub-slice norms / norm of the sum = {ratio:.1f})",
          flush=True)
    assert err < TOL["c64"]
