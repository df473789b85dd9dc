"""End-to-end sliced contraction on the GPU through the C ABI vs the FP64
oracle (complex64 bar: normwise relative amplitude error <= 1e-5)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2111_01066_amd import tnrcs  # noqa: E402
from rqcgen import make_rqc, network_structure, random_bitstrings, slice_to_fit, Circuit, Gate  # noqa: E402
from rqcgen.order import bisection_order, greedy_order  # noqa: E402

TOL_C64 = 1e-5
DEV = "cuda"


def _amps(plan, n_open, ranges):
    amp = torch.zeros(1 << n_open, dtype=torch.complex128, device=DEV)
    for a, b in ranges:
        plan.contract(a, b, amp)
    torch.cuda.synchronize()
    return amp.cpu().numpy()


@pytest.fixture(scope="module")
def c1():
    c = make_rqc(4, 5, 8, seed=0)
    psi = oracle.statevector(c).reshape(-1)
    return c, psi


@pytest.mark.parametrize("use_graph", [True, False])
def test_config1_all_open_vs_statevector(c1, use_graph):
    c, psi = c1
    open_q = list(range(20))
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=0)
    print(f"C1 all-open graph={use_graph}", flush=True)
    plan = tnrcs.Plan(c, pairs, [], open_q, None, use_graph=use_graph)
    amp = _amps(plan, 20, [(0, 1)])
    assert plan.status() == 0
    err = oracle.relative_error_norm(amp, psi)
    assert err < TOL_C64, err
    # the config's 64 uniformly random bit strings, gathered from the bunch
    bs = random_bitstrings(20, 64, seed=1)
    idx = [int("".join(map(str, b)), 2) for b in bs]
    assert oracle.relative_error_norm(amp[idx], psi[idx]) < TOL_C64
    # FP64 norm reduction on the GPU
    out = torch.zeros(1, dtype=torch.float64, device=DEV)
    d = torch.from_numpy(amp).to(DEV)
    tnrcs.tn_amp_norm2(d, amp.size, out)
    assert abs(out.item() - 1.0) < 1e-5
    plan.close()


def test_config1_closed_bitstrings_greedy_order(c1):
    c, psi = c1
    ns = network_structure(c, [])
    pairs = greedy_order(ns, seed=0)
    bs = random_bitstrings(20, 4, seed=1)
    plan = tnrcs.Plan(c, pairs, [], [], bs[0])
    got, ref = [], []
    for b in bs:
        plan.set_output_bits(b)
        print("C1 closed", "".join(map(str, b)), flush=True)
        got.append(_amps(plan, 0, [(0, 1)])[0])
        ref.append(psi[int("".join(map(str, b)), 2)])
    plan.close()
    # normwise over the four closed amplitudes, the complex64 bar
    assert oracle.relative_error_norm(got, ref) < TOL_C64


@pytest.mark.parametrize("S,open_q", [(14, [0, 7, 13, 19]), (12, [3, 4])])
def test_sliced_sum_and_split_ranges(c1, S, open_q):
    c, psi = c1
    bits = random_bitstrings(20, 1, seed=5)[0]
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=1)
    sliced = slice_to_fit(ns, pairs, S)
    assert len(sliced) >= 2
    print(f"C1 sliced S={S} k={len(sliced)}", flush=True)
    plan = tnrcs.Plan(c, pairs, sliced, open_q, bits)
    n = 1 << len(sliced)
    full = _amps(plan, len(open_q), [(0, n)])
    ref = oracle.amplitudes_sv(c, open_q, bits)
    assert oracle.relative_error_norm(full, ref) < TOL_C64
    split = _amps(plan, len(open_q), [(0, 1), (1, n // 2), (n // 2, n // 2), (n // 2, n)])
    np.testing.assert_array_equal(split, full)   # same additions in the same order
    with pytest.raises(tnrcs.TnError):
        plan.contract(0, n + 1, torch.zeros(1 << len(open_q), dtype=torch.complex128, device=DEV))
    # per-slice values against the oracle's sliced network
    leaves, ow = oracle.build_network(c, open_q, bits)
    from oracle.tn import contract_slice
    for s in (0, n - 1):
        one = _amps(plan, len(open_q), [(s, s + 1)])
        ref_s = contract_slice(leaves, pairs, ow, sliced, s)
        assert oracle.relative_error_norm(one, ref_s) < TOL_C64
    plan.close()


@pytest.mark.parametrize("d,open_q,S", [(12, list(range(20)), 24), (12, [], 22), (10, [0, 1, 2, 3, 4, 5], 20)])
def test_deeper_circuit_dense_and_splitk_steps(d, open_q, S):
    c = make_rqc(4, 5, d, seed=5)
    bits = random_bitstrings(20, 1, seed=8)[0]
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=0)
    sliced = slice_to_fit(ns, pairs, S)
    plan = tnrcs.Plan(c, pairs, sliced, open_q, bits)
    info = plan.info()
    kinds = [o["kind"] for o in plan.json()["ops"]]
    assert info["n_dense"] > 0
    print(f"4x5 d={d} open={len(open_q)} dense={info['n_dense']} splitk={kinds.count(4)} k={len(sliced)}",
          flush=True)
    amp = _amps(plan, len(open_q), [(0, info["n_slices"])])
    ref = oracle.amplitudes_sv(c, open_q, bits)
    assert oracle.relative_error_norm(amp, ref) < TOL_C64
    plan.close()


def test_tiny_networks():
    c = Circuit(1, [])
    plan = tnrcs.Plan(c, [], [], [0], None)
    np.testing.assert_allclose(_amps(plan, 1, [(0, 1)]), [1, 0])
    plan.close()
    c = make_rqc(2, 2, 3, seed=2, two_qubit=False)
    open_q = [0, 1, 2, 3]
    ns = network_structure(c, open_q)
    plan = tnrcs.Plan(c, greedy_order(ns, 0), [], open_q, None)
    np.testing.assert_allclose(_amps(plan, 4, [(0, 1)]), oracle.statevector(c).reshape(-1), atol=1e-6)
    plan.close()


TOL_HALF = {"f16s": 1e-2, "bf16s": 6e-2}


@pytest.mark.parametrize("dtype", ["f16s", "bf16s"])
@pytest.mark.parametrize("d,open_q,S", [(8, list(range(20)), 40), (12, [], 22), (10, [0, 1, 2, 3, 4, 5], 20),
                                        (12, list(range(20)), 24)])
def test_scaled_half_precision_vs_oracle(dtype, d, open_q, S):
    c = make_rqc(4, 5, d, seed=5)
    bits = random_bitstrings(20, 1, seed=8)[0]
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=0)
    sliced = slice_to_fit(ns, pairs, S)
    print(f"{dtype} 4x5 d={d} open={len(open_q)} k={len(sliced)}", flush=True)
    plan = tnrcs.Plan(c, pairs, sliced, open_q, bits, dtype=dtype)
    info = plan.info()
    amp = _amps(plan, len(open_q), [(0, info["n_slices"])])
    flags = plan.status()
    ref = oracle.amplitudes_sv(c, open_q, bits)
    err = oracle.relative_error_norm(amp, ref)
    print(f"  relative error {err:.3e}, flags {flags}", flush=True)
    assert flags & (tnrcs.FLAG_NONFINITE | tnrcs.FLAG_OVERFLOW) == 0
    assert err < TOL_HALF[dtype], err
    plan.close()
