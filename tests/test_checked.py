"""Checked slices for scaled storage (tn_contract_slices_checked): a clean
run adds the same sums as the unchecked path; when the calibrated shifts do
not fit (forced here with tn_plan_shift_outputs), the range flags fire, the
plan recalibrates on the offending slice, runs it again and the result still
meets the oracle bar."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_2111_01066_amd import tnrcs  # noqa: E402
from rqcgen import make_rqc, network_structure, random_bitstrings, slice_to_fit  # noqa: E402
from rqcgen.order import bisection_order  # noqa: E402

TOL = {"c64": 1e-5, "f16s": 1e-2, "bf16s": 6e-2}


@pytest.fixture(scope="module")
def net():
    c = make_rqc(4, 5, 10, seed=5)
    open_q = [0, 1, 2, 3, 4, 5]
    bits = random_bitstrings(20, 1, seed=8)[0]
    ns = network_structure(c, open_q)
    pairs = bisection_order(ns, seed=0)
    sliced = slice_to_fit(ns, pairs, 18)
    assert len(sliced) == 3
    return c, open_q, bits, pairs, sliced, oracle.amplitudes_sv(c, open_q, bits)


def _plan(net, dtype):
    c, open_q, bits, pairs, sliced, _ = net
    return tnrcs.Plan(c, pairs, sliced, open_q, bits, dtype=dtype)


def _zeros():
    return torch.zeros(64, dtype=torch.complex128, device="cuda")


@pytest.mark.parametrize("dtype", ["c64", "f16s", "bf16s"])
def test_checked_equals_unchecked_when_clean(net, dtype):
    print(f"checked == unchecked {dtype}", flush=True)
    p = _plan(net, dtype)
    n = p.info()["n_slices"]
    a0, a1 = _zeros(), _zeros()
    p.contract(0, n, a0)
    assert p.contract_checked(0, n, a1) == 0
    torch.cuda.synchronize()
    x0, x1 = a0.cpu().numpy(), a1.cpu().numpy()
    np.testing.assert_allclose(x1, x0, rtol=0, atol=1e-13 * np.abs(x0).max())
    assert oracle.relative_error_norm(x1, net[5]) < TOL[dtype]
    assert p.status() == 0
    p.close()


@pytest.mark.parametrize("dtype", ["f16s", "bf16s"])
@pytest.mark.parametrize("delta,flag", [(-20, tnrcs.FLAG_OVERFLOW), (20, tnrcs.FLAG_UNDERFLOW)])
def test_range_flags_and_recalibration(net, dtype, delta, flag):
    print(f"forced shift {delta} {dtype}", flush=True)
    # unchecked: the range check raises the flag
    p = _plan(net, dtype)
    n = p.info()["n_slices"]
    p.shift_outputs(delta)
    a = _zeros()
    p.contract(0, n, a)
    assert p.status() & flag
    p.close()
    # checked: the first slice is recalibrated and re-run, the rest fit
    p = _plan(net, dtype)
    p.shift_outputs(delta)
    a = _zeros()
    retries = p.contract_checked(0, n, a)
    torch.cuda.synchronize()
    assert retries == 1
    assert p.status() == 0
    err = oracle.relative_error_norm(a.cpu().numpy(), net[5])
    print(f"  relative error after recalibration {err:.2e}", flush=True)
    assert err < TOL[dtype]
    p.close()


def test_shift_outputs_rejects_complex64(net):
    p = _plan(net, "c64")
    with pytest.raises(tnrcs.TnError) as e:
        p.shift_outputs(1)
    assert e.value.code == -1
    p.close()


@pytest.mark.parametrize("dtype", ["f16s", "bf16s"])
def test_power_of_two_shift_is_exact(net, dtype):
    """Scaled storage is exact under a power-of-two change of one exponent:
    moving one kernel's output shift by +-1 doubles or halves every stored
    value downstream of it and the root exponent compensates, so while
    nothing leaves the normal range the amplitudes are bitwise identical.
    Checked for the kernels whose stored results stay far from the range
    limits (all but those that produce the root)."""
    n = None
    ref = None
    p = _plan(net, dtype)
    n = p.info()["n_slices"]
    ops = p.json()["ops"]
    a = _zeros()
    p.contract(0, n, a)
    torch.cuda.synchronize()
    ref = a.cpu().numpy()
    p.close()
    producing = [i for i, o in enumerate(ops) if o["kind"] != 0]
    assert len(producing) >= 4
    for i in producing[:4]:
        for delta in (1, -1):
            print(f"shift +-1 exactness {dtype}: kernel {i} delta {delta}", flush=True)
            p = _plan(net, dtype)
            p.shift_outputs(delta, op=i)
            a = _zeros()
            p.contract(0, n, a)
            torch.cuda.synchronize()
            assert p.status() == 0
            assert np.array_equal(a.cpu().numpy(), ref), (i, delta)
            p.close()
