"""ctypes binding of libtnrcs.so (argument marshalling only).

Every function here converts Python arguments to the C ABI declared in
include/tnrcs.h and calls it; all contraction work runs in the library's
gfx950 kernels.  PyTorch tensors provide device memory and streams.  The
shared library must have been built (paper_2111_01066_amd.build.build());
importing this module without it raises ImportError.
"""
from __future__ import annotations

import ctypes
import json
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int32, c_int64, c_uint8, c_uint32, c_void_p
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtnrcs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2111_01066_amd.build.build() "
                      "(hipcc, gfx950) before using the library")
# PyTorch ships its own HIP runtime; load it first so that the library binds
# to the same runtime instance (two runtimes in one process do not share
# devices, streams or memory).
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = ctypes.CDLL(LIB_PATH)

TN_OK = 0
ERRORS = {-1: "TN_E_ARG", -2: "TN_E_TOPOLOGY", -3: "TN_E_MEM", -4: "TN_E_HIP",
          -5: "TN_E_UNSUPPORTED", -6: "TN_E_NUMERIC"}
DTYPES = {"c64": 0, "f16s": 1, "bf16s": 2}
GEMM_FORMS = {"auto": 0, "4m": 1, "3m": 2}
FLAG_NONFINITE, FLAG_OVERFLOW, FLAG_UNDERFLOW = 1, 2, 4


class TnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class tn_gate(ctypes.Structure):
    _fields_ = [("nq", c_int32), ("q", c_int32 * 2), ("m", c_double * 32)]


class tn_circuit(ctypes.Structure):
    _fields_ = [("n_qubits", c_int32), ("n_gates", c_int32), ("gates", POINTER(tn_gate)),
                ("out_bits", POINTER(c_uint8))]


class tn_plan_opts(ctypes.Structure):
    _fields_ = [("dtype", c_int32), ("gemm_form", c_int32), ("max_log2", c_int32), ("use_graph", c_int32),
                ("dry_run", c_int32), ("device", c_int32), ("host_fold_log2", c_int32),
                ("tune", c_int32), ("arena_bytes", c_int64), ("arena", c_void_p), ("tune_db", c_char_p)]


class tn_plan_stats(ctypes.Structure):
    _fields_ = [("n_slices", c_int64), ("n_leaves", c_int32), ("n_host_steps", c_int32),
                ("n_device_steps", c_int32), ("n_kernels", c_int32), ("max_log2", c_int32),
                ("n_open", c_int32), ("flops_per_slice", c_double), ("bytes_per_slice", c_double),
                ("moved_per_slice", c_double), ("arena_bytes", c_int64), ("leaf_bytes", c_int64),
                ("n_dense", c_int32), ("n_skinny", c_int32), ("n_generic", c_int32), ("n_permute", c_int32),
                ("k_hist", c_int32 * 64)]


_lib.tn_last_error.restype = c_char_p
_lib.tn_plan_opts_default.argtypes = [POINTER(tn_plan_opts)]
_lib.tn_plan_opts_default.restype = None
_lib.tn_plan.argtypes = [POINTER(tn_circuit), POINTER(c_int32), c_int32, POINTER(c_int32), c_int32,
                         POINTER(c_int32), c_int32, POINTER(tn_plan_opts), POINTER(c_void_p)]
_lib.tn_contract_slices.argtypes = [c_void_p, c_int64, c_int64, c_void_p, c_void_p]
_lib.tn_plan_info.argtypes = [c_void_p, POINTER(tn_plan_stats)]
_lib.tn_plan_json.argtypes = [c_void_p, c_char_p, c_int64, POINTER(c_int64)]
_lib.tn_plan_leaf.argtypes = [c_void_p, c_int32, POINTER(c_double), c_int64]
_lib.tn_plan_status.argtypes = [c_void_p, POINTER(c_uint32)]
_lib.tn_plan_set_output_bits.argtypes = [c_void_p, POINTER(c_uint8)]
_lib.tn_plan_destroy.argtypes = [c_void_p]
_lib.tn_plan_profile.argtypes = [c_void_p, c_int64, c_void_p, c_void_p, POINTER(ctypes.c_float), c_int32,
                                 POINTER(c_int32)]
_lib.tn_pair_plan.argtypes = [c_int32, POINTER(c_int32), c_int32, POINTER(c_int32), c_int32, POINTER(c_int32),
                              POINTER(tn_plan_opts), POINTER(c_void_p)]
_lib.tn_pair_run.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, ctypes.c_float, c_void_p]
_lib.tn_permute.argtypes = [c_void_p, c_void_p, c_int32, c_int32, POINTER(c_int32), c_int64, c_void_p]
_lib.tn_cgemm_half.argtypes = [c_int32, c_void_p, c_void_p, c_void_p, c_int64, c_int64, c_int64, c_int64, c_int32,
                               ctypes.c_float, c_void_p, c_int32, c_void_p, c_void_p]
_lib.tn_cgemm_c64.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_int64, c_int64, c_int64, c_int32,
                              c_void_p, c_int32, c_void_p]
_lib.tn_cgemm_c64_noalloc.argtypes = [c_void_p, c_void_p, c_void_p, c_int64, c_int64, c_int64, c_int32, c_int32,
                                         c_void_p]
_lib.tn_contract_slices_checked.argtypes = [c_void_p, c_int64, c_int64, c_void_p, c_void_p, POINTER(c_int32)]
_lib.tn_plan_shift_outputs.argtypes = [c_void_p, c_int32, c_int32]
_lib.tn_batch_create.argtypes = [POINTER(c_void_p), c_int32, POINTER(c_int64), POINTER(c_void_p), POINTER(c_void_p)]
_lib.tn_batch_run.argtypes = [c_void_p, c_void_p]
_lib.tn_batch_destroy.argtypes = [c_void_p]
_lib.tn_contract_batch.argtypes = [POINTER(c_void_p), POINTER(c_int64), POINTER(c_void_p), c_int32, c_void_p]
_lib.tn_probe_mfma.argtypes = [c_int32, c_int64, c_void_p, POINTER(c_double), c_void_p]
_lib.tn_probe_mfma_out_floats.restype = c_int64
_lib.tn_probe_copy.argtypes = [c_void_p, c_void_p, c_int64, c_void_p]
_lib.tn_amp_frugal.argtypes = [c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_double, c_double, c_void_p,
                               c_void_p, c_void_p]
_lib.tn_amp_norm2.argtypes = [c_void_p, c_int64, c_void_p, c_void_p]
_lib.tn_amp_xeb.argtypes = [c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p]
_lib.tn_amp_hist.argtypes = [c_void_p, c_int64, c_double, c_double, c_int32, c_void_p, c_void_p]

EXPORTED = ["tn_plan_opts_default", "tn_plan", "tn_contract_slices", "tn_plan_info", "tn_plan_json",
            "tn_plan_leaf", "tn_plan_status", "tn_plan_profile", "tn_plan_set_output_bits", "tn_plan_destroy", "tn_last_error", "tn_pair_plan", "tn_pair_run",
            "tn_contract_slices_checked", "tn_plan_shift_outputs", "tn_batch_create", "tn_batch_run", "tn_batch_destroy", "tn_contract_batch",
            "tn_probe_mfma", "tn_probe_mfma_out_floats", "tn_probe_copy", "tn_permute", "tn_cgemm_c64", "tn_cgemm_c64_noalloc", "tn_cgemm_half", "tn_amp_norm2", "tn_amp_xeb", "tn_amp_frugal", "tn_amp_hist"]


def _check(rc: int):
    if rc != TN_OK:
        raise TnError(rc, _lib.tn_last_error().decode(errors="replace"))


def _i32(seq) -> ctypes.Array:
    seq = [int(x) for x in seq]
    return (c_int32 * max(1, len(seq)))(*seq)


def _ptr(t) -> int:
    """Device pointer of a torch tensor (or an int address)."""
    if isinstance(t, int):
        return t
    return int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def marshal_circuit(circuit, out_bits=None):
    """tn_circuit from an object with n_qubits and gates (qubits, matrix)."""
    gates = (tn_gate * max(1, len(circuit.gates)))()
    for i, g in enumerate(circuit.gates):
        m = np.asarray(g.matrix, dtype=np.complex128).reshape(-1)
        gates[i].nq = len(g.qubits)
        for j, q in enumerate(g.qubits):
            gates[i].q[j] = int(q)
        flat = np.empty(2 * m.size)
        flat[0::2], flat[1::2] = m.real, m.imag
        for j, v in enumerate(flat):
            gates[i].m[j] = float(v)
    n = circuit.n_qubits
    bits = np.zeros(n, dtype=np.uint8) if out_bits is None else np.asarray(out_bits, dtype=np.uint8)
    if bits.shape != (n,):
        raise ValueError("out_bits must have one entry per qubit")
    bits_c = (c_uint8 * n)(*[int(b) & 1 for b in bits])
    c = tn_circuit(n, len(circuit.gates), gates, bits_c)
    return c, (gates, bits_c)


def tn_plan_opts_default() -> tn_plan_opts:
    o = tn_plan_opts()
    _lib.tn_plan_opts_default(byref(o))
    return o


class Plan:
    """Owns a tn_plan_t (see include/tnrcs.h, tn_plan)."""

    def __init__(self, circuit, pairs: Sequence, sliced: Sequence[int] = (), open_qubits: Sequence[int] = (),
                 out_bits=None, dtype: str = "c64", gemm_form: str = "auto", dry_run: bool = False,
                 use_graph: bool = True, host_fold_log2: int = 12, device: int = 0, arena_bytes: int = 0,
                 max_log2: int = 0, tune: bool = False, tune_db: Optional[str] = None, arena=None):
        """arena: a caller-owned device workspace for the intermediates (a
        torch tensor, or an int address with arena_bytes); it must outlive
        the plan and may be shared by plans whose runs are ordered."""
        self._h = None
        c, keep = marshal_circuit(circuit, out_bits)
        flat = [int(x) for p in pairs for x in p]
        o = tn_plan_opts_default()
        o.dtype = DTYPES[dtype]
        o.gemm_form = GEMM_FORMS[gemm_form]
        o.dry_run = int(dry_run)
        o.use_graph = int(use_graph)
        o.host_fold_log2 = int(host_fold_log2)
        o.device = int(device)
        o.arena_bytes = int(arena_bytes)
        o.max_log2 = int(max_log2)
        o.tune = int(tune)
        db = tune_db.encode() if tune_db else None
        o.tune_db = db
        self._arena = arena
        if arena is not None:
            o.arena = _ptr(arena)
            if not isinstance(arena, int):
                o.arena_bytes = int(arena.numel() * arena.element_size())
        h = c_void_p()
        _check(_lib.tn_plan(byref(c), _i32(flat), len(pairs), _i32(sliced), len(sliced), _i32(open_qubits),
                            len(open_qubits), byref(o), byref(h)))
        del keep
        self._h = h
        self.n_qubits = circuit.n_qubits
        self.n_open = len(open_qubits)
        self.dry_run = bool(dry_run)

    def contract(self, s_begin: int, s_end: int, amp, stream=None):
        """tn_contract_slices: amp (device complex128, 2^n_open) += sum of slices."""
        _check(_lib.tn_contract_slices(self._h, int(s_begin), int(s_end), c_void_p(_ptr(amp)),
                                       c_void_p(_stream(stream))))

    def contract_checked(self, s_begin: int, s_end: int, amp, stream=None) -> int:
        """tn_contract_slices_checked; returns the number of re-run slices."""
        r = c_int32()
        _check(_lib.tn_contract_slices_checked(self._h, int(s_begin), int(s_end), c_void_p(_ptr(amp)),
                                               c_void_p(_stream(stream)), byref(r)))
        return int(r.value)

    def shift_outputs(self, delta: int, op: int = -1):
        """tn_plan_shift_outputs (scaled storage): kernel `op`, or all if op < 0."""
        _check(_lib.tn_plan_shift_outputs(self._h, int(op), int(delta)))

    def info(self) -> dict:
        s = tn_plan_stats()
        _check(_lib.tn_plan_info(self._h, byref(s)))
        d = {name: getattr(s, name) for name, _ in tn_plan_stats._fields_ if name != "k_hist"}
        d["k_hist"] = {i: int(v) for i, v in enumerate(s.k_hist) if v}
        return d

    def json(self) -> dict:
        need = c_int64()
        _check(_lib.tn_plan_json(self._h, None, 0, byref(need)))
        buf = ctypes.create_string_buffer(need.value)
        _check(_lib.tn_plan_json(self._h, buf, need.value, byref(need)))
        return json.loads(buf.value.decode())

    def leaf(self, i: int, n_elems: int) -> np.ndarray:
        out = (c_double * (2 * n_elems))()
        _check(_lib.tn_plan_leaf(self._h, int(i), out, 2 * n_elems))
        a = np.frombuffer(out, dtype=np.float64)
        return a[0::2] + 1j * a[1::2]

    def profile(self, slice_id: int, amp, stream=None) -> np.ndarray:
        """tn_plan_profile: per-kernel milliseconds of one slice (HIP events)."""
        n = c_int32()
        _lib.tn_plan_profile(self._h, int(slice_id), c_void_p(_ptr(amp)), c_void_p(_stream(stream)), None, 0,
                             byref(n))
        buf = (ctypes.c_float * n.value)()
        _check(_lib.tn_plan_profile(self._h, int(slice_id), c_void_p(_ptr(amp)), c_void_p(_stream(stream)), buf,
                                    n.value, byref(n)))
        return np.frombuffer(buf, dtype=np.float32).copy()

    def status(self) -> int:
        f = c_uint32()
        _check(_lib.tn_plan_status(self._h, byref(f)))
        return int(f.value)

    def set_output_bits(self, out_bits):
        bits = (c_uint8 * self.n_qubits)(*[int(b) & 1 for b in out_bits])
        _check(_lib.tn_plan_set_output_bits(self._h, bits))

    def close(self):
        if self._h is not None:
            _check(_lib.tn_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Owns a tn_batch_t that runs plans[i] over the slice range ranges[i]
    into amps[i], for all i (in list order within a lane of plans that share
    an arena workspace)."""

    def __init__(self, plans: Sequence[Plan], ranges: Sequence, amps: Sequence):
        self._h = None
        n = len(plans)
        if len(ranges) != n or len(amps) != n:
            raise ValueError("plans, ranges and amps must have the same length")
        self._plans = list(plans)      # keep the plans and buffers alive
        self._amps = list(amps)
        hp = (c_void_p * max(1, n))(*[p._h for p in plans])
        rg = (c_int64 * max(1, 2 * n))(*[int(x) for r in ranges for x in r])
        am = (c_void_p * max(1, n))(*[_ptr(a) for a in amps])
        h = c_void_p()
        _check(_lib.tn_batch_create(hp, n, rg, am, byref(h)))
        self._h = h

    def run(self, stream=None):
        _check(_lib.tn_batch_run(self._h, c_void_p(_stream(stream))))

    def close(self):
        if self._h is not None:
            _check(_lib.tn_batch_destroy(self._h))
            self._h = None

    __del__ = Plan.__del__
    __enter__ = Plan.__enter__
    __exit__ = Plan.__exit__


def tn_contract_batch(plans: Sequence[Plan], ranges: Sequence, amps: Sequence, stream=None):
    """One-shot batch: create, run, wait, release."""
    n = len(plans)
    hp = (c_void_p * max(1, n))(*[p._h for p in plans])
    rg = (c_int64 * max(1, 2 * n))(*[int(x) for r in ranges for x in r])
    am = (c_void_p * max(1, n))(*[_ptr(a) for a in amps])
    _check(_lib.tn_contract_batch(hp, rg, am, n, c_void_p(_stream(stream))))


class PairPlan:
    """Owns a pairwise-contraction plan (tn_pair_plan / tn_pair_run)."""

    def __init__(self, labels_a, labels_b, labels_c, dtype: str = "c64", gemm_form: str = "auto",
                 dry_run: bool = False, device: int = 0):
        self._h = None
        o = tn_plan_opts_default()
        o.dtype = DTYPES[dtype]
        o.gemm_form = GEMM_FORMS[gemm_form]
        o.dry_run = int(dry_run)
        o.device = int(device)
        h = c_void_p()
        _check(_lib.tn_pair_plan(len(labels_a), _i32(labels_a), len(labels_b), _i32(labels_b), len(labels_c),
                                 _i32(labels_c), byref(o), byref(h)))
        self._h = h

    def run(self, A, B, C, batch: int = 1, out_scale: float = 1.0, stream=None):
        _check(_lib.tn_pair_run(self._h, c_void_p(_ptr(A)), c_void_p(_ptr(B)), c_void_p(_ptr(C)), int(batch),
                                float(out_scale), c_void_p(_stream(stream))))

    info = Plan.info
    json = Plan.json
    close = Plan.close
    __del__ = Plan.__del__


def tn_pair_plan(labels_a, labels_b, labels_c, **kw) -> PairPlan:
    return PairPlan(labels_a, labels_b, labels_c, **kw)


def tn_pair_run(pp: PairPlan, A, B, C, batch: int = 1, out_scale: float = 1.0, stream=None):
    pp.run(A, B, C, batch, out_scale, stream)


def tn_plan(circuit, pairs, sliced=(), open_qubits=(), out_bits=None, **kw) -> Plan:
    return Plan(circuit, pairs, sliced, open_qubits, out_bits, **kw)


def tn_contract_slices(plan: Plan, s_begin: int, s_end: int, amp, stream=None):
    plan.contract(s_begin, s_end, amp, stream)


def tn_plan_info(plan: Plan) -> dict:
    return plan.info()


def tn_plan_status(plan: Plan) -> int:
    return plan.status()


def tn_plan_destroy(plan: Plan):
    plan.close()


def tn_last_error() -> str:
    return _lib.tn_last_error().decode(errors="replace")


def tn_permute(inp, out, perm: Sequence[int], batch: int = 1, elem_bytes: int = 8, stream=None):
    _check(_lib.tn_permute(c_void_p(_ptr(inp)), c_void_p(_ptr(out)), int(elem_bytes), len(perm), _i32(perm),
                           int(batch), c_void_p(_stream(stream))))


def tn_cgemm_c64(A, B, C, M: int, N: int, K: int, batch: int = 1, form: str = "4m", work=None, splits: int = 1,
                 stream=None):
    _check(_lib.tn_cgemm_c64(c_void_p(_ptr(A)), c_void_p(_ptr(B)), c_void_p(_ptr(C)), int(M), int(N), int(K),
                             int(batch), GEMM_FORMS[form], c_void_p(_ptr(work) if work is not None else None),
                             int(splits), c_void_p(_stream(stream))))


def tn_cgemm_c64_noalloc(A, B, C, M: int, N: int, K: int, form: str = "4m", splits: int = 1, stream=None):
    _check(_lib.tn_cgemm_c64_noalloc(c_void_p(_ptr(A)), c_void_p(_ptr(B)), c_void_p(_ptr(C)), int(M), int(N), int(K),
                                     GEMM_FORMS[form], int(splits), c_void_p(_stream(stream))))


def tn_cgemm_half(dtype: str, A, B, C, M: int, N: int, K: int, batch: int = 1, form: str = "4m",
                  out_scale: float = 1.0, work=None, splits: int = 1, max_out=None, stream=None):
    _check(_lib.tn_cgemm_half(DTYPES[dtype], c_void_p(_ptr(A)), c_void_p(_ptr(B)), c_void_p(_ptr(C)), int(M), int(N),
                              int(K), int(batch), GEMM_FORMS[form], float(out_scale),
                              c_void_p(_ptr(work) if work is not None else None), int(splits),
                              c_void_p(_ptr(max_out) if max_out is not None else None), c_void_p(_stream(stream))))


def tn_amp_norm2(amp, n: int, out, stream=None):
    _check(_lib.tn_amp_norm2(c_void_p(_ptr(amp)), int(n), c_void_p(_ptr(out)), c_void_p(_stream(stream))))


def tn_amp_xeb(amp, n: int, idx, n_idx: int, out, stream=None):
    _check(_lib.tn_amp_xeb(c_void_p(_ptr(amp)), int(n), c_void_p(_ptr(idx)), int(n_idx), c_void_p(_ptr(out)),
                           c_void_p(_stream(stream))))


def tn_amp_hist(amp, n: int, scale: float, xmax: float, n_bins: int, counts, stream=None):
    _check(_lib.tn_amp_hist(c_void_p(_ptr(amp)), int(n), float(scale), float(xmax), int(n_bins),
                            c_void_p(_ptr(counts)), c_void_p(_stream(stream))))


def tn_probe_mfma(kind: str, iters: int, out, stream=None) -> float:
    """MFMA issue loop ('f32', 'f16' or 'bf16'); returns the flops issued."""
    fl = c_double()
    _check(_lib.tn_probe_mfma({"f32": 0, "f16": 1, "bf16": 2}[kind], int(iters), c_void_p(_ptr(out)), byref(fl),
                              c_void_p(_stream(stream))))
    return fl.value


def tn_probe_mfma_out_floats() -> int:
    return int(_lib.tn_probe_mfma_out_floats())


def tn_probe_copy(src, dst, nbytes: int, stream=None):
    _check(_lib.tn_probe_copy(c_void_p(_ptr(src)), c_void_p(_ptr(dst)), int(nbytes), c_void_p(_stream(stream))))


def tn_amp_frugal(amp, n: int, idx, n_cand: int, u, scale: float, m: float, out_idx, count, stream=None):
    """Frugal rejection sampling (see include/tnrcs.h); idx may be None."""
    _check(_lib.tn_amp_frugal(c_void_p(_ptr(amp)), int(n), None if idx is None else c_void_p(_ptr(idx)),
                              int(n_cand), c_void_p(_ptr(u)), float(scale), float(m), c_void_p(_ptr(out_idx)),
                              c_void_p(_ptr(count)), c_void_p(_stream(stream))))
