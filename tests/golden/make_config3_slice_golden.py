"""Writes tests/golden/config3_slices.txt: the 64 amplitudes of two slices
of the 53-qubit, 14-cycle benchmark network (slice 0 and one seeded slice of
its frozen order), computed by the FP64 oracle alone.

A slice of the benchmark plan has intermediates of up to 2^32 entries, too
large for host memory in FP64, so each slice is computed as the sum of its
sub-slices: more wires are sliced (the input-side greedy slicer, seeded
only by the order) until every tensor has at most 2^SUB_LOG2 entries, and
the oracle's pairwise FP64 contraction of every sub-slice is summed.  That
sum equals the slice exactly up to rounding, because a sliced network is the
sum of its slices (main text, customized-TNC section).  Only oracle/
computes values; rqcgen/ supplies the circuit, order and sliced wires.

  python tests/golden/make_config3_slice_golden.py [--sub-log2 29] [--slices 2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.tn import contract_network, slice_assignment  # noqa: E402
from rqcgen import network_structure, slice_to_fit  # noqa: E402
from rqcgen.workloads import config3  # noqa: E402

OUT = os.path.join(HERE, "config3_slices.txt")
SEEDED_SLICE_RNG = 11


def order_digest(pairs, sliced) -> str:
    """Identity of a (pairs, sliced) order: the fixture holds for this order only."""
    blob = json.dumps([[list(map(int, p)) for p in pairs], [int(w) for w in sliced]]).encode()
    return hashlib.sha256(blob).hexdigest()[:16]


def seeded_slice(k: int) -> int:
    return int(np.random.default_rng(SEEDED_SLICE_RNG).integers(1, 1 << k))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sub-log2", type=int, default=29)
    ap.add_argument("--slices", type=int, default=2, help="slice 0, then the seeded slice")
    a = ap.parse_args()
    w = config3()
    ns = network_structure(w.circuit, w.open_qubits)
    k = len(w.sliced)
    allsl = slice_to_fit(ns, w.pairs, a.sub_log2, initial=w.sliced)
    extra = allsl[k:]
    leaves, ow = oracle.build_network(w.circuit, w.open_qubits, w.out_bits)
    slices = [0, seeded_slice(k)][: a.slices]
    results = []
    for s in slices:
        t0 = time.perf_counter()
        total = None
        for e in range(1 << len(extra)):
            v = contract_network(leaves, w.pairs, ow, slice_assignment(allsl, s | (e << k)))
            total = v if total is None else total + v
            print(f"slice {s}: sub-slice {e + 1}/{1 << len(extra)} done ({time.perf_counter() - t0:.0f} s)",
                  file=sys.stderr, flush=True)
        results.append(total)
        # the file is rewritten after every slice, so a finished slice is kept
        with open(OUT, "w") as f:
            f.write("# 53-qubit 14-cycle network (6x9 grid, one missing site, seed 3), qubits 47-52 open\n")
            f.write("# FP64 oracle: each slice as the sum of its sub-slices "
                    "(tests/golden/make_config3_slice_golden.py)\n")
            f.write(f"order_digest {order_digest(w.pairs, w.sliced)}\n")
            f.write(f"sliced {' '.join(map(str, w.sliced))}\n")
            f.write(f"sub_sliced {' '.join(map(str, extra))} sub_log2 {a.sub_log2}\n")
            for sl, amp in zip(slices, results):
                f.write(f"slice {sl}\n")
                for z in amp:
                    f.write(f"{z.real:.17e} {z.imag:.17e}\n")
        print(f"wrote {OUT} ({len(results)} slice(s))", file=sys.stderr, flush=True)


def load():
    """(digest, {slice: amplitudes}) from the fixture file."""
    amps, cur, digest = {}, None, None
    with open(OUT) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tok = line.split()
            if tok[0] == "order_digest":
                digest = tok[1]
            elif tok[0] == "slice":
                cur = int(tok[1])
                amps[cur] = []
            elif tok[0] in ("sliced", "sub_sliced"):
                continue
            else:
                amps[cur].append(complex(float(tok[0]), float(tok[1])))
    return digest, {s: np.array(v, dtype=np.complex128) for s, v in amps.items()}


if __name__ == "__main__":
    main()
