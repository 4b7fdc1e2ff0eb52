"""Writes the oracle's outputs of the large random-layer + QFT workload (config 3) at its
full complex128 size, 31 qubits, into ``config3_31q_oracle.txt`` beside this script.

The values come from the FP64 CPU oracle only (``oracle.apply`` gate by gate, App. A's plain
state-vector method) on the seeded gate list of ``workloads.config3(31)``: 100 layers of U3 on
every qubit plus a low/high CX matching, then the exact QFT (App. D.2).  The file holds the
amplitude at each of the 1024 seeded basis states of ``workloads.config3_indices(31)`` (their
probabilities follow), <Z_0 Z_30> and the norm sum_i |alpha_i|^2.

The oracle needs a 32 GiB complex128 state and about 1.1e13 amplitude updates (roughly 1.5 h
on 8 cores), so the GPU test reads this file instead of re-running it.

    python tests/golden/make_config3_golden.py [n_qubits]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2504_03967_amd import workloads as W  # noqa: E402


def main(n: int = 31) -> str:
    circ = W.config3(n)
    psi = oracle.zero_state(n)
    chunk = 4 * (n + n // 2)  # four layers per call, so that progress can be reported
    t0 = time.time()
    for g0 in range(0, circ.n_gates, chunk):
        g1 = min(circ.n_gates, g0 + chunk)
        part = W.Circuit(n, circ.gate_type[g0:g1], circ.gate_param[g0:g1], circ.param_idx[g0:g1])
        oracle.apply(part, psi)
        print(f"gates {g1}/{circ.n_gates}  {time.time() - t0:.0f} s", flush=True)
    idx = W.config3_indices(n)
    amp = psi[idx.astype(np.int64)]
    norm, zz = oracle.expval(psi, np.array([0, 1 | (1 << (n - 1))], dtype=np.uint64))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"config3_{n}q_oracle.txt")
    with open(out, "w") as f:
        f.write(f"# FP64 oracle, config 3 at {n} qubits: {circ.n_gates} gates (100 layers + QFT({n})),\n")
        f.write("# written by tests/golden/make_config3_golden.py (oracle only).\n")
        f.write(f"norm {float(norm)!r}\n")
        f.write(f"zz_0_{n - 1} {float(zz)!r}\n")
        f.write("# index re im\n")
        for i, a in zip(idx, amp):
            f.write(f"{int(i)} {float(a.real)!r} {float(a.imag)!r}\n")
    print(f"wrote {out} in {time.time() - t0:.0f} s")
    return out


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 31)
