"""Benchmark of the state-vector hot path on one MI355X.

One step = the 30-qubit complex128 gate sweep on a 16 GiB state (U3 on every
target qubit, CX / CP / SWAP on low, mixed and high qubit pairs, then groups of
2..6 U3 gates fused into one pass) followed by the reductions of the method:
probabilities of 1024 basis states, 10,000 seeded shots and the 29
Z_i Z_{i+1} expectations.  Inputs are synthetic and seeded; the state is
resident in HBM before the timed region starts.

Prints one JSON line: amplitude updates per second (2^n per gate, the paper's
O(2^n d) cost model of App. A), the roofline of the dominant kernel (the tile
pass of a single U3, measured with HIP events on the stream it runs on), and
the FP64 oracle timed on the host cores on a bounded sample of the same gates.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--skip-cpu", action="store_true", help="omit the oracle CPU baseline")
    ap.add_argument("--cpu-gates", type=int, default=8, help="sweep gates the oracle sample applies")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 4 GiB device copy (reference kernel for HBM byte counters)")
    ap.add_argument("--parts-json", default="", help="write per-part timings to this file")
    return ap.parse_args()


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_2504_03967_amd import qg
    from paper_2504_03967_amd import workloads as W

    torch.cuda.set_device(0)
    n = args.n
    amp_bytes = 16 if args.dtype == "c128" else 8
    prep, full, parts = W.sweep(n)
    st = qg.State(n, args.dtype)
    st.apply(prep, qg.FUSE_NONE)
    masks = W.zz_chain_masks(n)
    idx = W.config3_indices(n, count=1024)
    stream = torch.cuda.current_stream()

    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.complex128, device="cuda")  # 4 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def modes(name):
        return qg.FUSE_GREEDY if name.startswith("fused") else qg.FUSE_NONE

    events = []

    def step(record: bool):
        for name, circ in parts:
            if record:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
            st.apply(circ, modes(name))
            if record:
                e1.record(stream)
                events.append((name, e0, e1))
        st.probs(idx)
        st.sample(10000, W.SEED_BASE)
        st.expval(masks, np.ones(masks.size))

    log(f"state ready: {n} qubits {args.dtype}")
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log("warmup done")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {elapsed:.3f} s")

    gates_per_step = full.n_gates
    amp_updates = gates_per_step * (1 << n) * args.steps
    value = amp_updates / elapsed

    per = {}
    for name, e0, e1 in events:
        per.setdefault(name, []).append(e0.elapsed_time(e1) * 1e-3)
    pass_bytes = 2 * (1 << n) * amp_bytes
    u3 = np.array([np.mean(per[f"u3_t{t}"]) for t in range(n)])
    u3_gbs = pass_bytes / u3 / 1e9
    achieved = pass_bytes / float(np.mean(u3)) / 1e9

    def part_gbs(name, frac):
        return round(frac * pass_bytes / float(np.mean(per[name])) / 1e9, 1)

    sweep = {"u3_GBps_min": round(float(u3_gbs.min()), 1),
             "u3_GBps_geomean": round(float(np.exp(np.mean(np.log(u3_gbs)))), 1),
             "u3_GBps_max": round(float(u3_gbs.max()), 1)}
    # Bytes each part's pass moves: a single-gate tile holds the target and the
    # lowest 11 other qubits (12 tile qubits); controls and diagonal qubits outside
    # the tile restrict the pass to the tiles where their bits are 1.
    tile_bits = 12 if args.dtype == "c128" else 13
    for name, _ in parts:
        if name.startswith(("cx", "cp", "swap")):
            a, b = (int(v) for v in name.split("_")[1:])
            if name.startswith("cx"):
                frac = 0.5 if a >= tile_bits - 1 else 1.0
            elif name.startswith("cp"):
                frac = 0.5 ** ((a >= tile_bits) + (b >= tile_bits))
            else:
                frac = 1.0
            sweep[name + "_GBps"] = part_gbs(name, frac)
        elif name.startswith("fused"):
            sweep[name + "_GBps"] = part_gbs(name, 1.0)
    if args.parts_json:
        with open(args.parts_json, "w") as f:
            json.dump({k: float(np.mean(v)) for k, v in per.items()}, f, indent=1)

    st.close()
    del st
    torch.cuda.empty_cache()

    cpu = None
    if not args.skip_cpu:
        import oracle
        threads = oracle.num_threads()
        n_cpu = args.cpu_gates
        sample = W.concat(parts[0][1], parts[1][1])
        for name, c in parts[2:n_cpu]:
            sample = W.concat(sample, c)
        psi = oracle.zero_state(n)
        t1 = time.perf_counter()
        oracle.apply(sample, psi)
        dt = time.perf_counter() - t1
        log(f"oracle sample: {sample.n_gates} gates in {dt:.1f} s on {threads} threads")
        del psi
        cpu = {"value": sample.n_gates * (1 << n) / dt, "unit": "amp-updates/s", "cores": threads,
               "kind": "oracle",
               "sample": f"first {sample.n_gates} gates of the {n}-qubit sweep (U3 on targets 0..{sample.n_gates - 1}) "
                         f"on a 2^{n} complex128 state, {dt:.1f} s"}

    out = {
        "metric": "amp-updates/s (30q c128 gate sweep)",
        "value": value,
        "unit": "amp-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.dtype == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": f"gate sweep, {n} qubits {args.dtype}: U3 x{n} targets, CX/CP/SWAP x5 pairs, "
                               f"fused U3 groups k=2..6, then probs(1024), 10^4 shots, {n - 1} ZZ expvals",
                   "n_qubits": n, "gates_per_step": gates_per_step, "state_GiB": (1 << n) * amp_bytes / 2 ** 30},
        "hbm_frac": achieved / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_tile_inl (single-U3 pass)", "bytes_per_launch": pass_bytes},
        "sweep": sweep,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
