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
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of the tile pass measured with rocprofv3 FETCH_SIZE / WRITE_SIZE on this
# benchmark (profiles/tile_pass_sweep30_c128.md), valid only for the kernel and planner
# sources it was taken with (sha256 prefix of KERNEL_SOURCES); otherwise null.
KERNEL_SOURCES = ("paper_2504_03967_amd/csrc/qg_tile_dev.h", "paper_2504_03967_amd/csrc/qg_tile.hip",
                  "paper_2504_03967_amd/csrc/qg_plan.cpp", "paper_2504_03967_amd/csrc/qg_internal.h",
                  "paper_2504_03967_amd/csrc/qg_api.cpp")
MEASURED_TRAFFIC = {"sources": "066cae024e0531af", "traffic_over_algorithmic": 1.00062}


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--skip-cpu", action="store_true", help="omit the oracle CPU baseline")
    ap.add_argument("--cpu-gates", type=int, default=40, help="sweep parts the oracle sample applies")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 4 GiB device copy (reference kernel for HBM byte counters)")
    ap.add_argument("--parts-json", default="", help="write per-part timings to this file")
    ap.add_argument("--no-extras", action="store_true",
                    help="omit the adjoint / batched speed-ups and the learned-fusion gain")
    ap.add_argument("--cm-samples", type=int, default=1500, help="timed passes for the cost-model dataset")
    ap.add_argument("--config3-only", type=int, default=0, metavar="N",
                    help="only time config 3 on N qubits (c128) and print its JSON line (profiling)")
    return ap.parse_args()


def timed(fn, sync):
    sync()
    t0 = time.perf_counter()
    r = fn()
    sync()
    return time.perf_counter() - t0, r


FP64_PEAK_TFLOPS = 78.6  # MI355X vector (and matrix) FP64


def algorithmic_flops_per_index(circ, W) -> float:
    """Floating-point operations per amplitude index of a circuit, counting what the gate
    requires (a fused multiply-add is 2): a general 2x2 complex gate 14 per amplitude (two
    complex products and a complex sum), a real or RX-form matrix 6 (two real-by-complex
    products and a sum), RZ 6 (one complex product), CP / CZ 1.5 (one complex product on a
    quarter of the amplitudes), CX / SWAP / X 0 (data movement only)."""
    ops = circ.gate_type[:, 0]
    per = {W.U3: 14.0, W.H: 6.0, W.RY: 6.0, W.RX: 6.0, W.RZ: 6.0, W.CP: 1.5, W.CZ: 1.5}
    return float(sum(per.get(int(o), 0.0) for o in ops))


def config3_timing(qg, W, torch, n: int = 31):
    """The paper-shaped large circuit: 100 random U3 + CX layers and a QFT on n qubits
    (complex128; 32 GiB at 31 qubits), greedy (commutation-aware) fusion.  Its fused passes
    hold ~20 gates each, so they are bound by FP64 issue and register-layout exchanges
    rather than HBM: both rooflines are reported."""
    circ = W.config3(n)
    st = qg.State(n, "c128")
    _, npass = qg.plan_passes(circ, "c128", qg.FUSE_GREEDY)
    st.apply(circ, qg.FUSE_GREEDY)  # warm-up (plans, code)
    st.reset()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    st.apply(circ, qg.FUSE_GREEDY)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3
    st.close()
    torch.cuda.empty_cache()
    flops = algorithmic_flops_per_index(circ, W) * (1 << n)
    hbm = npass * 2 * (1 << n) * 16
    return {"workload": f"{n} qubits c128: 100 layers (U3 on every qubit, {n // 2} low/high CX) + QFT({n}), "
                        f"{circ.n_gates} gates",
            "passes": npass, "t_s": round(t, 3), "amp_updates_per_s": circ.n_gates * (1 << n) / t,
            "fp64_TFLOPs": round(flops / t / 1e12, 2),
            "fp64_frac": round(flops / t / 1e12 / FP64_PEAK_TFLOPS, 4),
            "full_pass_equivalent_GBps": round(hbm / t / 1e9, 1),
            "hbm_frac": round(hbm / t / 1e9 / HBM_PEAK_GBS, 4)}


def paper_shaped(qg, W, torch, n: int = 30):
    """The paper's other benchmark circuit shapes at n qubits (complex128, greedy fusion):
    QFT(n), and random CX-block unitaries of 100 ('short') and 1000 blocks."""
    st = qg.State(n, "c128")
    out = {}
    for name, circ in (("qft", W.qft(n).build()), ("cx_blocks_100", W.cx_blocks(n, 100, W.SEED_BASE + 7)),
                       ("cx_blocks_1000", W.cx_blocks(n, 1000, W.SEED_BASE + 8))):
        _, npass = qg.plan_passes(circ, "c128", qg.FUSE_GREEDY)
        st.apply(circ, qg.FUSE_GREEDY)  # warm-up
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st.apply(circ, qg.FUSE_GREEDY)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3
        out[name] = {"gates": circ.n_gates, "passes": npass, "t_ms": round(t * 1e3, 2),
                     "amp_updates_per_s": circ.n_gates * (1 << n) / t}
    st.close()
    torch.cuda.empty_cache()
    return {"n_qubits": n, **out}


def large_shots(qg, W, torch, shots: int = 3000 << 15):
    """Shot sampling at the paper's large shot counts (3000 * 2^m shots, m = 15): seeded
    samples of a random product state at 15, 20 and 25 qubits (complex128), one call each."""
    out = {"shots": shots}
    for n in (15, 20, 25):
        st = qg.State(n, "c128")
        b = W.CircuitBuilder(n)
        rng = W.SplitMix64(W.SEED_BASE + 40 + n)
        for q in range(n):
            b.g1(W.U3, q, *(2 * math.pi * rng.uniform(3)))
        st.apply(b.build(), qg.FUSE_GREEDY)
        st.sample(1000, 1)
        ts = []
        for r in range(3):
            t, idx = timed(lambda: st.sample(shots, W.SEED_BASE + r), torch.cuda.synchronize)
            del idx
            ts.append(t)
        t = float(np.median(ts))
        out[f"n{n}"] = {"t_ms": round(t * 1e3, 2), "shots_per_s": shots / t}
        st.close()
        torch.cuda.empty_cache()
    return out


def precision_gap(qg, W, torch, n: int = 26):
    """complex64 against complex128 on config 3's circuit shape (n qubits, 20 layers + QFT):
    largest amplitude difference and the fidelity |<psi64|psi128>|^2, on the host."""
    circ = W.config3(n, layers=20)
    res = {}
    for dt in ("c128", "c64"):
        st = qg.State(n, dt)
        st.apply(circ, qg.FUSE_GREEDY)
        torch.cuda.synchronize()
        res[dt] = st.tensor.cpu().numpy().astype(np.complex128)
        st.close()
    torch.cuda.empty_cache()
    a, b = res["c128"], res["c64"]
    return {"workload": f"config 3 shape, {n} qubits, 20 layers + QFT({n}), {circ.n_gates} gates",
            "max_abs_diff": float(np.max(np.abs(a - b))), "max_abs_amplitude": float(np.max(np.abs(a))),
            "fidelity_c64": float(abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real))}


def adjoint_speedup(qg, W, torch):
    """Config 5: gradient of sum <Z_i Z_i+1> (24 qubits, 480 parameters) by one adjoint sweep
    vs the plain method, central differences (960 forward simulations + expectations)."""
    circ = W.config5()
    n, npar = circ.n_qubits, circ.n_params
    masks = W.zz_chain_masks(n)
    coeffs = np.ones(n - 1)
    qg.adjoint_grad(circ, masks, coeffs, npar)  # warm
    t_adj, _ = timed(lambda: qg.adjoint_grad(circ, masks, coeffs, npar), torch.cuda.synchronize)
    st = qg.State(n, "c128")
    h = 1e-6
    shifted = []
    for k in range(npar):
        (g,) = np.nonzero(circ.param_idx == k)
        for sgn in (1, -1):
            c = circ.copy()
            c.gate_param[g, 0] += sgn * h
            shifted.append(c)

    def plain():
        vals = []
        for c in shifted:
            st.reset()
            st.apply(c, qg.FUSE_GREEDY)
            vals.append(st.expval(masks, coeffs)[1])
        return vals

    st.apply(circ, qg.FUSE_GREEDY)
    t_fd, _ = timed(plain, torch.cuda.synchronize)
    st.close()
    return {"workload": "24 qubits c128, 10-layer ansatz, 480 parameters, 710 gates",
            "t_adjoint_s": round(t_adj, 4), "t_plain_fd_s": round(t_fd, 3),
            "plain": "central differences, 960 greedy-fused forward passes + expval",
            "speedup": round(t_fd / t_adj, 1)}


def batched_speedup(qg, W, torch):
    """Config 4: 4096 ansatz circuits (8..20 qubits) in one graph-replayed persistent launch
    vs the plain loop (per circuit: reset, apply with one pass per gate, expval)."""
    circs = W.config4()
    stream = torch.cuda.Stream()
    out = {"workload": "4096 ansatz circuits, 8..20 qubits, 2..12 layers, sum Z_i Z_i+1 each"}
    amp_updates = float(sum(c.n_gates * (1 << c.n_qubits) for c in circs))
    with torch.cuda.stream(stream):
        for dtype in ("c128", "c64"):
            b = qg.Batch(circs, dtype, stream=stream)
            b.launch()
            t_b, _ = timed(b.launch, stream.synchronize)
            b.close()
            out[f"t_batched_{dtype}_s"] = round(t_b, 4)
            out[f"amp_updates_per_s_batched_{dtype}"] = amp_updates / t_b
        states = {}
        for n in sorted({c.n_qubits for c in circs}):
            states[n] = qg.State(n, "c128", stream=stream)
        zz = {n: W.zz_chain_masks(n) for n in states}

        def plain():
            for c in circs:
                st = states[c.n_qubits]
                st.reset()
                st.apply(c, qg.FUSE_NONE)
                st.expval(zz[c.n_qubits], np.ones(c.n_qubits - 1))

        t_p, _ = timed(plain, stream.synchronize)
        for st in states.values():
            st.close()
    out["t_plain_loop_c128_s"] = round(t_p, 3)
    out["plain"] = "per-circuit qg_apply_circuit (one pass per gate) + qg_expval, c128"
    out["speedup_c128"] = round(t_p / out["t_batched_c128_s"], 1)
    return out


def learned_gain(qg, W, torch, samples, log):
    """Cost model trained on pass timings the simulator makes (library MLP kernels), then
    measured time of greedy width-5 plans vs learned plans on held-out circuits."""
    from paper_2504_03967_amd import costmodel as cm
    t0 = time.perf_counter()
    X, y = cm.collect(samples, n_values=(20, 22, 24, 26, 28), log=log)
    t_collect = time.perf_counter() - t0
    n_train = int(0.85 * len(y))
    t1 = time.perf_counter()
    model, losses = cm.train(X[:n_train], y[:n_train], epochs=300, batch=128, lr=2e-3)
    t_train = time.perf_counter() - t1
    err = cm.mape(model, X[n_train:], y[n_train:])
    model.install()
    circs = cm.held_out_circuits(count=20)
    res = cm.compare_plans(circs)
    qg.clear_cost_model()
    model.close()
    return {"samples": int(len(y)), "t_collect_s": round(t_collect, 1), "t_train_s": round(t_train, 2),
            "train_loss_first_last": [round(float(losses[0]), 4), round(float(losses[-1]), 4)],
            "heldout_mape": round(err, 3), "circuits": len(circs),
            "t_greedy5_s": round(res["t_greedy_s"], 4), "t_learned_s": round(res["t_learned_s"], 4),
            "gain": round(res["gain"], 3)}


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
    if args.config3_only:
        print(json.dumps({"config3": config3_timing(qg, W, torch, args.config3_only)}), flush=True)
        return
    n = args.n
    amp_bytes = 16 if args.dtype == "c128" else 8
    from paper_2504_03967_amd import autotune
    table, source = autotune.tuned(n, args.dtype)
    log(f"autotuned tile shapes ({source}): {table}")
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
    line_bits = 3 if args.dtype == "c128" else 4   # amplitudes per 128-byte line = 2^line_bits

    def algo_frac(name):
        """Algorithmic bytes of a part as a fraction of a full pass: the 128-byte lines that
        hold an amplitude the gate changes, read and written once."""
        if not name.startswith(("cx", "cp", "swap")):
            return 1.0
        a, b = (int(v) for v in name.split("_")[1:])
        if name.startswith("cx"):
            return 0.5 if a >= line_bits else 1.0
        if name.startswith("cp"):
            return 0.5 ** ((a >= line_bits) + (b >= line_bits))
        return 0.5 if min(a, b) >= line_bits else 1.0

    u3 = np.array([np.mean(per[f"u3_t{t}"]) for t in range(n)])
    u3_gbs = pass_bytes / u3 / 1e9
    sweep = {"u3_GBps_min": round(float(u3_gbs.min()), 1),
             "u3_GBps_geomean": round(float(np.exp(np.mean(np.log(u3_gbs)))), 1),
             "u3_GBps_max": round(float(u3_gbs.max()), 1)}
    for name, _ in parts:
        if not name.startswith("u3"):
            sweep[name + "_GBps"] = round(algo_frac(name) * pass_bytes / float(np.mean(per[name])) / 1e9, 1)
    # Dominant kernel: the tile pass.  The planner sends standalone SWAPs to the permutation
    # kernels and single gates with their target inside a cache line to the lane kernel; those
    # parts stay out of the tile-pass figure.
    kernels_of = {nm: qg.plan_kernels(c, args.dtype, modes(nm)) for nm, c in parts}
    tile_parts = [nm for nm, _ in parts if set(kernels_of[nm]) == {"tile"}]
    tile_bytes = sum(algo_frac(nm) * pass_bytes for nm in tile_parts)
    tile_time = sum(float(np.mean(per[nm])) for nm in tile_parts)
    achieved = tile_bytes / tile_time / 1e9
    bytes_per_launch = tile_bytes / len(tile_parts)
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
               "kind": "oracle", "nproc": len(os.sched_getaffinity(0)), "cpu_model": cpu_model(),
               "sample": f"first {sample.n_gates} gates of the {n}-qubit sweep on a 2^{n} complex128 state "
                         f"(one FP64 pass per gate), {dt:.1f} s"}

    traffic = None
    if MEASURED_TRAFFIC["traffic_over_algorithmic"] and MEASURED_TRAFFIC["sources"] == kernel_sources_hash():
        traffic = round(MEASURED_TRAFFIC["traffic_over_algorithmic"] * bytes_per_launch)

    extras = {}
    if not args.no_extras:
        log("config 3 (31 qubits c128, 5111 gates) timing")
        extras["config3"] = config3_timing(qg, W, torch)
        log("QFT and random CX-block unitaries (30 qubits c128)")
        extras["paper_shaped"] = paper_shaped(qg, W, torch)
        log("large shot counts; complex64 vs complex128")
        extras["large_shots"] = large_shots(qg, W, torch)
        extras["precision"] = precision_gap(qg, W, torch)
        log("adjoint vs finite differences (config 5)")
        extras["adjoint"] = adjoint_speedup(qg, W, torch)
        log(f"adjoint speedup {extras['adjoint']['speedup']}x; batched vs plain loop (config 4)")
        extras["batched"] = batched_speedup(qg, W, torch)
        log(f"batched speedup {extras['batched']['speedup_c128']}x; learned fusion")
        extras["learned_fusion"] = learned_gain(qg, W, torch, args.cm_samples, log)
        log(f"learned fusion gain {extras['learned_fusion']['gain']}")

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
        "hbm_frac": round(achieved / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_tile_inl (tile pass)", "launches_per_step": len(tile_parts),
                     "other_parts": {k: sorted(set(v)) for k, v in kernels_of.items() if set(v) != {"tile"}},
                     "algorithmic_bytes_per_launch": round(bytes_per_launch),
                     "avg_launch_ms": round(tile_time / len(tile_parts) * 1e3, 4)},
        "sweep": sweep,
        "autotune": {"source": source, "classes": "target <3 | <12 | <20 | >=20 | diagonal",
                     "tile_reg_swz": table,
                     "per_target_tile_reg_swz_xcd": autotune.current_targets(args.dtype)[:n]},
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
