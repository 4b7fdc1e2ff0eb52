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
MEASURED_TRAFFIC = {"sources": "50e30ebc0950c6b7", "traffic_over_algorithmic": 1.00077}


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
    ap.add_argument("--form-only", choices=["adjoint", "batched"], default="",
                    help="only run the adjoint gradient (24 qubits) or the batched launch (4096 circuits) "
                         "twice, for profiling")
    ap.add_argument("--paper-workloads", action="store_true",
                    help="only run the paper's short and long CX-block unitaries at 28-34 qubits (minutes)")
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
    # the same circuit through qg_apply_from_zero (reset included): passes skip the tiles
    # that are still zero
    t0 = event_time(stream, torch, lambda: st.apply_from_zero(circ, qg.FUSE_GREEDY))
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
            "hbm_frac": round(hbm / t / 1e9 / HBM_PEAK_GBS, 4),
            "t_from_zero_s": round(t0, 3)}


def paper_shaped(qg, W, torch, n: int = 30):
    """The QFT at n qubits (complex128, greedy fusion)."""
    st = qg.State(n, "c128")
    out = {}
    for name, circ in (("qft", W.qft(n).build()),):
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
        st.apply_from_zero(circ, qg.FUSE_GREEDY)
        t0 = event_time(stream, torch, lambda: st.apply_from_zero(circ, qg.FUSE_GREEDY))
        out[name] = {"gates": circ.n_gates, "passes": npass, "t_ms": round(t * 1e3, 2),
                     "amp_updates_per_s": circ.n_gates * (1 << n) / t,
                     "t_from_zero_ms": round(t0 * 1e3, 2)}
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


def event_time(stream, torch, fn) -> float:
    """Seconds between HIP events recorded around fn() on `stream`."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3


TABLE2 = [(10, 5), (11, 8), (12, 6), (13, 12), (14, 6), (15, 3)]  # (address, data) qubits


def qcrank_table2(qg, W, torch):
    """QCrank image encoding at Table 2's shapes (m address + d data qubits, 2^m d pixels =
    CX gates, 3000 * 2^m shots; synthetic pixels): the encoding circuit and the shot draw
    timed separately, complex128, greedy fusion."""
    stream = torch.cuda.current_stream()
    out = {}
    for m, nd in TABLE2:
        circ, _ = W.config2(seed=W.SEED_BASE + 20 + m, n_addr=m, n_data=nd)
        n = m + nd
        st = qg.State(n, "c128")
        st.apply(circ, qg.FUSE_GREEDY)  # warm-up
        st.reset()
        t_apply = event_time(stream, torch, lambda: st.apply(circ, qg.FUSE_GREEDY))
        shots = 3000 << m
        st.sample(1000, 1)
        t_shots = min(event_time(stream, torch, lambda: st.sample(shots, W.SEED_BASE + r)) for r in range(2))
        _, npass = qg.plan_passes(circ, "c128", qg.FUSE_GREEDY)
        out[f"m{m}_d{nd}"] = {"qubits": n, "pixels": nd << m, "gates": circ.n_gates, "passes": npass,
                              "t_apply_ms": round(t_apply * 1e3, 3),
                              "amp_updates_per_s": circ.n_gates * (1 << n) / t_apply,
                              "shots": shots, "t_shots_ms": round(t_shots * 1e3, 3), "shots_per_s": shots / t_shots}
        st.close()
        torch.cuda.empty_cache()
    return out


def qft_study(qg, W, torch):
    """The QFT's precision and approximation (Table 1's QFT row, App. D.2's rotation-angle
    approximation): after a random U3 layer, the exact QFT and versions with every CP of
    angle below eps dropped, at 30 qubits complex128 and 32 complex64: passes, time, and the
    fidelity |<exact|approx>|^2 (computed on the GPU in FP64).  Then the complex64 result
    against the complex128 one for the exact QFT at 16, 24 and 33 qubits."""
    stream = torch.cuda.current_stream()

    def prep(n):
        rng = W.SplitMix64(W.SEED_BASE + 60 + n)
        b = W.CircuitBuilder(n)
        for q in range(n):
            b.g1(W.U3, q, *(2 * math.pi * rng.uniform(3)))
        return b.build()

    def overlap(a, b, chunk=1 << 26):
        """<a|b>, |a|^2, |b|^2 in FP64 over chunks (either state may be complex64)."""
        ab = aa = bb = 0.0 + 0j
        for i in range(0, a.numel(), chunk):
            x = a[i:i + chunk].to(torch.complex128)
            y = b[i:i + chunk].to(torch.complex128)
            ab += complex(torch.vdot(x, y).item())
            aa += complex(torch.vdot(x, x).item())
            bb += complex(torch.vdot(y, y).item())
        return ab, aa.real, bb.real

    out = {"approx": {}, "c64_vs_c128": {}}
    for n, dt in ((30, "c128"), (32, "c64")):
        exact = W.qft(n).build()
        p = prep(n)
        ref = qg.State(n, dt)
        ref.apply(p, qg.FUSE_GREEDY)
        ref.apply(exact, qg.FUSE_GREEDY)
        st = qg.State(n, dt)
        rows = {}
        for k in (0, 16, 12, 8, 6, 4):
            eps = 0.0 if k == 0 else math.pi / 2 ** k
            circ = W.prune_small_rotations(exact, eps)
            st.reset()
            st.apply(p, qg.FUSE_GREEDY)
            st.apply(circ, qg.FUSE_GREEDY)  # warm-up
            st.reset()
            st.apply(p, qg.FUSE_GREEDY)
            t = event_time(stream, torch, lambda: st.apply(circ, qg.FUSE_GREEDY))
            ab, aa, bb = overlap(ref.tensor, st.tensor)
            _, npass = qg.plan_passes(circ, dt, qg.FUSE_GREEDY)
            rows["exact" if k == 0 else f"eps_pi_over_2^{k}"] = {
                "gates": circ.n_gates, "passes": npass, "t_ms": round(t * 1e3, 2),
                "fidelity": abs(ab) ** 2 / (aa * bb)}
        out["approx"][f"{n}q_{dt}"] = rows
        st.close()
        ref.close()
        torch.cuda.empty_cache()
    for n in (16, 24, 33):
        circ = W.concat(prep(n), W.qft(n).build())
        a = qg.State(n, "c128")
        a.apply(circ, qg.FUSE_GREEDY)
        b = qg.State(n, "c64")
        b.apply(circ, qg.FUSE_GREEDY)
        ab, aa, bb = overlap(a.tensor, b.tensor)
        dmax = 0.0
        for i in range(0, a.tensor.numel(), 1 << 26):
            d = (a.tensor[i:i + (1 << 26)] - b.tensor[i:i + (1 << 26)].to(torch.complex128)).abs().max().item()
            dmax = max(dmax, d)
        out["c64_vs_c128"][f"{n}q"] = {"gates": circ.n_gates, "max_abs_diff": dmax,
                                       "one_minus_fidelity": 1.0 - abs(ab) ** 2 / (aa * bb),
                                       "norm_c64_minus_1": bb - 1.0}
        a.close()
        b.close()
        torch.cuda.empty_cache()
    return out


def cx_block_workloads(qg, W, torch, sizes, blocks_list, fusions, log, shots: int = 3000):
    """The paper's random CX-block unitaries (Alg. 1; 'short' = 100 blocks, 'long' = 10,000)
    followed by a 3000-shot draw, at each (qubits, dtype) of `sizes`: apply time, passes,
    amplitude updates per second, the plan's HBM bytes per second against the 8 TB/s peak,
    and the shot time, for each fusion mode (greedy width 5, learned)."""
    stream = torch.cuda.current_stream()
    out = {}
    for n, dt in sizes:
        st = qg.State(n, dt)
        for blocks in blocks_list:
            circ = W.cx_blocks(n, blocks, W.SEED_BASE + 70 + blocks)
            for fusion in fusions:
                fname = "greedy" if fusion == qg.FUSE_GREEDY else "learned"
                passes, hbm = qg.plan_bytes(circ, dt, qg.FORM_APPLY, fusion)
                st.reset()
                t = event_time(stream, torch, lambda: st.apply(circ, fusion))
                log(f"{n}q {dt} {blocks} blocks {fname}: apply {t:.4f} s")
                st.sample(100, 1)
                ts = event_time(stream, torch, lambda: st.sample(shots, W.SEED_BASE + 71))
                # the same through qg_apply_from_zero (reset included; zero tiles skipped)
                t0 = event_time(stream, torch, lambda: st.apply_from_zero(circ, fusion))
                key = f"{n}q_{dt}_{blocks}blocks_{fname}"
                out[key] = {"gates": circ.n_gates, "passes": passes, "t_s": round(t, 4),
                            "amp_updates_per_s": circ.n_gates * (1 << n) / t,
                            "hbm_frac": round(hbm / t / 1e9 / HBM_PEAK_GBS, 4),
                            "t_shots_ms": round(ts * 1e3, 3), "t_from_zero_s": round(t0, 4)}
                log(f"{key}: {out[key]}")
        st.close()
        torch.cuda.empty_cache()
    return out


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
    passes, hbm = qg.plan_bytes(circ, "c128", qg.FORM_ADJOINT)
    return {"workload": "24 qubits c128, 10-layer ansatz, 480 parameters, 710 gates",
            "t_adjoint_s": round(t_adj, 4), "t_plain_fd_s": round(t_fd, 3),
            "passes": passes, "hbm_bytes": hbm, "hbm_frac": round(hbm / t_adj / 1e9 / HBM_PEAK_GBS, 4),
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
            hbm = sum(qg.plan_bytes(c, dtype, qg.FORM_BATCHED)[1] for c in circs)
            out[f"t_batched_{dtype}_s"] = round(t_b, 4)
            out[f"amp_updates_per_s_batched_{dtype}"] = amp_updates / t_b
            # circuits above one tile stream their states in device memory, once
            # per pass and once for the observable: the bytes they move
            out[f"hbm_bytes_{dtype}"] = hbm
            out[f"hbm_frac_{dtype}"] = round(hbm / t_b / 1e9 / HBM_PEAK_GBS, 4)
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


def train_cost_model(qg, samples, log):
    """Cost model trained on pass timings the simulator makes (library MLP kernels):
    (model, info)."""
    from paper_2504_03967_amd import costmodel as cm
    t0 = time.perf_counter()
    X, y = cm.collect(samples, n_values=(20, 22, 24, 26, 28, 30, 32), log=log)
    t_collect = time.perf_counter() - t0
    n_train = int(0.85 * len(y))
    t1 = time.perf_counter()
    model, losses = cm.train(X[:n_train], y[:n_train], epochs=300, batch=128, lr=2e-3)
    t_train = time.perf_counter() - t1
    err = cm.mape(model, X[n_train:], y[n_train:])
    return model, {"samples": int(len(y)), "t_collect_s": round(t_collect, 1), "t_train_s": round(t_train, 2),
                   "train_loss_first_last": [round(float(losses[0]), 4), round(float(losses[-1]), 4)],
                   "heldout_mape": round(err, 3)}


def learned_gain(qg, W, torch, samples, log):
    """Measured time of greedy width-5 plans vs learned plans: 20 held-out CX-block / QFT
    circuits (20-30 qubits) and config 3 at 28 qubits (also against the unfused plain
    method), five alternating repeats each for the spread."""
    from paper_2504_03967_amd import costmodel as cm
    model, info = train_cost_model(qg, samples, log)
    model.install()
    circs = cm.held_out_circuits(count=20)
    res = cm.compare_plans(circs, reps=1, repeats=5)
    c3 = cm.compare_plans([W.config3(28)], reps=1, repeats=5, unfused=True)
    qg.clear_cost_model()
    model.close()
    return {**info, "circuits": len(circs),
            "t_greedy5_s": round(res["t_greedy_s"], 4), "t_learned_s": round(res["t_learned_s"], 4),
            "gain": round(res["gain"], 3), "gain_range_5_repeats": [round(res["gain_min"], 3), round(res["gain_max"], 3)],
            "greedy_spread": round(res["greedy_spread"], 4),
            "config3_28q": {"t_greedy5_s": round(c3["t_greedy_s"], 4), "t_learned_s": round(c3["t_learned_s"], 4),
                            "t_unfused_s": round(c3["t_unfused_s"], 3), "gain": round(c3["gain"], 3),
                            "gain_range_5_repeats": [round(c3["gain_min"], 3), round(c3["gain_max"], 3)],
                            "gain_vs_unfused": round(c3["gain_vs_unfused"], 2)},
            "gain_config3": round(c3["gain"], 3)}


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
        print(json.dumps({"error": "the benchmark runs on one GPU (the state and its kernels on cuda:0); --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_2504_03967_amd import qg
    from paper_2504_03967_amd import workloads as W

    torch.cuda.set_device(0)
    if args.config3_only:
        print(json.dumps({"config3": config3_timing(qg, W, torch, args.config3_only)}), flush=True)
        return
    if args.form_only == "adjoint":
        circ = W.config5()
        masks = W.zz_chain_masks(circ.n_qubits)
        for _ in range(2):
            t, _ = timed(lambda: qg.adjoint_grad(circ, masks, np.ones(masks.size), circ.n_params),
                         torch.cuda.synchronize)
        passes, hbm = qg.plan_bytes(circ, "c128", qg.FORM_ADJOINT)
        print(json.dumps({"adjoint": {"t_s": round(t, 5), "passes": passes, "hbm_bytes": hbm,
                                      "hbm_frac": round(hbm / t / 1e9 / HBM_PEAK_GBS, 4)}}), flush=True)
        return
    if args.form_only == "batched":
        circs = W.config4()
        out = {}
        for dtype in ("c128", "c64"):
            b = qg.Batch(circs, dtype)
            b.launch()
            t, _ = timed(b.launch, torch.cuda.synchronize)
            b.close()
            hbm = sum(qg.plan_bytes(c, dtype, qg.FORM_BATCHED)[1] for c in circs)
            out[dtype] = {"t_s": round(t, 5), "hbm_bytes": hbm,
                          "hbm_frac": round(hbm / t / 1e9 / HBM_PEAK_GBS, 4)}
        print(json.dumps({"batched": out}), flush=True)
        return
    if args.paper_workloads:
        model = train_cost_model(qg, args.cm_samples, log)[0]
        model.install()
        res = cx_block_workloads(qg, W, torch, [(28, "c128"), (30, "c128"), (32, "c128"), (34, "c64")],
                                 (100, 10000), (qg.FUSE_GREEDY, qg.FUSE_LEARNED), log)
        qg.clear_cost_model()
        model.close()
        print(json.dumps({"cx_block_workloads": res}), flush=True)
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
        return qg.FUSE_GREEDY if name.startswith(("fused", "dense")) else qg.FUSE_NONE

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
    dense_names = [nm for nm, _ in parts if nm.startswith("dense")]
    dense_gates = sum(c.n_gates for nm, c in parts if nm in dense_names)
    dense_time = sum(e0.elapsed_time(e1) * 1e-3 for nm, e0, e1 in events if nm in dense_names)
    value_nodense = (gates_per_step - dense_gates) * (1 << n) * args.steps / (elapsed - dense_time)

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
    # Dense blocks are dense complex products on the matrix cores: 8 2^(n + k) flops for a
    # k-qubit block (4 real products of 2^k x 2^k by 2^k x 2^(n - k)), against the MFMA peak
    # of the precision (FP64 78.6 TFLOP/s for complex128, FP32 157.3 for complex64).
    mfma_peak = 78.6 if args.dtype == "c128" else 157.3
    for name, c in parts:
        if name.startswith("dense_k"):
            k = int(name[-1])
            tf = 8.0 * 2.0 ** (n + k) / float(np.mean(per[name])) / 1e12
            sweep[name + "_TFLOPs"] = round(tf, 2)
            sweep[name + "_mfma_frac"] = round(tf / mfma_peak, 4)
            sweep[name + "_hbm_frac"] = round(sweep[name + "_GBps"] / HBM_PEAK_GBS, 4)
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
        extras["paper_shaped"]["cx_blocks"] = cx_block_workloads(qg, W, torch, [(30, "c128")], (100, 1000),
                                                                 (qg.FUSE_GREEDY,), log)
        log("QCrank at Table 2 shapes")
        extras["qcrank_table2"] = qcrank_table2(qg, W, torch)
        log("QFT precision and approximation")
        extras["qft_study"] = qft_study(qg, W, torch)
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
                               f"fused U3 groups k=2..6, dense blocks of 48 / 64 gates on 5 / 6 qubits, "
                               f"then probs(1024), 10^4 shots, {n - 1} ZZ expvals",
                   "n_qubits": n, "gates_per_step": gates_per_step, "state_GiB": (1 << n) * amp_bytes / 2 ** 30},
        "hbm_frac": round(achieved / HBM_PEAK_GBS, 4),
        # the same step without its two dense-block parts (112 of its gates), for
        # comparison with sweeps that have none
        "value_without_dense_parts": value_nodense,
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
