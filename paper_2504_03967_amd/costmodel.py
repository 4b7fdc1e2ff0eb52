"""Learned fusion: timing dataset, GPU training and evaluation of the cost model.

The dataset is made by the simulator itself: random candidate passes (the first
greedy pass of a random gate list under one of the candidate fusion
configurations) are executed on the GPU and timed with HIP events; the
features are the library's own pass features (qg_pass_features).  The target
is ln(pass time in microseconds).  Training runs the library's MLP kernels.
"""
from __future__ import annotations

import math
import time
from typing import Dict, List, Sequence, Tuple

import numpy as np
import torch

from . import qg
from . import workloads as W


def _config_knobs(dtype: str, k: int) -> Dict[str, int]:
    d = "c128" if dtype == "c128" else "c64"
    tile = int(qg.get_tuning(f"tile_bits_{d}"))
    high = 4 + k
    return {f"tile_bits_{d}": tile, f"max_high_{d}": high, f"low_bits_{d}": tile - high}


def set_config(dtype: str, k: int) -> Dict[str, int]:
    """Points the greedy planner at candidate config k; returns the previous knob values."""
    prev = {}
    for key, v in _config_knobs(dtype, k).items():
        prev[key] = qg.get_tuning(key)
    # order matters for clamping: widen max_high before shrinking low_bits and back
    for key in sorted(prev, key=lambda s: 0 if s.startswith("max_high") else 1):
        qg.set_tuning(key, _config_knobs(dtype, k)[key])
    return prev


def restore(prev: Dict[str, int]) -> None:
    for key, v in prev.items():
        qg.set_tuning(key, v)


def random_gates(n: int, n_gates: int, rng: W.SplitMix64, ops: Sequence[int] = tuple(range(10)),
                 max_pool: int = 0) -> W.Circuit:
    """Random gate list on a random subset of the qubits (locality varies per call)."""
    top = n if max_pool <= 0 else min(n, max_pool)
    size = 2 + int(rng.below(top - 1)[0])
    pool = rng.shuffle(range(n))[:size]
    b = W.CircuitBuilder(n)
    for _ in range(n_gates):
        op = ops[int(rng.below(len(ops))[0])]
        q1 = pool[int(rng.below(len(pool))[0])]
        q0 = -1
        if op in W.TWO_QUBIT:
            q0 = pool[int(rng.below(len(pool))[0])]
            while q0 == q1:
                q0 = pool[int(rng.below(len(pool))[0])] if len(pool) > 1 else (q1 + 1) % n
        b.add(op, q0, q1, 2 * math.pi * rng.uniform(3))
    return b.build()


def first_pass(circ: W.Circuit, dtype: str, k: int) -> W.Circuit:
    """The first pass greedy config k forms on circ, as a circuit of its own."""
    prev = set_config(dtype, k)
    try:
        pog, _ = qg.plan_passes(circ, dtype, qg.FUSE_GREEDY)
    finally:
        restore(prev)
    sel = pog == 0
    return W.Circuit(circ.n_qubits, circ.gate_type[sel].copy(), circ.gate_param[sel].copy(),
                     np.full(int(sel.sum()), -1, np.int32))


def time_apply(st: "qg.State", circ: W.Circuit, fusion: int, reps: int = 3) -> float:
    """Median wall time (seconds, HIP events) of applying circ to the state."""
    stream = torch.cuda.current_stream()
    st.apply(circ, fusion)  # warm (plan cache, code)
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st.apply(circ, fusion)
        e1.record(stream)
        ts.append((e0, e1))
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ts])) * 1e-3


def collect(n_samples: int, n_values: Sequence[int] = (20, 22, 24, 26, 28, 30, 32),
            dtypes: Sequence[str] = ("c128", "c64"), seed: int = W.SEED_BASE + 5, reps: int = 3,
            log=None) -> Tuple[np.ndarray, np.ndarray]:
    """(X [N, 24] float32 features, y [N] float32 = ln(us)) of timed random passes."""
    rng = W.SplitMix64(seed)
    states: Dict[Tuple[int, str], qg.State] = {}
    X, y = [], []
    t0 = time.time()
    for s in range(n_samples):
        n = int(n_values[int(rng.below(len(n_values))[0])])
        dtype = dtypes[int(rng.below(len(dtypes))[0])]
        k = int(rng.below(qg.PASS_CONFIGS)[0])
        G = 1 + int(rng.below(80)[0])
        if k == qg.PASS_DENSE:
            # a run on at most 6 qubits, executed as one dense block
            block = random_gates(n, G, rng, max_pool=6)
        else:
            block = first_pass(random_gates(n, G, rng), dtype, k)
        f, npass = qg.pass_features(block, dtype, k)
        assert npass == 1
        key = (n, dtype)
        if key not in states:
            states[key] = qg.State(n, dtype)
            states[key].apply(W.uniform_superposition(n), qg.FUSE_GREEDY)
        prev = set_config(dtype, 3 if k == qg.PASS_DENSE else k)
        prev_dense = qg.get_tuning("dense_min_gates")
        # the sample runs as the strategy its features name: a dense block, or a tile
        # pass even where the planner's own threshold would pick a dense block
        qg.set_tuning("dense_min_gates", 1 if k == qg.PASS_DENSE else 1 << 30)
        try:
            t = time_apply(states[key], block, qg.FUSE_GREEDY, reps)
        finally:
            restore(prev)
            qg.set_tuning("dense_min_gates", prev_dense)
        X.append(f)
        y.append(math.log(t * 1e6))
        if log and (s + 1) % 200 == 0:
            log(f"cost model: {s + 1}/{n_samples} passes timed ({time.time() - t0:.1f} s)")
    for st in states.values():
        st.close()
    return np.array(X, np.float32), np.array(y, np.float32)


def train(X: np.ndarray, y: np.ndarray, epochs: int = 200, batch: int = 128, lr: float = 2e-3,
          seed: int = 0) -> Tuple["qg.MLP", np.ndarray]:
    m = qg.MLP(qg.PASS_FEATURES, seed=seed)
    losses = m.train(X, y, epochs=epochs, batch=batch, lr=lr, seed=seed + 1)
    return m, losses


def mape(model: "qg.MLP", X: np.ndarray, y: np.ndarray) -> float:
    """Mean absolute percentage error of predicted pass time vs measured."""
    pred = model.forward(X)
    return float(np.mean(np.abs(np.exp(pred) - np.exp(y)) / np.exp(y)))


def held_out_circuits(count: int = 20, seed: int = W.SEED_BASE + 6, n_values=(20, 24, 26, 28, 30)):
    """Random CX-block unitaries (Alg. 1) of 30-89 blocks, every other one followed by a QFT,
    for plan comparisons."""
    rng = W.SplitMix64(seed)
    out = []
    for c in range(count):
        n = int(n_values[c % len(n_values)])
        blocks = 30 + int(rng.below(60)[0])
        circ = W.cx_blocks(n, blocks, int(rng.next_u64(1)[0] % np.uint64(1 << 62)))
        if c % 2 == 0:
            circ = W.concat(circ, W.qft(n).build())
        out.append(circ)
    return out


def compare_plans(circs: List[W.Circuit], dtype: str = "c128", reps: int = 3, repeats: int = 1,
                  unfused: bool = False) -> Dict[str, object]:
    """Measured time of greedy-5 vs learned plans (the installed model) on the same circuits,
    summed over the circuits, `repeats` times in alternation (greedy, learned, greedy, ...),
    so that the spread of the totals shows the run-to-run noise; optionally the unfused plain
    method (one pass per gate) once."""
    states: Dict[int, qg.State] = {}
    rows = []
    tg = np.zeros(repeats)
    tl = np.zeros(repeats)
    tn = 0.0
    for c in circs:
        if c.n_qubits not in states:
            states[c.n_qubits] = qg.State(c.n_qubits, dtype)
        st = states[c.n_qubits]
        g = np.zeros(repeats)
        l = np.zeros(repeats)
        for r in range(repeats):
            g[r] = time_apply(st, c, qg.FUSE_GREEDY, reps)
            l[r] = time_apply(st, c, qg.FUSE_LEARNED, reps)
        tg += g
        tl += l
        if unfused:
            tn += time_apply(st, c, qg.FUSE_NONE, 1)
        rows.append((c.n_qubits, c.n_gates, qg.plan_passes(c, dtype, qg.FUSE_GREEDY)[1],
                     qg.plan_passes(c, dtype, qg.FUSE_LEARNED)[1], float(np.median(g)), float(np.median(l))))
    for st in states.values():
        st.close()
    gains = tg / tl
    out = {"t_greedy_s": float(np.median(tg)), "t_learned_s": float(np.median(tl)),
           "gain": float(np.median(tg) / np.median(tl)),
           "gain_min": float(gains.min()), "gain_max": float(gains.max()),
           # run-to-run spread of the same plan: relative range of the greedy totals
           "greedy_spread": float((tg.max() - tg.min()) / np.median(tg)), "rows": rows}
    if unfused:
        out["t_unfused_s"] = tn
        out["gain_vs_unfused"] = tn / float(np.median(tl))
    return out
