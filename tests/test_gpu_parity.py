"""GPU path (libqg.so through its C ABI) against the FP64 oracle, element by element.

Tolerances: max amplitude error 1e-12 (complex128) / 1e-5 (complex64);
expectations per Z-string term to the same; shots by chi-square p > 0.01 and,
with the shared Philox stream, >= 99.9 % of shots identical to the oracle's.
"""
import math

import numpy as np
import pytest
import torch
from scipy.stats import chi2

import oracle
from paper_2504_03967_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module")
def qg():
    from paper_2504_03967_amd import qg as lib
    assert torch.cuda.is_available()
    return lib


def run(qg, circ, dtype="c128", fusion=1):
    st = qg.State(circ.n_qubits, dtype)
    st.apply(circ, fusion)
    return st


def host(st):
    torch.cuda.synchronize()
    return st.tensor.cpu().numpy().astype(np.complex128)


def prep_layer(n, seed):
    rng = W.SplitMix64(seed)
    b = W.CircuitBuilder(n)
    for q in range(n):
        b.g1(W.U3, q, *(2 * math.pi * rng.uniform(3)))
    return b.build()


def chi_square_p(counts, p, shots):
    obs, exp_ = [], []
    o = e = 0.0
    for c, pi in zip(counts, p):
        o += c
        e += pi * shots
        if e >= 5:
            obs.append(o); exp_.append(e); o = e = 0.0
    if e > 0 and obs:
        obs[-1] += o; exp_[-1] += e
    obs, exp_ = np.array(obs), np.array(exp_)
    return chi2.sf(np.sum((obs - exp_) ** 2 / exp_), len(obs) - 1)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 9, 13, 15])
def test_every_op_at_every_position(qg, n, dtype):
    rng = np.random.default_rng(n)
    for op in range(10):
        if op in W.TWO_QUBIT and n < 2:
            continue
        b = W.CircuitBuilder(n)
        prep = prep_layer(n, 17 * n + op)
        for (o, q0, q1), p in zip(prep.gate_type, prep.gate_param):
            b.add(o, q0, q1, p)
        for t in range(n):
            for c in (range(n) if op in W.TWO_QUBIT else [-1]):
                if c == t:
                    continue
                b.add(op, c, t, rng.uniform(0, 2 * math.pi, 3))
        circ = b.build()
        ref = oracle.simulate(circ)
        for fusion in (0, 1):
            got = host(run(qg, circ, dtype, fusion))
            err = np.max(np.abs(got - ref))
            assert err < TOL[dtype], (op, fusion, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 7, 12, 16, 20])
def test_random_circuits(qg, n, dtype):
    circ = W.random_circuit(n, 300, seed=500 + n)
    ref = oracle.simulate(circ)
    for fusion in (0, 1):
        got = host(run(qg, circ, dtype, fusion))
        assert np.max(np.abs(got - ref)) < TOL[dtype], fusion


def test_config1_outputs(qg):
    circ = W.config1()
    st = run(qg, circ, "c128", 1)
    psi = oracle.simulate(circ)
    assert np.max(np.abs(host(st) - psi)) < 1e-12
    p_ref = oracle.probs(psi)
    assert np.max(np.abs(st.probs().cpu().numpy() - p_ref)) < 1e-12
    masks = W.zz_chain_masks(12)
    terms, total = st.expval(masks, np.ones(11))
    ev = oracle.expval(psi, masks)
    assert np.max(np.abs(terms.cpu().numpy() - ev)) < 1e-12
    assert abs(float(total) - ev.sum()) < 11e-12
    seed = W.SEED_BASE
    shots = st.sample(10000, seed).cpu().numpy().astype(np.uint64)
    ref_shots = oracle.sample(psi, 10000, seed)
    assert np.mean(shots == ref_shots) >= 0.999
    counts = np.bincount(shots.astype(np.int64), minlength=4096)
    assert chi_square_p(counts, p_ref, 10000) > 0.01


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_config2_qcrank_closed_form_and_shots(qg, dtype):
    circ, p = W.config2()
    st = run(qg, circ, dtype, 1)
    got = host(st)
    a = np.arange(1 << 16) & 0xFF
    amp = np.full(1 << 16, 2 ** -4.0)
    for d in range(8):
        bit = (np.arange(1 << 16) >> (8 + d)) & 1
        amp *= np.where(bit == 0, np.sqrt(p[d, a]), np.sqrt(1 - p[d, a]))
    assert np.max(np.abs(got - amp)) < TOL[dtype]
    psi = oracle.simulate(circ)
    assert np.max(np.abs(got - psi)) < TOL[dtype]
    shots = st.sample(1_000_000, W.SEED_BASE + 1).cpu().numpy().astype(np.int64)
    counts = np.bincount(shots, minlength=1 << 16)
    assert chi_square_p(counts, np.abs(psi) ** 2, 1_000_000) > 0.01
    if dtype == "c128":
        ref = oracle.sample(psi, 1_000_000, W.SEED_BASE + 1).astype(np.int64)
        assert np.mean(shots == ref) >= 0.999
    # reconstruction of the synthetic pixels: p_hat(d, a) = counts(a, d = 0) / counts(a)
    addr = shots & 0xFF
    n_a = np.bincount(addr, minlength=256)
    for d in range(8):
        zero = ((shots >> (8 + d)) & 1) == 0
        n0 = np.bincount(addr[zero], minlength=256)
        phat = n0 / n_a
        z = (phat - p[d]) / np.sqrt(np.maximum(p[d] * (1 - p[d]), 1e-12) / n_a)
        assert np.all(np.abs(z) < 5.5)


@pytest.fixture(scope="module")
def config3_26q():
    n = 26
    circ = W.config3(n)
    return circ, oracle.simulate(circ)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_config3_full_depth_every_amplitude(qg, config3_26q, dtype):
    """The large-circuit workload at full depth (100 random U3 + CX layers, then the exact
    QFT, 4264 gates) on 26 qubits, greedy fusion as at full size (deep multi-layout tile
    passes, fused diagonal runs, standalone SWAPs): every amplitude against the oracle, the
    whole-state 2-norm of the error, the 1024 seeded probabilities and <Z_0 Z_25>."""
    circ, psi = config3_26q
    n = circ.n_qubits
    kinds = qg.plan_kernels(circ, dtype, qg.FUSE_GREEDY)
    passes = qg.plan_passes(circ, dtype, qg.FUSE_GREEDY)[1]
    assert kinds.count("tile") > 100 and passes < circ.n_gates / 10
    st = run(qg, circ, dtype, 1)
    got = host(st)
    err = np.abs(got - psi)
    assert err.max() < TOL[dtype], float(err.max())
    assert np.linalg.norm(got - psi) < TOL[dtype], float(np.linalg.norm(got - psi))
    idx = W.config3_indices(n)
    p = st.probs(idx).cpu().numpy()
    pref = np.abs(psi[idx.astype(np.int64)]) ** 2
    # probabilities are ~2^-26: compare them on their own scale as well
    assert np.max(np.abs(p - pref)) / pref.mean() < (1e-10 if dtype == "c128" else 1e-4)
    masks = np.array([0, (1 << 0) | (1 << (n - 1))], dtype=np.uint64)
    terms, _ = st.expval(masks)
    ref = oracle.expval(psi, masks)
    assert np.max(np.abs(terms.cpu().numpy() - ref)) < TOL[dtype]
    assert abs(terms[0].item() - 1) < (1e-13 if dtype == "c128" else 1e-5)
    st.close()


@pytest.mark.parametrize("n", [3, 9, 14, 23])
def test_expval_many_terms_and_weights(qg, n):
    """Up to 64 masks share one read of the state; 150 masks take three reads.  Masks with
    bits only in the thread part (index bits 0..7), only in the row part (8..11), only above,
    and random ones; states smaller than one 4096-amplitude group as well."""
    circ = W.random_circuit(n, 200, seed=3 + n)
    st = run(qg, circ)
    psi = oracle.simulate(circ)
    rng = np.random.default_rng(n)
    full = (1 << n) - 1
    fixed = [0, full, 0xFF & full, 0xF00 & full, full & ~0xFFF, 1 << (n - 1), 0x101 & full]
    masks = np.concatenate([np.array(fixed, dtype=np.uint64),
                            rng.integers(0, 1 << n, 150 - len(fixed)).astype(np.uint64)])
    coeffs = rng.normal(size=masks.size)
    for k in (1, 3, 16, 41, 64, 65, 150):
        terms, total = st.expval(masks[:k], coeffs[:k])
        ref = oracle.expval(psi, masks[:k])
        assert np.max(np.abs(terms.cpu().numpy() - ref)) < 1e-12, k
        assert abs(float(total) - np.dot(coeffs[:k], ref)) < 1e-12 * np.sum(np.abs(coeffs[:k])), k


def test_probs_index_list_ragged(qg):
    n = 18
    circ = W.random_circuit(n, 100, seed=4)
    st = run(qg, circ)
    psi = oracle.simulate(circ)
    idx = np.random.default_rng(1).integers(0, 1 << n, 1003).astype(np.uint64)
    p = st.probs(idx).cpu().numpy()
    assert np.max(np.abs(p - np.abs(psi[idx.astype(np.int64)]) ** 2)) < 1e-12
    full = st.probs().cpu().numpy()
    assert np.max(np.abs(full - np.abs(psi) ** 2)) < 1e-12


@pytest.mark.parametrize("n", [1, 6, 7, 13])
def test_sampling_small_and_degenerate(qg, n):
    b = W.CircuitBuilder(n).g1(W.X, n - 1)
    st = run(qg, b.build())
    s = st.sample(777, 5).cpu().numpy()
    assert np.all(s == (1 << (n - 1)))
    assert st.sample(0, 5).numel() == 0
    circ = W.random_circuit(n, 50, seed=n)
    st = run(qg, circ)
    psi = oracle.simulate(circ)
    got = st.sample(5000, 99).cpu().numpy().astype(np.uint64)
    assert np.mean(got == oracle.sample(psi, 5000, 99)) >= 0.999


def test_reset_and_repeat_are_bitwise_deterministic(qg):
    circ = W.config3(16, layers=10)
    st = run(qg, circ)
    a = host(st)
    t1, _ = st.expval(W.zz_chain_masks(16))
    st.reset()
    st.apply(circ, 1)
    b = host(st)
    t2, _ = st.expval(W.zz_chain_masks(16))
    assert np.array_equal(a, b)
    assert torch.equal(t1, t2)


def test_validation_errors_leave_state_untouched(qg):
    st = run(qg, W.config1())
    before = host(st)
    bad = W.CircuitBuilder(12).g2(W.CX, 3, 3).build()
    with pytest.raises(qg.QGError) as e:
        st.apply(bad)
    assert e.value.status == qg.QG_EINVAL and "q0 == q1" in str(e.value)
    with pytest.raises(qg.QGError):
        st.apply(W.CircuitBuilder(11).g1(W.H, 0).build())
    with pytest.raises(qg.QGError):
        st.expval([1 << 12])
    with pytest.raises(qg.QGError):
        st.probs([1 << 12])
    nan = W.CircuitBuilder(12).g1(W.RX, 0, float("nan")).build()
    with pytest.raises(qg.QGError):
        st.apply(nan)
    assert np.array_equal(host(st), before)


def test_tile_order_settings_are_bitwise_identical(qg):
    """The tile order of a launch (XCD-contiguous ranges, XOR swizzle, persistent blocks that
    prefetch their next tile) only changes which workgroup streams which tile: the state must
    come out bit for bit the same, and match the oracle.  The circuit has fused, single-gate,
    controlled and standalone-SWAP passes."""
    n = 22  # 1024 tiles: persistent blocks stream several tiles each
    circ = W.concat(W.random_circuit(n, 80, seed=41),
                    W.CircuitBuilder(n).g2(W.SWAP, 5, 14).g2(W.SWAP, 16, 9).g2(W.CX, 15, 3).build())
    ref = oracle.simulate(circ)
    keys = ("xcd", "pipe", "swz_bits") + tuple(f"cls{k}_swz_c128" for k in range(5))
    saved = {k: qg.get_tuning(k) for k in keys}
    states = []
    try:
        for xcd, pipe, swz in ((0, 0, 0), (0, 0, 3), (1, 0, 0), (1, 0, 3), (0, 2, 0), (1, 2, 3), (1, 1, 0)):
            qg.set_tuning("xcd", xcd)
            qg.set_tuning("pipe", pipe)
            for k in keys[2:]:
                qg.set_tuning(k, swz)
            st = run(qg, circ)
            states.append(host(st))
            st.close()
    finally:
        for k, v in saved.items():
            qg.set_tuning(k, v)
    assert np.max(np.abs(states[0] - ref)) < TOL["c128"]
    for s in states[1:]:
        assert np.array_equal(s, states[0])


def test_persistent_prefetching_blocks_complex64(qg):
    """complex64 passes on persistent blocks (several tiles per block, prefetch of the next
    tile) give the same bits as one tile per block."""
    n = 24
    circ = W.random_circuit(n, 60, seed=43)
    saved = qg.get_tuning("pipe")
    out = []
    try:
        for pipe in (0, 2):
            qg.set_tuning("pipe", pipe)
            st = run(qg, circ, "c64")
            torch.cuda.synchronize()
            out.append(st.tensor.cpu().numpy())
            st.close()
    finally:
        qg.set_tuning("pipe", saved)
    assert np.array_equal(out[0], out[1])
    assert abs(np.sum(np.abs(out[0].astype(np.complex128)) ** 2) - 1) < 1e-4


def diagonal_heavy_circuit(n, seed, blocks=12):
    """Layers of U3 separated by long runs of CP / CZ / RZ on random qubits, so that passes
    hold diagonal runs whose qubits are register slots, thread bits and qubits outside the
    tile, in every combination."""
    rng = W.SplitMix64(seed)
    b = W.CircuitBuilder(n)
    for _ in range(blocks):
        for q in range(n):
            b.g1(W.U3, q, *(2 * math.pi * rng.uniform(3)))
        for _ in range(3 * n):
            op = (W.CP, W.CZ, W.RZ)[int(rng.below(3)[0])]
            q1 = int(rng.below(n)[0])
            if op == W.RZ:
                b.g1(W.RZ, q1, float(2 * math.pi * rng.uniform(1)[0]))
                continue
            q0 = int(rng.below(n)[0])
            while q0 == q1:
                q0 = int(rng.below(n)[0])
            b.add(op, q0, q1, [float(2 * math.pi * rng.uniform(1)[0]), 0.0, 0.0])
    return b.build()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [9, 14, 17])
def test_fused_diagonal_runs_match_oracle(qg, n, dtype):
    """Runs of diagonal gates fused into one factor per amplitude (tables built on the host,
    per-thread entries on the device) against the oracle, and against unfused runs."""
    circ = W.concat(diagonal_heavy_circuit(n, 100 + n), W.qft(n).build())
    ref = oracle.simulate(circ)
    saved = qg.get_tuning("diag_run_min")
    out = []
    try:
        for m in (3, 0):
            qg.set_tuning("diag_run_min", m)
            for fusion in (0, 1):
                st = run(qg, circ, dtype, fusion)
                out.append(host(st))
                st.close()
    finally:
        qg.set_tuning("diag_run_min", saved)
    for o in out:
        assert np.max(np.abs(o - ref)) < TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_cx_block_unitary_matches_oracle(qg, dtype):
    """A random CX-block unitary (the paper's Alg. 1 generator) on 16 qubits."""
    circ = W.cx_blocks(16, 400, seed=W.SEED_BASE + 9)
    ref = oracle.simulate(circ)
    for fusion in (0, 1):
        st = run(qg, circ, dtype, fusion)
        assert np.max(np.abs(host(st) - ref)) < TOL[dtype]
        st.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [12, 16])
def test_standalone_swaps_as_permutations(qg, n, dtype):
    """Standalone SWAPs run as permutation kernels (half the state when both qubits are above
    the cache-line bits, a cross-lane exchange when the lower one is inside a line): against
    the oracle, and bit for bit against the same SWAPs run as tile passes."""
    pairs = [(0, 1), (1, 2), (2, 0), (0, 5), (3, 4), (1, n - 1), (n - 1, 4), (5, 6), (6, n - 2), (2, 7)]
    b = W.CircuitBuilder(n)
    prep = prep_layer(n, 300 + n)
    for (o, q0, q1), p in zip(prep.gate_type, prep.gate_param):
        b.add(o, q0, q1, p)
    for x, y in pairs:
        b.g2(W.SWAP, x, y)
    circ = b.build()
    ref = oracle.simulate(circ)
    saved = qg.get_tuning("lane_swap")
    out = []
    try:
        for lane in (1, 0):
            qg.set_tuning("lane_swap", lane)
            st = run(qg, circ, dtype, 0)
            out.append(host(st))
            st.close()
    finally:
        qg.set_tuning("lane_swap", saved)
    assert np.max(np.abs(out[0] - ref)) < TOL[dtype]
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [12, 17])
def test_lane_gates_match_oracle(qg, n, dtype):
    """Single one-qubit gates and CX whose target lies inside a cache line run as a cross-lane
    exchange (whole-line accesses): every op on every such target, CX controls below, inside
    and above the line, against the oracle and against the same gates as tile passes."""
    lb = 4 if dtype == "c64" else 3
    rng = np.random.default_rng(n)
    b = W.CircuitBuilder(n)
    prep = prep_layer(n, 500 + n)
    for (o, q0, q1), p in zip(prep.gate_type, prep.gate_param):
        b.add(o, q0, q1, p)
    for t in range(lb):
        for op in (W.H, W.X, W.RX, W.RY, W.U3):
            b.add(op, -1, t, rng.uniform(0, 2 * math.pi, 3))
        for c in sorted({(t + 1) % lb, lb, 5, n - 1} - {t}):
            b.g2(W.CX, c, t)
    circ = b.build()
    ref = oracle.simulate(circ)
    saved = qg.get_tuning("lane_gate")
    try:
        for lane in (1, 0):
            qg.set_tuning("lane_gate", lane)
            st = run(qg, circ, dtype, 0)
            assert np.max(np.abs(host(st) - ref)) < TOL[dtype]
            st.close()
    finally:
        qg.set_tuning("lane_gate", saved)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_half_lds_exchanges_are_bitwise_identical(qg, dtype):
    """Multi-phase passes move the tile between register layouts through LDS either as whole
    complex values or as real parts then imaginary parts: a permutation either way, so the
    states (forward passes) and the adjoint gradients (two states per pass) agree bit for bit,
    and match the oracle."""
    n = 18
    circ = W.config3(n, layers=6)
    ref = oracle.simulate(circ)
    _, npass = qg.plan_passes(circ, dtype, 1)
    assert npass < circ.n_gates
    train = W.config5(n=16, layers=4)
    masks = W.zz_chain_masks(train.n_qubits)
    coeffs = np.linspace(0.5, 1.5, masks.size)
    key = f"half_lds_{dtype}"
    saved = qg.get_tuning(key)
    states, grads = [], []
    try:
        for h in (0, 1):
            qg.set_tuning(key, h)
            st = run(qg, circ, dtype, 1)
            states.append(host(st))
            st.close()
            grads.append(qg.adjoint_grad(train, masks, coeffs, train.n_params, dtype)[1].cpu().numpy())
    finally:
        qg.set_tuning(key, saved)
    assert np.max(np.abs(states[0] - ref)) < TOL[dtype]
    assert np.array_equal(states[0], states[1])
    assert np.array_equal(grads[0], grads[1])


def test_large_shot_counts(qg):
    """3000 * 2^12 shots (the paper's 3000 * 2^m shot rule) from one call: every index is in
    range and the counts pass the chi-square test against the oracle's probabilities; a
    prefix of the shots equals the oracle's draws for the same Philox counters."""
    n = 12
    shots = 3000 << n
    circ = prep_layer(n, 77)
    psi = oracle.simulate(circ)
    st = run(qg, circ, "c128", 1)
    idx = st.sample(shots, 1234).cpu().numpy().astype(np.uint64)
    st.close()
    assert idx.size == shots and int(idx.max()) < (1 << n)
    counts = np.bincount(idx.astype(np.int64), minlength=1 << n)
    assert chi_square_p(counts, np.abs(psi) ** 2, shots) > 0.01
    assert np.mean(idx[:10000] == oracle.sample(psi, 10000, 1234)) >= 0.999


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_apply_from_zero_equals_reset_and_apply(qg, dtype):
    """qg_apply_from_zero passes visit only the tiles that can hold nonzero amplitudes; the
    state equals qg_state_reset + qg_apply_circuit bit for bit, for both fusion modes, on
    circuits whose passes run on the tile, lane-gate, SWAP and dense kernels; and it matches
    the oracle."""
    n = 20 if dtype == "c128" else 21
    special = W.CircuitBuilder(n)
    special.g2(W.SWAP, n - 1, n - 3)          # standalone SWAP first: nothing is skipped after it
    special.g1(W.H, 0)
    special = W.concat(special.build(), W.random_circuit(n, 40, seed=9))
    lane = W.CircuitBuilder(n)
    for q in range(6, n):
        lane.g1(W.H, q)                       # tile passes first, then a lane-kernel gate
    lane.g1(W.RY, 1, 0.3)
    lane = W.concat(lane.build(), W.cx_blocks(n, 20, 4))
    circs = [W.qft(n).build(), W.cx_blocks(n, 60, 3), W.config3(n, layers=3), special, lane]
    a = qg.State(n, dtype)
    b = qg.State(n, dtype)
    junk = prep_layer(n, 5)
    for k, c in enumerate(circs):
        for fusion in (qg.FUSE_NONE, qg.FUSE_GREEDY):
            a.reset()
            a.apply(c, fusion)
            b.apply(junk, qg.FUSE_GREEDY)     # any prior contents: the call resets first
            b.apply_from_zero(c, fusion)
            torch.cuda.synchronize()
            assert torch.equal(a.tensor, b.tensor), (k, fusion)
            if k == 1 and fusion == qg.FUSE_GREEDY:
                assert np.max(np.abs(host(b) - oracle.simulate(c))) < TOL[dtype]
    # a dense block among the passes
    saved = qg.get_tuning("dense_min_gates")
    try:
        qg.set_tuning("dense_min_gates", 1)
        db = W.CircuitBuilder(n)
        for q in range(n):
            db.g1(W.H, q)
        for q in (0, 3, 7, 12):
            db.g1(W.RY, q, 0.1 * q + 0.2)
        for q in (0, 3, 7):
            db.g2(W.CX, q, 12)
        c = db.build()
        a.reset()
        a.apply(c, qg.FUSE_GREEDY)
        b.apply_from_zero(c, qg.FUSE_GREEDY)
        torch.cuda.synchronize()
        assert torch.equal(a.tensor, b.tensor)
    finally:
        qg.set_tuning("dense_min_gates", saved)
    a.close()
    b.close()
