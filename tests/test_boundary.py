"""Host-side checks of the C ABI: the library loads, exports every declared symbol,
validates its inputs, and plans every gate exactly once, in order (no GPU needed)."""
import os
import re

import numpy as np
import pytest

from paper_2504_03967_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def qg():
    from paper_2504_03967_amd import qg as lib
    return lib


def declared_functions():
    text = open(os.path.join(ROOT, "include", "qg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qg_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function(qg):
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(qg.lib, name), name
    assert set(qg.EXPORTS) == set(names)
    assert "gfx950" in qg.version()


def dependency_order_ok(circ, pog):
    """Gates that share a qubit keep their order across passes."""
    last = {}
    for i, (op, q0, q1) in enumerate(circ.gate_type):
        for q in ((q0, q1) if op in W.TWO_QUBIT else (q1,)):
            if q in last and pog[last[q]] > pog[i]:
                return False
            last[q] = i
    return True


def test_plan_covers_every_gate_once_respecting_dependencies(qg):
    for circ in (W.config1(), W.config2()[0], W.config3(26, layers=5), W.random_circuit(20, 500, seed=1)):
        for dtype in ("c128", "c64"):
            for fusion in (0, 1, 2):
                pog, npass = qg.plan_passes(circ, dtype, fusion)
                assert pog.size == circ.n_gates
                assert pog.min() == 0 and pog.max() == npass - 1
                assert set(np.unique(pog)) == set(range(npass))
                assert dependency_order_ok(circ, pog)
                if fusion == 0:
                    assert npass == circ.n_gates and np.all(np.diff(pog) == 1)


def test_commutation_aware_schedule_reduces_passes(qg):
    circ = W.config3(31)
    _, npass = qg.plan_passes(circ, "c128", 1)
    assert npass < 300  # in-order greedy fusion needs 721 passes here


def test_greedy_fusion_respects_width(qg):
    circ = W.config3(30, layers=4, with_qft=False)
    for dtype, low in (("c128", 7), ("c64", 8)):
        pog, npass = qg.plan_passes(circ, dtype, 1)
        assert npass < circ.n_gates / 4
        for p in range(npass):
            rows = circ.gate_type[pog == p]
            targets = set()
            for op, q0, q1 in rows:
                if op in (W.H, W.X, W.RX, W.RY, W.U3, W.CX):
                    targets.add(int(q1))
                elif op == W.SWAP:
                    targets |= {int(q0), int(q1)}
            assert len([q for q in targets if q >= low]) <= 5


def test_small_states_are_one_pass(qg):
    for circ in (W.config1(), W.random_circuit(9, 300, seed=2)):
        _, npass = qg.plan_passes(circ, "c128", 1)
        assert npass == 1


@pytest.mark.parametrize("bad,msg", [
    (W.CircuitBuilder(4).g2(W.CX, 2, 2).build(), "q0 == q1"),
    (W.CircuitBuilder(4).g1(W.H, 4).build(), "out of range"),
    (W.CircuitBuilder(4).g2(W.CZ, -1, 1).build(), "out of range"),
    (W.CircuitBuilder(4).add(11, -1, 0).build(), "unknown gate code"),
    (W.CircuitBuilder(4).g1(W.RY, 0, float("inf")).build(), "non-finite"),
    (W.CircuitBuilder(4).g1(W.H, 0, pidx=0).build(), "trainable"),
])
def test_validation_messages(qg, bad, msg):
    with pytest.raises(qg.QGError) as e:
        qg.plan_passes(bad)
    assert e.value.status == qg.QG_EINVAL
    assert msg in str(e.value)


def test_qubit_count_limits(qg):
    with pytest.raises(qg.QGError):
        qg.plan_passes(W.Circuit(35, np.zeros((0, 3), np.int32), np.zeros((0, 3)), np.zeros(0, np.int32)))
    with pytest.raises(qg.QGError):
        qg.plan_passes(W.Circuit(0, np.zeros((0, 3), np.int32), np.zeros((0, 3)), np.zeros(0, np.int32)))


@pytest.mark.parametrize("dtype,line_bits", [("c128", 3), ("c64", 4)])
def test_plan_kernels_pick_the_permutation_and_lane_kernels(qg, dtype, line_bits):
    """One pass per gate without fusion; the kernel of each follows the gate and where its
    qubits sit relative to the cache-line bits (2^line_bits amplitudes per 128-byte line)."""
    n = 20
    b = W.CircuitBuilder(n)
    want = []
    for t in range(n):
        b.g1(W.U3, t, 0.1, 0.2, 0.3)
        want.append("lane_gate" if t < line_bits else "tile")
        b.g1(W.RZ, t, 0.4)
        want.append("tile")
    for c, t in ((0, 1), (n - 1, 0), (1, n - 1), (8, 9), (line_bits, line_bits - 1)):
        b.g2(W.CX, c, t)
        want.append("lane_gate" if t < line_bits else "tile")
    for x, y in ((0, 1), (2, n - 1), (line_bits, n - 1), (8, 9)):
        b.g2(W.SWAP, x, y)
        want.append("swap_half" if min(x, y) >= line_bits else "swap_lane")
    circ = b.build()
    saved = {k: qg.get_tuning(k) for k in ("lane_gate", "lane_swap")}
    try:
        for k in saved:
            qg.set_tuning(k, 1)
        assert qg.plan_kernels(circ, dtype, qg.FUSE_NONE) == want
        qg.set_tuning("lane_gate", 0)
        qg.set_tuning("lane_swap", 0)
        assert qg.plan_kernels(circ, dtype, qg.FUSE_NONE) == [
            "swap_half" if w == "swap_half" else "tile" for w in want]
    finally:
        for k, v in saved.items():
            qg.set_tuning(k, v)
    # below 12 qubits every gate stays on the tile pass; fused plans match the pass count
    assert set(qg.plan_kernels(W.random_circuit(10, 50, seed=3), dtype, qg.FUSE_NONE)) == {"tile"}
    circ = W.config3(26, layers=5)
    assert len(qg.plan_kernels(circ, dtype, qg.FUSE_GREEDY)) == qg.plan_passes(circ, dtype, qg.FUSE_GREEDY)[1]


def test_plan_kernels_validates_and_reports_counts(qg):
    """qg_plan_kernels rejects what qg_plan_passes rejects, and a bad fusion mode or a negative
    capacity; with capacity 0 it only counts; an empty circuit has no passes."""
    import ctypes
    bad = W.CircuitBuilder(4).g2(W.CX, 2, 2).build()
    with pytest.raises(qg.QGError) as e:
        qg.plan_kernels(bad)
    assert e.value.status == qg.QG_EINVAL
    circ = W.random_circuit(14, 40, seed=5)
    ca = qg.CircuitArgs(circ)
    n = ctypes.c_int32(-1)
    assert qg.lib.qg_plan_kernels(ca.ptr, qg.C128, 7, None, 0, ctypes.byref(n)) == qg.QG_EINVAL
    assert qg.lib.qg_plan_kernels(ca.ptr, qg.C128, qg.FUSE_NONE, None, -1, ctypes.byref(n)) == qg.QG_EINVAL
    assert qg.lib.qg_plan_kernels(ca.ptr, qg.C128, qg.FUSE_NONE, None, 0, ctypes.byref(n)) == qg.QG_OK
    assert n.value == circ.n_gates
    k = np.full(3, -7, dtype=np.int32)
    assert qg.lib.qg_plan_kernels(ca.ptr, qg.C128, qg.FUSE_NONE, k.ctypes.data, 2, ctypes.byref(n)) == qg.QG_OK
    assert k[2] == -7 and set(k[:2]) <= set(range(len(qg.KERNEL_NAMES)))
    empty = W.Circuit(14, np.zeros((0, 3), np.int32), np.zeros((0, 3)), np.zeros(0, np.int32))
    assert qg.plan_kernels(empty) == []


@pytest.mark.parametrize("dtype,amp,tile", [("c128", 16, 12), ("c64", 8, 13)])
def test_batched_plan_bytes(qg, dtype, amp, tile):
    """Batched form's byte count: a circuit that fits one tile moves nothing; a larger one is
    filled with |0...0>, its first pass writes only the tile holding index 0, a later pass
    skips the tiles where a qubit no earlier pass held is 1 (still zero), and the observable
    reads the state once."""
    small = W.CircuitBuilder(tile)
    for q in range(tile):
        small.g1(W.H, q)
    assert qg.plan_bytes(small.build(), dtype, qg.FORM_BATCHED) == (1, 0.0)
    n = 20
    b = W.CircuitBuilder(n)
    low = tile - 5                        # the batched tile: low block plus 5 high qubits
    for q in range(low, low + 5):
        b.g1(W.H, q)                      # pass 0: tile = qubits 0 .. tile-1
    for q in range(low + 5, low + 10):
        b.g1(W.H, q)                      # pass 1: 5 new high qubits
    passes, hbm = qg.plan_bytes(b.build(), dtype, qg.FORM_BATCHED)
    state = float(amp << n)
    # the state is filled with |0...0> and read once by the observable; pass 0 writes its
    # tile 0 only (the other tiles stay zero); pass 1 visits only the tiles whose free
    # qubits above qubit low + 9 are 0: 2^(n - low - 10) of them
    unseen = n - (low + 10)
    assert passes == 2
    assert hbm == 2 * state + (amp << tile) + 2 * state / (1 << unseen)


def test_from_zero_plan_bytes(qg):
    """qg_apply_from_zero's byte count: the reset writes the state; the first pass visits only
    tile 0 (every other tile is zero); the second visits the tiles whose free qubits outside
    the first pass's tile are 0."""
    n = 20
    b = W.CircuitBuilder(n)
    for q in range(7, 17):
        b.g1(W.H, q)                          # two greedy passes: high qubits 7..11, 12..16
    circ = b.build()
    state = float(16 << n)
    passes, full = qg.plan_bytes(circ, "c128", qg.FORM_APPLY)
    assert passes == 2 and full == 4 * state
    passes, zero = qg.plan_bytes(circ, "c128", qg.FORM_FROM_ZERO)
    assert passes == 2
    assert zero == state + 2 * (16 << 12) + 2 * state / 8
