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
