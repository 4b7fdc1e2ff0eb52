"""Seeded generators: gate counts of each workload and bit-identical regeneration."""
import numpy as np

from paper_2504_03967_amd import workloads as W


def test_config_gate_counts():
    assert W.config1().n_gates == 20 * (12 + 6) == 360
    c2, p = W.config2()
    assert c2.n_gates == 4104 and p.shape == (8, 256) and c2.n_qubits == 16
    assert W.config3(31).n_gates == 5111
    assert W.config3(32).n_gates == 5344
    c5 = W.config5()
    assert c5.n_gates == 710 and c5.n_params == 480
    assert sorted(set(c5.param_idx[c5.param_idx >= 0].tolist())) == list(range(480))


def test_config4_shape_small_sample():
    circs = W.config4(n_circuits=64)
    assert len(circs) == 64
    for c in circs:
        assert 8 <= c.n_qubits <= 20
        L = c.n_gates // (3 * c.n_qubits - 1)
        assert 2 <= L <= 12 and c.n_gates == L * (3 * c.n_qubits - 1)
        assert np.all(np.abs(c.gate_param[:, 0]) <= np.pi)


def test_regeneration_is_bit_identical():
    a, b = W.config1(), W.config1()
    assert np.array_equal(a.gate_type, b.gate_type) and np.array_equal(a.gate_param, b.gate_param)
    x, y = W.config4(n_circuits=8), W.config4(n_circuits=8)
    for c, d in zip(x, y):
        assert np.array_equal(c.gate_param, d.gate_param)
    assert not np.array_equal(W.config1(seed=1).gate_param, a.gate_param)


def test_config1_cx_pairs_are_perfect_matchings():
    c = W.config1()
    cx = c.gate_type[c.gate_type[:, 0] == W.CX]
    for layer in range(20):
        qs = cx[6 * layer:6 * layer + 6, 1:].ravel()
        assert sorted(qs.tolist()) == list(range(12))


def test_config3_pairs_span_low_and_high_halves():
    n = 31
    c = W.config3(n, layers=3, with_qft=False)
    cx = c.gate_type[c.gate_type[:, 0] == W.CX][:, 1:]
    h = (n + 1) // 2
    for a, b in cx:
        assert (a < h) != (b < h)
    idx = W.config3_indices(n)
    assert idx.size == 1024 and np.unique(idx).size == 1024 and idx.max() < (1 << n)


def test_splitmix64_reference_values():
    # SplitMix64 seeded with 0: the first outputs of the generator as published with
    # Vigna's reference implementation (splitmix64.c).
    r = W.SplitMix64(0)
    assert [int(v) for v in r.next_u64(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_sweep_parts():
    prep, full, parts = W.sweep(30)
    assert prep.n_gates == 30
    names = [p[0] for p in parts]
    assert names[:30] == [f"u3_t{t}" for t in range(30)]
    assert sum(c.n_gates for _, c in parts) == full.n_gates == 30 + 15 + sum(range(2, 7)) + sum(W.SWEEP_DENSE_GATES.values())
    # the dense blocks stay on the qubits the CX / CP / SWAP pairs already entangle
    pair_qubits = {q for a, b in W.SWEEP_PAIRS for q in (a, b)}
    for name, c in parts[-2:]:
        assert name.startswith("dense_k")
        used = set(int(q) for q in c.gate_type[:, 1:].ravel() if q >= 0)
        assert used <= pair_qubits and len(used) == int(name[-1])


def test_cx_blocks_follow_the_generator():
    """Alg. 1 blocks: RY on the control, RZ on a distinct target, then CX(control -> target);
    angles in [0, 2 pi); the same seed gives the same circuit."""
    c = W.cx_blocks(12, 200, seed=3)
    assert c.n_gates == 600
    g = c.gate_type.reshape(200, 3, 3)
    assert np.all(g[:, 0, 0] == W.RY) and np.all(g[:, 1, 0] == W.RZ) and np.all(g[:, 2, 0] == W.CX)
    qc, qt = g[:, 2, 1], g[:, 2, 2]
    assert np.all(qc != qt) and np.all(g[:, 0, 2] == qc) and np.all(g[:, 1, 2] == qt)
    ang = c.gate_param.reshape(200, 3, 3)[:, :2, 0]
    assert np.all((ang >= 0) & (ang < 2 * np.pi))
    assert np.array_equal(W.cx_blocks(12, 200, seed=3).gate_param, c.gate_param)
    assert len(set(map(tuple, np.stack([qc, qt], 1)))) > 100  # pairs drawn with replacement over 132
