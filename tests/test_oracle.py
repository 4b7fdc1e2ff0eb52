"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each check uses a formulation independent of the oracle's pair loops: dense
Kronecker-product operators (eq. (tp), Lemma 1), matrix exponentials of Paulis,
the discrete Fourier transform, closed-form states, published known-answer
vectors, or brute force on tiny inputs.
"""
import math
import os

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.stats import chi2

import oracle
from paper_2504_03967_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
I2 = np.eye(2, dtype=complex)
P0 = np.array([[1, 0], [0, 0]], dtype=complex)
P1 = np.array([[0, 0], [0, 1]], dtype=complex)


def rot(P, a):
    return expm(-0.5j * a * P)


def ref_1q(op, p):
    """Single-qubit matrices from Pauli exponentials (not from the oracle's formulas)."""
    if op == W.H:
        return (PX + PZ) / math.sqrt(2)
    if op == W.X:
        return PX
    if op == W.RX:
        return rot(PX, p[0])
    if op == W.RY:
        return rot(PY, p[0])
    if op == W.RZ:
        return rot(PZ, p[0])
    if op == W.U3:  # U3(a,b,l) = e^{i(b+l)/2} RZ(b) RY(a) RZ(l)
        return np.exp(0.5j * (p[1] + p[2])) * rot(PZ, p[1]) @ rot(PY, p[0]) @ rot(PZ, p[2])
    raise ValueError(op)


def kron_op(n, factors):
    """Dense operator: factors {qubit: 2x2}; little-endian, so qubit n-1 is the leftmost factor."""
    out = np.array([[1.0 + 0j]])
    for q in range(n - 1, -1, -1):
        out = np.kron(out, factors.get(q, I2))
    return out


def dense_gate(n, op, q0, q1, p):
    if op <= W.U3:
        return kron_op(n, {q1: ref_1q(op, p)})
    if op == W.CX:
        return kron_op(n, {q0: P0}) + kron_op(n, {q0: P1, q1: PX})
    if op == W.CZ:
        return np.eye(1 << n) - 2 * kron_op(n, {q0: P1, q1: P1})
    if op == W.CP:
        return np.eye(1 << n) + (np.exp(1j * p[0]) - 1) * kron_op(n, {q0: P1, q1: P1})
    if op == W.SWAP:  # (I + XX + YY + ZZ) / 2
        return 0.5 * (np.eye(1 << n) + kron_op(n, {q0: PX, q1: PX}) + kron_op(n, {q0: PY, q1: PY})
                      + kron_op(n, {q0: PZ, q1: PZ}))
    raise ValueError(op)


def dense_circuit(circ):
    n = circ.n_qubits
    U = np.eye(1 << n, dtype=complex)
    for (op, q0, q1), p in zip(circ.gate_type, circ.gate_param):
        U = dense_gate(n, op, q0, q1, p) @ U
    return U


def oracle_matrix_1q(op, p):
    b = W.CircuitBuilder(1).add(op, -1, 0, p).build()
    cols = []
    for x in range(2):
        psi = np.zeros(2, complex)
        psi[x] = 1
        cols.append(oracle.apply(b, psi))
    return np.stack(cols, axis=1)


# ------------------------------------------------------------------ gates

@pytest.mark.parametrize("op", [W.H, W.X, W.RX, W.RY, W.RZ, W.U3])
def test_single_qubit_matrices_match_pauli_exponentials(op):
    rng = np.random.default_rng(op)
    for _ in range(5):
        p = rng.uniform(-7, 7, 3)
        M = oracle_matrix_1q(op, p)
        assert np.allclose(M, ref_1q(op, p), atol=1e-15, rtol=0)
        assert np.allclose(M.conj().T @ M, I2, atol=1e-15)


def test_gate_identities():
    pi = math.pi
    assert np.allclose(oracle_matrix_1q(W.RX, [pi, 0, 0]), -1j * PX, atol=1e-15)
    assert np.allclose(oracle_matrix_1q(W.RY, [pi, 0, 0]), -1j * PY, atol=1e-15)
    assert np.allclose(oracle_matrix_1q(W.RZ, [pi, 0, 0]), -1j * PZ, atol=1e-15)
    for a in (0.3, 1.7, -2.2):
        assert np.allclose(oracle_matrix_1q(W.U3, [a, -pi / 2, pi / 2]), oracle_matrix_1q(W.RX, [a, 0, 0]), atol=1e-15)
        assert np.allclose(oracle_matrix_1q(W.U3, [a, 0, 0]), oracle_matrix_1q(W.RY, [a, 0, 0]), atol=1e-15)
    Hm = oracle_matrix_1q(W.H, [0, 0, 0])
    assert np.allclose(Hm @ Hm, I2, atol=1e-15)
    # CP(pi) == CZ on every basis state of 2 qubits
    for x in range(4):
        a = np.zeros(4, complex); a[x] = 1
        b = a.copy()
        oracle.apply(W.CircuitBuilder(2).g2(W.CP, 0, 1, pi).build(), a)
        oracle.apply(W.CircuitBuilder(2).g2(W.CZ, 0, 1).build(), b)
        assert np.allclose(a, b, atol=1e-15)


@pytest.mark.parametrize("n", list(range(1, 9)))
def test_oracle_equals_dense_kronecker_product(n):
    """Lemma 1 / eq. (tp): every gate as an explicit 2^n x 2^n operator."""
    circ = W.random_circuit(n, 40 if n < 7 else 24, seed=1000 + n)
    U = dense_circuit(circ)
    rng = np.random.default_rng(n)
    psi0 = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi0 /= np.linalg.norm(psi0)
    got = oracle.apply(circ, psi0.copy())
    assert np.max(np.abs(got - U @ psi0)) < 1e-13
    got0 = oracle.simulate(circ)
    assert np.max(np.abs(got0 - U[:, 0])) < 1e-13


def test_all_ops_at_all_positions_n4():
    n = 4
    rng = np.random.default_rng(7)
    for op in range(10):
        for q1 in range(n):
            for q0 in (range(n) if op in W.TWO_QUBIT else [-1]):
                if q0 == q1:
                    continue
                p = rng.uniform(0, 2 * math.pi, 3)
                c = W.CircuitBuilder(n).add(op, q0, q1, p).build()
                psi0 = rng.normal(size=16) + 1j * rng.normal(size=16)
                got = oracle.apply(c, psi0.copy())
                assert np.max(np.abs(got - dense_gate(n, op, q0, q1, p) @ psi0)) < 1e-13, (op, q0, q1)


def test_cx_worked_example():
    """App. A: CX with control q0 and target q2 on 3 qubits exchanges exactly the listed pairs."""
    pairs = []
    for line in open(os.path.join(GOLDEN, "cx_worked_example.txt")):
        if line.strip() and not line.startswith("#"):
            ka, kb = line.split()
            idx = lambda k: sum(int(ch) << q for q, ch in enumerate(k))  # ket q0 q1 q2
            pairs.append((idx(ka), idx(kb)))
    assert sorted(pairs) == [(1, 5), (3, 7)]
    psi = (np.arange(8) + 1) * (1 + 0.5j)
    before = psi.copy()
    oracle.apply(W.CircuitBuilder(3).g2(W.CX, 0, 2).build(), psi)
    expect = before.copy()
    for a, b in pairs:
        expect[a], expect[b] = before[b], before[a]
    assert np.array_equal(psi, expect)


# --------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", list(range(1, 9)))
def test_qft_closed_form_all_basis_states(n):
    circ = W.qft(n).build()
    N = 1 << n
    k = np.arange(N)
    for x in range(N):
        psi = np.zeros(N, complex); psi[x] = 1
        oracle.apply(circ, psi)
        expect = np.exp(2j * np.pi * x * k / N) / math.sqrt(N)
        assert np.max(np.abs(psi - expect)) < 1e-13


def test_qft_matches_inverse_dft_random_state():
    n = 12
    rng = np.random.default_rng(3)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    got = oracle.apply(W.qft(n).build(), psi.copy())
    assert np.max(np.abs(got - np.fft.ifft(psi) * math.sqrt(1 << n))) < 1e-13


@pytest.mark.parametrize("n", [2, 5, 13, 18])
def test_ghz_and_uniform(n):
    psi = oracle.simulate(W.ghz(n))
    p = oracle.probs(psi)
    assert abs(p[0] - 0.5) < 1e-13 and abs(p[-1] - 0.5) < 1e-13
    assert abs(p[1:-1].sum()) < 1e-13
    masks = [(1 << i) | (1 << j) for i in range(n) for j in range(i + 1, n)][:20] + [1 << i for i in range(n)]
    ev = oracle.expval(psi, masks)
    nzz = min(20, n * (n - 1) // 2)
    assert np.allclose(ev[:nzz], 1, atol=1e-13) and np.allclose(ev[nzz:], 0, atol=1e-13)
    u = oracle.simulate(W.uniform_superposition(n))
    assert np.max(np.abs(u - 2 ** (-n / 2))) < 1e-13
    assert np.allclose(oracle.expval(u, [1, 3, (1 << n) - 1]), 0, atol=1e-13)


def test_norm_conservation_random_circuits():
    for n in (10, 13):
        psi = oracle.simulate(W.random_circuit(n, 400, seed=77 + n))
        assert abs(np.sum(oracle.probs(psi)) - 1) < 1e-13


def test_mirror_circuit_returns_to_zero():
    circ = W.config3(10, layers=6)
    full = W.concat(circ, W.inverse(circ))
    psi = oracle.simulate(full)
    assert abs(psi[0] - 1) < 1e-12 and np.max(np.abs(psi[1:])) < 1e-12


def test_qcrank_closed_form_config2():
    """Uniformly controlled RY: alpha(a, data) = 2^{-m/2} prod_d (sqrt p or sqrt(1-p))."""
    circ, p = W.config2()
    assert circ.n_gates == 4104
    assert int((circ.gate_type[:, 0] == W.CX).sum()) == 8 * 256  # #CX = #pixels (Table 2)
    psi = oracle.simulate(circ)
    m, nd = 8, 8
    a = np.arange(1 << 16) & 0xFF
    amp = np.full(1 << 16, 2 ** (-m / 2), dtype=float)
    for d in range(nd):
        bit = (np.arange(1 << 16) >> (m + d)) & 1
        amp *= np.where(bit == 0, np.sqrt(p[d, a]), np.sqrt(1 - p[d, a]))
    assert np.max(np.abs(psi - amp)) < 1e-12


def test_expval_pins():
    n = 6
    for x in (0, 5, 37, 63):
        psi = np.zeros(1 << n, complex); psi[x] = 1
        masks = np.arange(1 << n, dtype=np.uint64)
        ev = oracle.expval(psi, masks)
        expect = np.array([(-1) ** bin(x & m).count("1") for m in range(1 << n)], float)
        assert np.array_equal(ev, expect)
    # random state against dense Z-string operators
    rng = np.random.default_rng(11)
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi /= np.linalg.norm(psi)
    for m in (1, 6, 33, 63):
        Zm = kron_op(n, {q: PZ for q in range(n) if (m >> q) & 1})
        assert abs(oracle.expval(psi, [m])[0] - np.vdot(psi, Zm @ psi).real) < 1e-14


def test_batch_zz_chain_closed_forms():
    """The oracle's batched entry (independent circuits side by side) on circuits whose open-
    chain sum_q <Z_q Z_{q+1}> is known in closed form: GHZ (every term 1), basis states
    (term q is (-1)^{x_q xor x_{q+1}}), the uniform superposition (every term 0), and a dense
    Z Z operator on a random 4-qubit circuit."""
    circs, expect = [], []
    for n in (1, 2, 7, 12):
        circs.append(W.ghz(n))
        expect.append(n - 1)
    for n, x in ((5, 0b10110), (9, 0b101010101), (3, 0b111)):
        b = W.CircuitBuilder(n)
        for q in range(n):
            if (x >> q) & 1:
                b.g1(W.X, q)
        circs.append(b.build())
        expect.append(sum((-1) ** (((x >> q) ^ (x >> (q + 1))) & 1) for q in range(n - 1)))
    circs.append(W.uniform_superposition(10))
    expect.append(0.0)
    r = W.random_circuit(4, 60, seed=8)
    psi = dense_circuit(r)[:, 0]
    zz = sum(kron_op(4, {q: PZ, q + 1: PZ}) for q in range(3))
    circs.append(r)
    expect.append(np.vdot(psi, zz @ psi).real)
    got = oracle.batch_zz_chain(circs)
    assert np.max(np.abs(got - np.array(expect, float))) < 1e-13


# --------------------------------------------------------------- sampling

def test_philox_known_answer_vectors():
    for line in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(v, 16) for v in line.split()]
        assert list(oracle.philox4x32_10(w[0:4], w[4:6])) == w[6:10]


def test_sampler_is_inverse_cdf_of_shot_uniforms():
    rng = np.random.default_rng(5)
    n = 6
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    psi[[3, 17, 40]] = 0
    psi /= np.linalg.norm(psi)
    seed = 0xC0FFEE
    shots = oracle.sample(psi, 3000, seed)
    p = np.abs(psi) ** 2
    cdf = np.cumsum(p)
    u = np.array([oracle.shot_uniform(seed, s) for s in range(3000)])
    expect = np.searchsorted(cdf, u * cdf[-1], side="right")
    assert np.array_equal(shots, expect.astype(np.uint64))
    assert not np.isin(shots, [3, 17, 40]).any()
    # uniforms are in [0, 1) and well spread
    assert u.min() >= 0 and u.max() < 1 and abs(u.mean() - 0.5) < 0.02


def chi_square_p(counts, p, shots):
    """Merge consecutive outcomes until the expected count reaches 5; X^2 with bins-1 dof."""
    obs, exp_ = [], []
    o = e = 0.0
    for c, pi in zip(counts, p):
        o += c; e += pi * shots
        if e >= 5:
            obs.append(o); exp_.append(e); o = e = 0.0
    if e > 0 and obs:
        obs[-1] += o; exp_[-1] += e
    obs, exp_ = np.array(obs), np.array(exp_)
    x2 = np.sum((obs - exp_) ** 2 / exp_)
    return chi2.sf(x2, len(obs) - 1)


def test_sampler_chi_square():
    psi = oracle.simulate(W.random_circuit(10, 200, seed=99))
    p = oracle.probs(psi)
    shots = 200000
    s = oracle.sample(psi, shots, seed=12345)
    counts = np.bincount(s.astype(np.int64), minlength=p.size)
    assert chi_square_p(counts, p, shots) > 0.01


def test_sampler_degenerate_basis_state():
    psi = np.zeros(16, complex); psi[9] = 1
    assert np.all(oracle.sample(psi, 500, 1) == 9)


# ---------------------------------------------------------------- adjoint

def f_value(circ, masks, coeffs):
    psi = oracle.simulate(circ)
    return float(np.dot(coeffs, oracle.expval(psi, masks)))


def trainable_circuit(n, layers, seed):
    rng = W.SplitMix64(seed)
    b = W.CircuitBuilder(n)
    k = 0
    for _ in range(layers):
        for q in range(n):
            op = [W.RX, W.RY, W.RZ][int(rng.below(3)[0])]
            b.g1(op, q, float(rng.uniform(1)[0]) * 6.28, pidx=k); k += 1
        b.g1(W.H, int(rng.below(n)[0]))
        b.g1(W.U3, int(rng.below(n)[0]), *(6.28 * rng.uniform(3)))
        for q in range(n - 1):
            b.g2(W.CX, q, q + 1)
        b.g2(W.CP, 0, n - 1, float(rng.uniform(1)[0]) * 6.28, pidx=k); k += 1
        b.g2(W.SWAP, 0, 1)
        b.g2(W.CZ, 0, 2)
    return b.build(), k


@pytest.mark.parametrize("n", [3, 6])
def test_adjoint_matches_parameter_shift_and_fd(n):
    circ, npar = trainable_circuit(n, 3, seed=40 + n)
    masks = W.zz_chain_masks(n)
    coeffs = np.linspace(0.5, 1.5, masks.size)
    val, grad = oracle.adjoint_grad(circ, npar, masks, coeffs)
    assert abs(val - f_value(circ, masks, coeffs)) < 1e-13
    for k in range(npar):
        (g_idx,) = np.nonzero(circ.param_idx == k)
        plus, minus = circ.copy(), circ.copy()
        plus.gate_param[g_idx, 0] += math.pi / 2
        minus.gate_param[g_idx, 0] -= math.pi / 2
        shift = 0.5 * (f_value(plus, masks, coeffs) - f_value(minus, masks, coeffs))
        assert abs(grad[k] - shift) < 1e-10, k
        h = 1e-6
        plus.gate_param[g_idx, 0] += h - math.pi / 2
        minus.gate_param[g_idx, 0] -= h - math.pi / 2
        fd = (f_value(plus, masks, coeffs) - f_value(minus, masks, coeffs)) / (2 * h)
        assert abs(grad[k] - fd) < 1e-6, k


def test_adjoint_shared_parameter_slot_accumulates():
    n = 3
    b = W.CircuitBuilder(n)
    b.g1(W.RY, 0, 0.4, pidx=0).g1(W.RY, 1, 0.4, pidx=0).g2(W.CX, 0, 1).g1(W.RX, 2, 1.1, pidx=1)
    circ = b.build()
    masks = np.array([3, 6], np.uint64)
    coeffs = np.array([1.0, -0.7])
    _, grad = oracle.adjoint_grad(circ, 2, masks, coeffs)
    h = 1e-6
    plus, minus = circ.copy(), circ.copy()
    plus.gate_param[[0, 1], 0] += h
    minus.gate_param[[0, 1], 0] -= h
    fd = (f_value(plus, masks, coeffs) - f_value(minus, masks, coeffs)) / (2 * h)
    assert abs(grad[0] - fd) < 1e-7


def test_oracle_rejects_malformed_gates():
    bad = W.CircuitBuilder(3).g2(W.CX, 1, 1).build()
    with pytest.raises(ValueError):
        oracle.simulate(bad)
    bad = W.CircuitBuilder(3).g1(W.H, 3).build()
    with pytest.raises(ValueError):
        oracle.simulate(bad)
