"""Seeded synthetic circuit generators (the inputs both the GPU path and the oracle consume).

This module holds no simulation arithmetic: it only draws random numbers and
writes gate lists in the circuit encoding of Sec. 2.1 / App. B (one row per gate:
``gate_type = {code, q0, q1}``, ``gate_param = {theta, phi, lambda}``, padded
per Lemma 2 when circuits are batched).  Randomness comes from SplitMix64
(Steele, Lea & Flood, OOPSLA 2014), one stream per workload, in a fixed draw order
that each generator documents.

Workloads (shapes of the paper's experiments, Table 1 and App. D):
  * ``config1``  -- 12 qubits, 20 layers of U3 on every qubit + 6 CX on a random
    perfect matching (random entangling blocks in the spirit of Alg. 1).
  * ``config2``  -- QCrank-style uniformly controlled RY image encoding (App. D.3,
    Table 2): 8 address + 8 data qubits, Gray-code CX order, synthetic pixels.
  * ``config3``  -- 100 random U3 + low/high CX layers followed by an exact QFT
    (App. D.2) on 31 (c128) or 32 (c64) qubits.
  * ``config4``  -- 4096 hardware-efficient ansatz circuits (RY, RZ, CX ladder),
    8..20 qubits, 2..12 layers.
  * ``config5``  -- the same ansatz at 24 qubits, 10 layers, 480 trainable angles.
  * ``sweep``    -- the 30-qubit gate sweep used for the HBM roofline figure.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

# Gate codes of the circuit encoding.
H, X, RX, RY, RZ, U3, CX, CZ, CP, SWAP = range(10)
GATE_NAMES = ("h", "x", "rx", "ry", "rz", "u3", "cx", "cz", "cp", "swap")
TWO_QUBIT = (CX, CZ, CP, SWAP)

SEED_BASE = 250403967

_MASK64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


@dataclasses.dataclass
class Circuit:
    """One circuit: ``gate_type`` int32 [G,3], ``gate_param`` float64 [G,3], ``param_idx`` int32 [G]."""

    n_qubits: int
    gate_type: np.ndarray
    gate_param: np.ndarray
    param_idx: np.ndarray

    @property
    def n_gates(self) -> int:
        return int(self.gate_type.shape[0])

    @property
    def n_params(self) -> int:
        return int(self.param_idx.max()) + 1 if self.param_idx.size and self.param_idx.max() >= 0 else 0

    def copy(self) -> "Circuit":
        return Circuit(self.n_qubits, self.gate_type.copy(), self.gate_param.copy(), self.param_idx.copy())


class CircuitBuilder:
    def __init__(self, n: int):
        self.n = n
        self.rows: List[Tuple[int, int, int]] = []
        self.params: List[Tuple[float, float, float]] = []
        self.pidx: List[int] = []

    def add(self, op: int, q0: int, q1: int, p=(0.0, 0.0, 0.0), pidx: int = -1) -> "CircuitBuilder":
        p = tuple(float(v) for v in p) + (0.0,) * (3 - len(p))
        self.rows.append((int(op), int(q0), int(q1)))
        self.params.append(p)
        self.pidx.append(int(pidx))
        return self

    def g1(self, op: int, t: int, *p, pidx: int = -1) -> "CircuitBuilder":
        return self.add(op, -1, t, p, pidx)

    def g2(self, op: int, a: int, b: int, *p, pidx: int = -1) -> "CircuitBuilder":
        return self.add(op, a, b, p, pidx)

    def build(self) -> Circuit:
        g = len(self.rows)
        gt = np.array(self.rows, dtype=np.int32).reshape(g, 3)
        gp = np.array(self.params, dtype=np.float64).reshape(g, 3)
        pi = np.array(self.pidx, dtype=np.int32).reshape(g)
        return Circuit(self.n, gt, gp, pi)


def concat(a: Circuit, b: Circuit) -> Circuit:
    assert a.n_qubits == b.n_qubits
    return Circuit(a.n_qubits, np.concatenate([a.gate_type, b.gate_type]),
                   np.concatenate([a.gate_param, b.gate_param]),
                   np.concatenate([a.param_idx, b.param_idx]))


class SplitMix64:
    """SplitMix64: state += 0x9E3779B97F4A7C15, then the 30/27/31 xor-shift-multiply finaliser."""

    def __init__(self, seed: int):
        self.state = int(seed) & _MASK64

    def next_u64(self, k: int) -> np.ndarray:
        k = int(k)
        idx = np.arange(1, k + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = np.uint64(self.state) + idx * np.uint64(_GAMMA)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
        self.state = (self.state + k * _GAMMA) & _MASK64
        return z

    def uniform(self, k: int) -> np.ndarray:
        """k doubles in [0, 1): the top 53 bits of each draw times 2^-53."""
        return (self.next_u64(k) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def below(self, m: int, k: int = 1) -> np.ndarray:
        """k integers in [0, m) (draw modulo m)."""
        return (self.next_u64(k) % np.uint64(m)).astype(np.int64)

    def shuffle(self, seq: Sequence[int]) -> List[int]:
        """Fisher-Yates: for i = len-1 down to 1 swap item i with item (draw mod (i+1))."""
        out = list(seq)
        for i in range(len(out) - 1, 0, -1):
            j = int(self.below(i + 1)[0])
            out[i], out[j] = out[j], out[i]
        return out


# ----------------------------------------------------------------- circuits

def qft(n: int, builder: CircuitBuilder | None = None) -> CircuitBuilder:
    """Exact QFT (App. D.2 and eq. (cr1)): for i = n-1 down to 0, H(i) then CP(pi / 2^(i-j))
    on (j, i) for j = i-1 down to 0; then SWAP(i, n-1-i) for i < n/2.  Maps |x> to
    2^(-n/2) sum_k e^{+2 pi i x k / 2^n} |k>.  The paper's first qubit is our qubit n-1."""
    b = builder or CircuitBuilder(n)
    for i in range(n - 1, -1, -1):
        b.g1(H, i)
        for j in range(i - 1, -1, -1):
            b.g2(CP, j, i, math.pi / (1 << (i - j)))
    for i in range(n // 2):
        b.g2(SWAP, i, n - 1 - i)
    return b


def ghz(n: int) -> Circuit:
    b = CircuitBuilder(n).g1(H, 0)
    for q in range(n - 1):
        b.g2(CX, q, q + 1)
    return b.build()


def uniform_superposition(n: int) -> Circuit:
    b = CircuitBuilder(n)
    for q in range(n):
        b.g1(H, q)
    return b.build()


def cx_blocks(n: int, blocks: int, seed: int) -> Circuit:
    """Random CX-block unitary (the workload of the paper's Alg. 1, App. D.1): every block is
    an RY on a control qubit and an RZ on a different target qubit, angles uniform in
    [0, 2 pi), then CX(control -> target).  The ordered (control, target) pair is uniform over
    the n (n - 1) pairs of distinct qubits: one draw k below n (n - 1), control k // (n - 1),
    target the (k mod (n - 1))-th qubit other than the control.  Draw order per block: k, RY
    angle, RZ angle."""
    rng = SplitMix64(seed)
    b = CircuitBuilder(n)
    for _ in range(blocks):
        k = int(rng.below(n * (n - 1))[0])
        qc, r = divmod(k, n - 1)
        qt = r if r < qc else r + 1
        b.g1(RY, qc, float(2 * math.pi * rng.uniform(1)[0]))
        b.g1(RZ, qt, float(2 * math.pi * rng.uniform(1)[0]))
        b.g2(CX, qc, qt)
    return b.build()


def prune_small_rotations(circ: Circuit, eps: float) -> Circuit:
    """Approximate form of a circuit (the rotation-angle approximation of App. D.2, whose
    threshold the paper leaves open): every CP whose angle, taken in (-pi, pi], has magnitude
    below ``eps`` is dropped; everything else is kept in order.  eps = 0 keeps every gate."""
    lam = np.remainder(circ.gate_param[:, 0] + math.pi, 2 * math.pi) - math.pi
    keep = ~((circ.gate_type[:, 0] == CP) & (np.abs(lam) < eps))
    return Circuit(circ.n_qubits, circ.gate_type[keep].copy(), circ.gate_param[keep].copy(),
                   circ.param_idx[keep].copy())


def random_circuit(n: int, n_gates: int, seed: int, ops: Sequence[int] = tuple(range(10))) -> Circuit:
    """Random gates over ``ops`` on random qubits (a generalisation of Alg. 1: the second
    qubit is redrawn until it differs from the first).  Draw order per gate: op, q1,
    then q0 (redrawn while equal to q1) for two-qubit ops, then three angles in [0, 2 pi)."""
    rng = SplitMix64(seed)
    b = CircuitBuilder(n)
    ops = [o for o in ops if n >= 2 or o not in TWO_QUBIT]
    for _ in range(n_gates):
        op = ops[int(rng.below(len(ops))[0])]
        q1 = int(rng.below(n)[0])
        q0 = -1
        if op in TWO_QUBIT:
            q0 = int(rng.below(n)[0])
            while q0 == q1:
                q0 = int(rng.below(n)[0])
        ang = 2 * math.pi * rng.uniform(3)
        b.add(op, q0, q1, ang)
    return b.build()


def inverse(circ: Circuit) -> Circuit:
    """The gate list of U^dagger: reversed order, each gate replaced by its inverse
    (U3(a,b,l)^dag = U3(-a,-l,-b); rotations and CP negate their angle; H, X, CX, CZ
    and SWAP are their own inverses)."""
    gt = circ.gate_type[::-1].copy()
    gp = circ.gate_param[::-1].copy()
    for g in range(gt.shape[0]):
        op = gt[g, 0]
        if op in (RX, RY, RZ, CP):
            gp[g, 0] = -gp[g, 0]
        elif op == U3:
            a, b_, l = gp[g]
            gp[g] = (-a, -l, -b_)
    return Circuit(circ.n_qubits, gt, gp, np.full(gt.shape[0], -1, np.int32))


def config1(seed: int = SEED_BASE + 0, n: int = 12, layers: int = 20) -> Circuit:
    """Per layer: U3 on qubits 0..n-1 (theta, phi, lambda drawn in that order, each 2 pi u),
    then a Fisher-Yates shuffle of the qubits paired consecutively; first of each pair
    controls a CX on the second."""
    rng = SplitMix64(seed)
    b = CircuitBuilder(n)
    for _ in range(layers):
        ang = 2 * math.pi * rng.uniform(3 * n)
        for q in range(n):
            b.g1(U3, q, *ang[3 * q:3 * q + 3])
        perm = rng.shuffle(range(n))
        for k in range(n // 2):
            b.g2(CX, perm[2 * k], perm[2 * k + 1])
    return b.build()


def gray(j: int) -> int:
    return j ^ (j >> 1)


def config2(seed: int = SEED_BASE + 1, n_addr: int = 8, n_data: int = 8) -> Tuple[Circuit, np.ndarray]:
    """QCrank-style encoding (App. D.3): H on address qubits 0..m-1; for each data qubit d
    (qubit m+d) a uniformly controlled RY realised as 2^m x (RY(phi_{d,j}), CX from the
    address bit where gray(j) and gray(j+1 mod 2^m) differ).  Synthetic pixels
    p[d, a] ~ U[0,1] (drawn d-major) stand in for the images; the multiplexed angle for
    address a is theta = 2 arccos(sqrt(p)), so that P(data_d = 0 | a) = p[d, a], and
    phi_{d,j} = 2^-m sum_a (-1)^{popcount(a & gray(j))} theta_{d,a} (Walsh-Gray transform).
    Returns (circuit, p)."""
    rng = SplitMix64(seed)
    m = n_addr
    na = 1 << m
    p = rng.uniform(n_data * na).reshape(n_data, na)
    theta = 2.0 * np.arccos(np.sqrt(p))
    # Walsh transform over the address bits (butterflies), then read at gray(j).
    wt = theta.copy()
    h = 1
    while h < na:
        v = wt.reshape(n_data, na // (2 * h), 2, h)
        v[:, :, 0, :], v[:, :, 1, :] = v[:, :, 0, :] + v[:, :, 1, :], v[:, :, 0, :] - v[:, :, 1, :]
        h *= 2
    j = np.arange(na)
    gj = j ^ (j >> 1)
    phi = wt[:, gj] / na  # [d, j]
    # control of the CX after step j: the address bit where gray(j) and gray(j + 1 mod 2^m) differ
    diff = gj ^ np.roll(gj, -1)
    ctrl = np.floor(np.log2(diff)).astype(np.int32)
    G = m + 2 * n_data * na
    gt = np.zeros((G, 3), dtype=np.int32)
    gp = np.zeros((G, 3), dtype=np.float64)
    gt[:m, 0], gt[:m, 1], gt[:m, 2] = H, -1, np.arange(m)
    body_t = gt[m:].reshape(n_data, na, 2, 3)
    body_p = gp[m:].reshape(n_data, na, 2, 3)
    tgt = (m + np.arange(n_data))[:, None]
    body_t[:, :, 0, 0], body_t[:, :, 0, 1], body_t[:, :, 0, 2] = RY, -1, tgt
    body_p[:, :, 0, 0] = phi
    body_t[:, :, 1, 0], body_t[:, :, 1, 1], body_t[:, :, 1, 2] = CX, ctrl[None, :], tgt
    return Circuit(m + n_data, gt, gp, np.full(G, -1, np.int32)), p


def config3(n: int, seed: int | None = None, layers: int = 100, with_qft: bool = True) -> Circuit:
    """Per layer: U3 on qubits 0..n-1 (3 angles each in [0, 2 pi)); then floor(n/2) CX
    pairing a Fisher-Yates shuffle of the low half {0..ceil(n/2)-1} with the high half in
    order, direction drawn per pair (draw 1: low qubit controls).  Then the exact QFT(n)."""
    seed = SEED_BASE + 2 if seed is None else seed
    rng = SplitMix64(seed)
    h = (n + 1) // 2
    b = CircuitBuilder(n)
    for _ in range(layers):
        ang = 2 * math.pi * rng.uniform(3 * n)
        for q in range(n):
            b.g1(U3, q, *ang[3 * q:3 * q + 3])
        low = rng.shuffle(range(h))
        dirs = rng.below(2, n // 2)
        for k in range(n // 2):
            lo, hi = low[k], h + k
            if dirs[k]:
                b.g2(CX, lo, hi)
            else:
                b.g2(CX, hi, lo)
    if with_qft:
        qft(n, b)
    return b.build()


def config3_indices(n: int, seed: int | None = None, count: int = 1024) -> np.ndarray:
    """``count`` distinct basis states of [0, 2^n) in draw order (duplicates redrawn)."""
    seed = SEED_BASE + 2 if seed is None else seed
    rng = SplitMix64(seed ^ 0x5EED1D5)
    seen, out = set(), []
    while len(out) < count:
        v = int(rng.next_u64(1)[0] % np.uint64(1 << n))
        if v not in seen:
            seen.add(v)
            out.append(v)
    return np.array(out, dtype=np.uint64)


def ansatz(n: int, angles: np.ndarray, layers: int, trainable: bool = True) -> Circuit:
    """Hardware-efficient ansatz: per layer RY(q) for q = 0..n-1, RZ(q) for q = 0..n-1, then
    CX(q, q+1) for q = 0..n-2.  ``angles`` is layer-major [layers, 2, n]; parameter slot of
    RY(l, q) is 2 n l + q and of RZ(l, q) is 2 n l + n + q."""
    a = np.asarray(angles, dtype=np.float64).reshape(layers, 2, n)
    b = CircuitBuilder(n)
    for l in range(layers):
        for q in range(n):
            b.g1(RY, q, a[l, 0, q], pidx=(2 * n * l + q) if trainable else -1)
        for q in range(n):
            b.g1(RZ, q, a[l, 1, q], pidx=(2 * n * l + n + q) if trainable else -1)
        for q in range(n - 1):
            b.g2(CX, q, q + 1)
    return b.build()


def zz_chain_masks(n: int) -> np.ndarray:
    """Masks of Z_i Z_{i+1}, i = 0..n-2 (open chain)."""
    return np.array([(1 << i) | (1 << (i + 1)) for i in range(n - 1)], dtype=np.uint64)


def config4(seed: int = SEED_BASE + 3, n_circuits: int = 4096, n_min: int = 8, n_max: int = 20,
            l_min: int = 2, l_max: int = 12) -> List[Circuit]:
    """Per circuit: n = n_min + draw mod (n_max-n_min+1), L = l_min + draw mod (l_max-l_min+1),
    then 2 n L angles -pi + 2 pi u (layer-major, RY block before RZ block)."""
    rng = SplitMix64(seed)
    out = []
    for _ in range(n_circuits):
        n = n_min + int(rng.below(n_max - n_min + 1)[0])
        L = l_min + int(rng.below(l_max - l_min + 1)[0])
        ang = -math.pi + 2 * math.pi * rng.uniform(2 * n * L)
        out.append(ansatz(n, ang, L, trainable=False))
    return out


def config5(seed: int = SEED_BASE + 4, n: int = 24, layers: int = 10) -> Circuit:
    """24-qubit, 10-layer ansatz with 480 trainable angles -pi + 2 pi u."""
    rng = SplitMix64(seed)
    ang = -math.pi + 2 * math.pi * rng.uniform(2 * n * layers)
    return ansatz(n, ang, layers, trainable=True)


SWEEP_PAIRS = ((0, 1), (1, 29), (29, 0), (15, 16), (28, 29))
SWEEP_DENSE_GATES = {5: 48, 6: 64}


def sweep(n: int = 30, seed: int = SEED_BASE + 0) -> Tuple[Circuit, Circuit, List[Tuple[str, Circuit]]]:
    """Gate sweep on an n-qubit state: (prep, full, parts).  ``prep`` is one layer of random
    U3 on every qubit; ``parts`` are the timed pieces: U3 on each target t = 0..n-1, then
    CX, CP and SWAP on each pair of ``SWEEP_PAIRS`` (scaled into range for n < 30), then
    a k-gate group of U3 on k distinct random qubits for k = 2..6, then blocks of
    SWEEP_DENSE_GATES[k] random gates on k = 5 and 6 of the pair qubits (dense-block passes).
    ``full`` concatenates the parts."""
    rng = SplitMix64(seed)
    pb = CircuitBuilder(n)
    ang = 2 * math.pi * rng.uniform(3 * n)
    for q in range(n):
        pb.g1(U3, q, *ang[3 * q:3 * q + 3])
    prep = pb.build()
    parts = []
    for t in range(n):
        a = 2 * math.pi * rng.uniform(3)
        parts.append((f"u3_t{t}", CircuitBuilder(n).g1(U3, t, *a).build()))
    pairs = [(a % n, b % n) for a, b in SWEEP_PAIRS]
    pairs = [(a, b) if a != b else (a, (a + 1) % n) for a, b in pairs]
    for a, b in pairs:
        parts.append((f"cx_{a}_{b}", CircuitBuilder(n).g2(CX, a, b).build()))
    for a, b in pairs:
        lam = 2 * math.pi * float(rng.uniform(1)[0])
        parts.append((f"cp_{a}_{b}", CircuitBuilder(n).g2(CP, a, b, lam).build()))
    for a, b in pairs:
        parts.append((f"swap_{a}_{b}", CircuitBuilder(n).g2(SWAP, a, b).build()))
    for k in range(2, 7):
        qs = rng.shuffle(range(n))[:k]
        cb = CircuitBuilder(n)
        for q in qs:
            cb.g1(U3, q, *(2 * math.pi * rng.uniform(3)))
        parts.append((f"fused_k{k}", cb.build()))
    # dense blocks: SWEEP_DENSE_GATES[k] random gates (all ten ops) on k = 5 and 6 of
    # the qubits the pairs above already entangle
    ent = sorted({q for ab in pairs for q in ab})
    for k in (5, 6):
        qs = ent[:k] if k < len(ent) else ent
        cb = CircuitBuilder(n)
        for _ in range(SWEEP_DENSE_GATES[k]):
            op = int(rng.below(10)[0])
            t = qs[int(rng.below(len(qs))[0])]
            c = -1
            if op in TWO_QUBIT:
                c = qs[int(rng.below(len(qs))[0])]
                while c == t:
                    c = qs[int(rng.below(len(qs))[0])]
            cb.add(op, c, t, 2 * math.pi * rng.uniform(3))
        parts.append((f"dense_k{k}", cb.build()))
    full = parts[0][1]
    for _, c in parts[1:]:
        full = concat(full, c)
    return prep, full, parts


def amp_updates(circ: Circuit) -> int:
    """Amplitude updates the paper's cost model counts: 2^n per gate (App. A)."""
    return circ.n_gates << circ.n_qubits
