"""The paper's benchmark workloads at its own shapes, on the GPU path against the oracle and
closed forms: QCrank image encoding at Table 2's address/data splits with 3000 * 2^m shots
(App. D.3), the approximate QFT (rotation-angle pruning, App. D.2), and a long random
CX-block unitary (10,000 blocks of Alg. 1)."""
import math

import numpy as np
import pytest
import torch
from scipy.stats import binom

import oracle
from paper_2504_03967_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}
# Table 2: (address qubits m, data qubits); shots 3000 * 2^m
TABLE2 = [(10, 5), (11, 8), (12, 6), (13, 12), (14, 6), (15, 3)]


@pytest.fixture(scope="module")
def qg():
    from paper_2504_03967_amd import qg as lib
    assert torch.cuda.is_available()
    return lib


@pytest.fixture(autouse=True)
def free_memory():
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def qcrank_closed_form(p, m):
    """alpha(a, data bits) = 2^{-m/2} prod_d (sqrt p[d, a] if bit d = 0 else sqrt(1 - p[d, a]))."""
    nd = p.shape[0]
    i = np.arange(1 << (m + nd), dtype=np.int64)
    a = i & ((1 << m) - 1)
    amp = np.full(i.size, 2.0 ** (-m / 2))
    for d in range(nd):
        bit = (i >> (m + d)) & 1
        amp *= np.where(bit == 0, np.sqrt(p[d, a]), np.sqrt(1.0 - p[d, a]))
    return amp


@pytest.mark.parametrize("m,nd", TABLE2)
def test_qcrank_table2_shapes(qg, m, nd):
    """Every amplitude against the closed-form encoded state (and against the oracle where it
    finishes in seconds); then 3000 * 2^m shots: each pixel's estimate
    p_hat(d, a) = counts(a, d = 0) / counts(a) must be a plausible binomial draw around p
    (two-sided tail probability above 1e-9 / pixels, a Bonferroni bound)."""
    circ, p = W.config2(seed=W.SEED_BASE + 20 + m, n_addr=m, n_data=nd)
    n = m + nd
    assert int((circ.gate_type[:, 0] == W.CX).sum()) == nd << m  # #CX = #pixels
    st = qg.State(n, "c128")
    st.apply(circ, qg.FUSE_GREEDY)
    torch.cuda.synchronize()
    got = st.tensor.cpu().numpy()
    assert np.max(np.abs(got - qcrank_closed_form(p, m))) < TOL["c128"]
    if circ.n_gates * (1 << n) <= 2e10:
        assert np.max(np.abs(got - oracle.simulate(circ))) < TOL["c128"]
    del got
    shots = st.sample(3000 << m, W.SEED_BASE + m).cpu().numpy()
    st.close()
    addr = shots & ((1 << m) - 1)
    n_a = np.bincount(addr, minlength=1 << m)
    assert n_a.sum() == 3000 << m
    worst = 1.0
    for d in range(nd):
        zero = ((shots >> (m + d)) & 1) == 0
        n0 = np.bincount(addr[zero], minlength=1 << m)
        lo = binom.cdf(n0, n_a, p[d])
        hi = binom.sf(n0 - 1, n_a, p[d])
        worst = min(worst, float(np.min(2 * np.minimum(lo, hi))))
    assert worst > 1e-9 / (nd << m), worst


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("eps", [0.0, math.pi / 2 ** 4, math.pi / 2 ** 9])
def test_approximate_qft_matches_oracle(qg, dtype, eps):
    """QFT with its small rotations pruned (|lambda| < eps), after a random U3 layer: the GPU
    applies the pruned gate list, the oracle the same list."""
    n = 18
    rng = W.SplitMix64(W.SEED_BASE + 30)
    b = W.CircuitBuilder(n)
    for q in range(n):
        b.g1(W.U3, q, *(2 * math.pi * rng.uniform(3)))
    exact = W.concat(b.build(), W.qft(n).build())
    circ = W.prune_small_rotations(exact, eps)
    dropped = exact.n_gates - circ.n_gates
    assert dropped == (0 if eps == 0 else sum(n - d for d in range(1, n) if math.pi / 2 ** d < eps))
    st = qg.State(n, dtype)
    st.apply(circ, qg.FUSE_GREEDY)
    torch.cuda.synchronize()
    got = st.tensor.cpu().numpy().astype(np.complex128)
    st.close()
    assert np.max(np.abs(got - oracle.simulate(circ))) < TOL[dtype]


def test_long_cx_block_unitary(qg):
    """10,000 CX blocks of Alg. 1 (30,000 gates) on 22 qubits, both precisions, every amplitude
    against the oracle; then 3000 shots, >= 99.9 % identical to the oracle's draws."""
    n = 22
    circ = W.cx_blocks(n, 10000, W.SEED_BASE + 50)
    psi = oracle.simulate(circ)
    for dtype in ("c128", "c64"):
        st = qg.State(n, dtype)
        st.apply(circ, qg.FUSE_GREEDY)
        torch.cuda.synchronize()
        got = st.tensor.cpu().numpy().astype(np.complex128)
        assert np.max(np.abs(got - psi)) < TOL[dtype], dtype
        if dtype == "c128":
            shots = st.sample(3000, W.SEED_BASE + 51).cpu().numpy().astype(np.uint64)
            assert np.mean(shots == oracle.sample(psi, 3000, W.SEED_BASE + 51)) >= 0.999
        st.close()
