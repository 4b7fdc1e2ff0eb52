"""Dense k-qubit blocks on the matrix cores against the oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2504_03967_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture
def qg_dense():
    from paper_2504_03967_amd import qg
    old = qg.get_tuning("dense_min_gates")
    qg.set_tuning("dense_min_gates", 1)
    yield qg
    qg.set_tuning("dense_min_gates", old)


def local_circuit(n, k, n_gates, seed):
    rng = W.SplitMix64(seed)
    pool = rng.shuffle(range(n))[:k]
    b = W.CircuitBuilder(n)
    for q in range(n):
        b.g1(W.H, q)
    prep = b.build()
    b = W.CircuitBuilder(n)
    for _ in range(n_gates):
        op = int(rng.below(10 if k > 1 else 6)[0])
        t = pool[int(rng.below(k)[0])]
        c = -1
        if op >= W.CX:
            c = pool[int(rng.below(k)[0])]
            while c == t:
                c = pool[int(rng.below(k)[0])]
        b.add(op, c, t, 2 * math.pi * rng.uniform(3))
    return prep, b.build()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,k", [(10, 4), (12, 5), (13, 6), (16, 3), (18, 5), (20, 6), (21, 2)])
def test_dense_block_matches_oracle(qg_dense, n, k, dtype):
    prep, circ = local_circuit(n, k, 40, seed=100 * n + k)
    kinds = qg_dense.plan_kernels(circ, dtype, qg_dense.FUSE_GREEDY)
    assert kinds and all(x == "dense" for x in kinds), kinds
    st = qg_dense.State(n, dtype)
    st.apply(prep, qg_dense.FUSE_NONE)      # generic start state
    st.apply(circ, qg_dense.FUSE_GREEDY)    # one pass on <= 6 qubits -> dense block
    torch.cuda.synchronize()
    psi = oracle.apply(circ, oracle.simulate(prep))
    got = st.tensor.cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - psi)) < TOL[dtype]
    st.close()


def test_dense_in_a_full_circuit(qg_dense):
    """Dense blocks between tile passes: random layers, a run of 40 gates on 5 qubits, a run
    of 30 gates on 6 qubits, random layers again."""
    n = 18
    circ = W.concat(W.concat(W.config3(n, layers=3, with_qft=False), local_circuit(n, 5, 40, seed=7)[1]),
                    W.concat(local_circuit(n, 6, 30, seed=8)[1], W.config3(n, seed=5, layers=3)))
    qg_dense.set_tuning("dense_min_gates", 20)  # the two local runs, not the random layers
    kinds = qg_dense.plan_kernels(circ, "c128", qg_dense.FUSE_GREEDY)
    assert kinds.count("dense") >= 2 and "tile" in kinds, kinds
    st = qg_dense.State(n, "c128")
    st.apply(circ, qg_dense.FUSE_GREEDY)
    torch.cuda.synchronize()
    assert np.max(np.abs(st.tensor.cpu().numpy() - oracle.simulate(circ))) < 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_dense_tile_widths_bitwise_equal(qg_dense, dtype):
    """Every dense tile width (2^10 .. 2^13 amplitudes: the kernel's (k, L) instantiations for
    k = 4, 5, 6) gives the same bits: each output sums the same k-steps in the same order;
    the default width also matches the oracle."""
    n = 16
    saved = qg_dense.get_tuning("dense_tile_bits")
    try:
        for k in (4, 5, 6):
            prep, circ = local_circuit(n, k, 40, seed=7 + k)
            psi = oracle.apply(circ, oracle.simulate(prep))
            ref = None
            for tb in (10, 11, 12, 13):
                qg_dense.set_tuning("dense_tile_bits", tb)
                assert qg_dense.plan_kernels(circ, dtype, qg_dense.FUSE_GREEDY) == ["dense"]
                st = qg_dense.State(n, dtype)
                st.apply(prep, qg_dense.FUSE_NONE)
                st.apply(circ, qg_dense.FUSE_GREEDY)
                got = st.tensor.cpu().numpy()
                st.close()
                if ref is None:
                    ref = got
                    assert np.max(np.abs(got.astype(np.complex128) - psi)) < TOL[dtype]
                assert np.array_equal(got, ref), (k, tb)
    finally:
        qg_dense.set_tuning("dense_tile_bits", saved)
