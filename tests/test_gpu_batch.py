"""Batched form (config 4 shape) against the oracle, per circuit: one-tile circuits in the
persistent launch, larger ones pass by pass."""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_03967_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


@pytest.fixture(scope="module")
def qg():
    from paper_2504_03967_amd import qg as lib
    assert torch.cuda.is_available()
    return lib


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_small_batch_all_sizes(qg, dtype):
    circs = W.config4(seed=11, n_circuits=60, n_min=1, n_max=16, l_min=1, l_max=4)
    out = qg.batch_expval(circs, dtype).cpu().numpy()
    ref = oracle.batch_zz_chain(circs)
    # tolerance per Z_i Z_{i+1} term, scaled by the number of terms
    scale = np.array([max(c.n_qubits - 1, 1) for c in circs])
    assert np.all(np.abs(out - ref) <= TOL[dtype] * scale)


def test_config4_every_circuit(qg):
    """All 4096 circuits of the batched workload, in both precisions, against the oracle
    (one FP64 run of every circuit; tolerance per Z_i Z_{i+1} term, times the n - 1 terms)."""
    circs = W.config4()
    assert len(circs) == 4096
    ref = oracle.batch_zz_chain(circs)
    terms = np.array([c.n_qubits - 1 for c in circs], dtype=np.float64)
    for dtype in ("c128", "c64"):
        out = qg.batch_expval(circs, dtype).cpu().numpy()
        err = np.abs(out - ref) / terms
        assert np.all(err <= TOL[dtype]), (dtype, int(np.argmax(err)), float(err.max()))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_first_pass_skipping_tiles(qg, dtype):
    """Multi-tile circuits whose first pass skips tiles (every op of it is conditioned on a
    qubit outside the tile) run it on the filled |0...0> like any later pass, also in device
    memory that held another batch's states just before."""
    lo = 13 if dtype == "c128" else 14
    amp = 16 if dtype == "c128" else 8
    junk = W.config4(seed=5, n_circuits=24, n_min=lo, n_max=17, l_min=2, l_max=3)
    qg.batch_expval(junk, dtype)
    torch.cuda.synchronize()
    circs = []
    for k, n in enumerate(range(lo, lo + 4)):
        b = W.CircuitBuilder(n)
        b.g2(W.CP, n - 1, n - 2, 0.3 + k)
        b.g2(W.CX, n - 1, 0)
        circs.append(b.build())
        # a fill, one pass over half the tiles (fixed control qubit), the observable's read
        assert qg.plan_bytes(circs[-1], dtype, qg.FORM_BATCHED) == (1, 3.0 * (amp << n))
    circs += W.config4(seed=6, n_circuits=8, n_min=lo, n_max=lo + 3, l_min=1, l_max=3)
    out = qg.batch_expval(circs, dtype).cpu().numpy()
    ref = oracle.batch_zz_chain(circs)
    terms = np.array([c.n_qubits - 1 for c in circs], dtype=np.float64)
    err = np.abs(out - ref) / terms
    assert np.all(err <= TOL[dtype]), (int(np.argmax(err)), float(err.max()))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_many_state_groups(qg, dtype):
    """With a small state budget the multi-tile circuits run in many groups that reuse one
    state buffer (each group: fill, passes, observable); results as with one group."""
    lo = 13 if dtype == "c128" else 14
    circs = W.config4(seed=8, n_circuits=24, n_min=lo - 3, n_max=18, l_min=1, l_max=4)
    for n in (lo, lo + 2):  # first passes that skip tiles: states filled per group
        b = W.CircuitBuilder(n)
        b.g2(W.CP, n - 1, n - 2, 0.4)
        b.g2(W.CX, n - 1, 0)
        circs.append(b.build())
    ref = oracle.batch_zz_chain(circs)
    terms = np.array([max(c.n_qubits - 1, 1) for c in circs], dtype=np.float64)
    one = qg.batch_expval(circs, dtype).cpu().numpy()
    saved = qg.get_tuning("batch_group_mib")
    try:
        qg.set_tuning("batch_group_mib", 4)  # about one 18-qubit complex128 state per group
        many = qg.batch_expval(circs, dtype).cpu().numpy()
    finally:
        qg.set_tuning("batch_group_mib", saved)
    for out in (one, many):
        err = np.abs(out - ref) / terms
        assert np.all(err <= TOL[dtype]), (int(np.argmax(err)), float(err.max()))
    assert np.array_equal(one, many)


def test_graph_replays_and_new_params(qg):
    circs = W.config4(seed=21, n_circuits=40, n_min=8, n_max=18, l_min=2, l_max=5)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = qg.Batch(circs, "c128", stream=stream)
        eager = qg.batch_expval(circs, "c128", stream=stream).clone()
        for rep in range(3):
            got = b.launch().clone()
            stream.synchronize()
            assert torch.allclose(got, eager, atol=1e-12, rtol=0), rep
            # eager work and a host sync between replays
            junk = torch.randn(1000, device="cuda").sum().item()
        # new angles, same structure
        rng = np.random.default_rng(3)
        new = []
        for c in circs:
            d = c.copy()
            d.gate_param[:, 0] = rng.uniform(-np.pi, np.pi, d.n_gates)
            new.append(d)
        b.set_params(new)
        got = b.launch().clone()
        stream.synchronize()
    ref = oracle.batch_zz_chain(new)
    assert np.max(np.abs(got.cpu().numpy() - ref) / np.array([c.n_qubits - 1 for c in new])) < 1e-12
    b.close()


def test_csr_observables(qg):
    circs = W.config4(seed=31, n_circuits=12, n_min=3, n_max=15, l_min=1, l_max=3)
    rng = np.random.default_rng(9)
    obs = []
    for c in circs:
        k = int(rng.integers(0, 5))
        obs.append((rng.integers(0, 1 << c.n_qubits, k).astype(np.uint64), rng.normal(size=k)))
    out = qg.batch_expval(circs, "c128", obs=obs).cpu().numpy()
    for c, (m, w), o in zip(circs, obs, out):
        ref = float(np.dot(w, oracle.expval(oracle.simulate(c), m))) if len(m) else 0.0
        assert abs(o - ref) < 1e-12 * max(1, len(m))


def test_batch_validation(qg):
    circs = W.config4(seed=1, n_circuits=2)
    bad = circs[0].copy()
    bad.gate_type[0, 2] = 40
    with pytest.raises(qg.QGError):
        qg.batch_expval([circs[1], bad])
    big = W.ghz(23)
    with pytest.raises(qg.QGError):
        qg.batch_expval([big])
    with pytest.raises(qg.QGError):
        qg.Batch(circs).set_params([circs[1], circs[0]])
