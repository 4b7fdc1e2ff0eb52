"""Learned fusion end to end on a small scale: timings made by the simulator, the MLP
trained by the library's kernels, the learned plan's results and measured time."""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_03967_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    from paper_2504_03967_amd import costmodel as cm
    from paper_2504_03967_amd import qg
    X, y = cm.collect(240, n_values=(16, 18, 20, 22), reps=2)
    assert X.shape == (240, qg.PASS_FEATURES) and np.all(np.isfinite(y))
    model, losses = cm.train(X[:200], y[:200], epochs=150, batch=50, lr=3e-3)
    assert losses[-1] < 0.5 * losses[0]
    err = cm.mape(model, X[200:], y[200:])
    model.install()
    yield qg, cm, model, err
    qg.clear_cost_model()
    model.close()


def test_model_error_is_bounded(trained):
    qg, cm, model, err = trained
    assert err < 0.6, err


def test_learned_plan_parity_and_time(trained):
    qg, cm, model, err = trained
    circs = cm.held_out_circuits(count=4, n_values=(14, 20))
    small = [c for c in circs if c.n_qubits == 14]
    for c in small:
        st = qg.State(c.n_qubits, "c128")
        st.apply(c, qg.FUSE_LEARNED)
        torch.cuda.synchronize()
        got = st.tensor.cpu().numpy()
        assert np.max(np.abs(got - oracle.simulate(c))) < 1e-12
        pog, npass = qg.plan_passes(c, "c128", qg.FUSE_LEARNED)
        assert set(np.unique(pog)) == set(range(npass))
        last = {}
        for i, (op, q0, q1) in enumerate(c.gate_type):  # gates sharing a qubit keep their order
            for q in ((q0, q1) if op in W.TWO_QUBIT else (q1,)):
                assert q not in last or pog[last[q]] <= pog[i]
                last[q] = i
    # learned plans must not be slower than greedy beyond the run-to-run spread of the
    # greedy plan itself (five alternating repeats of the same circuits)
    res = cm.compare_plans([c for c in circs if c.n_qubits == 20], reps=3, repeats=5)
    assert res["gain"] >= 1.0 - 2.0 * res["greedy_spread"] - 0.01, res
