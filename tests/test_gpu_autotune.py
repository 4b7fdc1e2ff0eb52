"""The autotuner picks a shape per pass class; results stay identical to the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_03967_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_then_parity(tmp_path, monkeypatch):
    from paper_2504_03967_amd import autotune, qg
    monkeypatch.setenv("QG_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    before = autotune.snapshot("c128")
    try:
        table, source = autotune.tuned(22, "c128", reps=2)
        assert source == "search" and len(table) == 5
        for tile, reg, swz in table:
            assert 10 <= tile <= 13 and 2 <= reg <= 4 and swz in (0, 4)
        targets = autotune.current_targets("c128")
        # targets inside a cache line (3 lowest qubits in complex128) run on the lane kernel:
        # no shape of their own
        lane = 3 if qg.get_tuning("lane_gate") else 0
        assert all(t[0] == 0 for t in targets[:lane])
        assert all(t[0] in (10, 11, 12, 13) for t in targets[lane:22]) and all(t[0] == 0 for t in targets[22:])
        autotune.apply_targets([[0, 1, 0, 0]] * autotune.N_TARGETS, "c128")
        again, source2 = autotune.tuned(22, "c128")
        assert source2 == "cache" and again == table and autotune.current_targets("c128") == targets
        circ = W.random_circuit(22, 60, seed=8)
        st = qg.State(22, "c128")
        for fusion in (0, 1):
            st.reset()
            st.apply(circ, fusion)
            torch.cuda.synchronize()
            assert np.max(np.abs(st.tensor.cpu().numpy() - oracle.simulate(circ))) < 1e-12
        st.close()
    finally:
        autotune.restore(before, "c128")
