"""The allocation-free expectation entry point (qg_expval_noalloc) against qg_expval.

Both run the same kernels on the same state, so their results agree bit for bit.  Two
calls in a row, the second with a smaller state and fewer masks, check that the shared
device scratch keeps nothing that matters between calls; over-large mask counts are
rejected before anything runs."""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_03967_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qg():
    from paper_2504_03967_amd import qg as lib
    assert torch.cuda.is_available()
    return lib


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_expval_matches_expval_twice(qg, dtype):
    tol = 1e-12 if dtype == "c128" else 1e-5
    for n, n_terms, seed in ((20, 200, 1), (11, 37, 2)):
        circ = W.random_circuit(n, 150, seed=seed)
        st = qg.State(n, dtype)
        st.apply(circ, qg.FUSE_GREEDY)
        rng = np.random.default_rng(seed)
        masks = rng.integers(0, 1 << n, n_terms).astype(np.uint64)
        coeffs = rng.normal(size=n_terms)
        ref_terms, ref_sum = st.expval(masks, coeffs)
        terms = torch.full((n_terms,), float("nan"), dtype=torch.float64, device="cuda")
        total = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        st.expval_noalloc(masks, coeffs, terms, total)
        torch.cuda.synchronize()
        assert torch.equal(terms, ref_terms)
        assert total.item() == ref_sum.item()
        ev = oracle.expval(oracle.simulate(circ), masks)
        assert np.max(np.abs(terms.cpu().numpy() - ev)) < tol
        # outputs are optional
        only = torch.full((n_terms,), float("nan"), dtype=torch.float64, device="cuda")
        st.expval_noalloc(masks, None, only, None)
        torch.cuda.synchronize()
        assert torch.equal(only, ref_terms)
        st.close()


def test_noalloc_expval_limits(qg):
    st = qg.State(10, "c128")
    total = torch.full((1,), 5.0, dtype=torch.float64, device="cuda")
    st.expval_noalloc([], [], None, total)  # no terms: the sum is 0
    torch.cuda.synchronize()
    assert total.item() == 0.0
    too_many = np.zeros(257, dtype=np.uint64)
    out = torch.empty(257, dtype=torch.float64, device="cuda")
    with pytest.raises(qg.QGError) as e:
        st.expval_noalloc(too_many, None, out, None)
    assert e.value.status == qg.QG_EINVAL and "256" in str(e.value)
    with pytest.raises(qg.QGError):
        st.expval_noalloc([1 << 10], None, out, None)
    st.close()
