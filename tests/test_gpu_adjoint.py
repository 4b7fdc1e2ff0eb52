"""Adjoint gradients of the GPU library against the oracle's adjoint recursion, the
parameter-shift rule and central finite differences (config 5 shape)."""
import math

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


def mixed_trainable(n, layers, seed):
    """RX/RY/RZ/CP trainable gates mixed with H, U3, CX, CZ, SWAP at all positions."""
    rng = W.SplitMix64(seed)
    b = W.CircuitBuilder(n)
    k = 0
    for _ in range(layers):
        for q in range(n):
            op = (W.RX, W.RY, W.RZ)[int(rng.below(3)[0])]
            b.g1(op, q, 6.28 * float(rng.uniform(1)[0]), pidx=k)
            k += 1
        b.g1(W.H, int(rng.below(n)[0]))
        b.g1(W.U3, int(rng.below(n)[0]), *(6.28 * rng.uniform(3)))
        for q in range(n - 1):
            b.g2(W.CX, q, q + 1)
        b.g2(W.CP, 0, n - 1, 6.28 * float(rng.uniform(1)[0]), pidx=k)
        k += 1
        a = int(rng.below(n)[0])
        b.g2(W.SWAP, a, (a + 1 + int(rng.below(n - 1)[0])) % n)
        b.g2(W.CZ, n - 1, 1)
    return b.build(), k


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [3, 8, 13, 15])
def test_adjoint_matches_oracle_adjoint(qg, n, dtype):
    circ, npar = mixed_trainable(n, 3, seed=70 + n)
    masks = W.zz_chain_masks(n)
    coeffs = np.linspace(0.5, 1.5, masks.size)
    val, grad = qg.adjoint_grad(circ, masks, coeffs, npar, dtype)
    rv, rg = oracle.adjoint_grad(circ, npar, masks, coeffs)
    # per Z-string term tolerance (1e-12 / 1e-5), times sum |coeff| for the weighted sum; a
    # gradient Im<lambda|P|psi> with lambda = sum_m c_m Z_m psi is such a sum as well.  The
    # complex128 gradients are held to the adjoint's 1e-10.
    w = float(np.sum(np.abs(coeffs)))
    assert abs(val.item() - rv) < (1e-12 if dtype == "c128" else 1e-5) * w
    assert np.max(np.abs(grad.cpu().numpy() - rg)) < (1e-10 if dtype == "c128" else 1e-5 * w)


@pytest.mark.parametrize("tile,low", [(8, 3), (9, 4), (11, 6)])
def test_adjoint_reverse_tile_shapes(qg, tile, low):
    """The reverse sweep's tile and low-block widths (tuning keys) change only the rounding:
    every shape matches the oracle's adjoint at the complex128 tolerances."""
    n = 15
    circ, npar = mixed_trainable(n, 3, seed=170 + tile)
    masks = W.zz_chain_masks(n)
    coeffs = np.linspace(0.5, 1.5, masks.size)
    rv, rg = oracle.adjoint_grad(circ, npar, masks, coeffs)
    saved = {k: qg.get_tuning(k) for k in ("adjoint_tile_bits", "adjoint_low_bits")}
    try:
        qg.set_tuning("adjoint_tile_bits", tile)
        qg.set_tuning("adjoint_low_bits", low)
        val, grad = qg.adjoint_grad(circ, masks, coeffs, npar, "c128")
    finally:
        for k, v in saved.items():
            qg.set_tuning(k, v)
    assert abs(val.item() - rv) < 1e-12 * float(np.sum(coeffs))
    assert np.max(np.abs(grad.cpu().numpy() - rg)) < 1e-10


def test_config5_adjoint_vs_parameter_shift_and_fd(qg):
    circ = W.config5()
    n, npar = circ.n_qubits, circ.n_params
    masks = W.zz_chain_masks(n)
    coeffs = np.ones(n - 1)
    val, grad = qg.adjoint_grad(circ, masks, coeffs, npar, "c128")
    grad = grad.cpu().numpy()
    st = qg.State(n, "c128")

    def f(c):
        st.reset()
        st.apply(c, qg.FUSE_GREEDY)
        return float(st.expval(masks, coeffs)[1])

    assert abs(val.item() - f(circ)) < 1e-12 * (n - 1)
    pick = W.SplitMix64(5).below(npar, 8)
    for k in pick:
        (g,) = np.nonzero(circ.param_idx == k)
        plus, minus = circ.copy(), circ.copy()
        plus.gate_param[g, 0] += math.pi / 2
        minus.gate_param[g, 0] -= math.pi / 2
        shift = 0.5 * (f(plus) - f(minus))
        assert abs(grad[k] - shift) < 1e-10, k
        h = 1e-6
        plus.gate_param[g, 0] += h - math.pi / 2
        minus.gate_param[g, 0] -= h - math.pi / 2
        fd = (f(plus) - f(minus)) / (2 * h)
        assert abs(grad[k] - fd) < 1e-5, k
    st.close()


def test_config5_adjoint_vs_oracle_sampled(qg):
    """Full 24-qubit config: value and all 480 gradients against the oracle adjoint."""
    circ = W.config5()
    masks = W.zz_chain_masks(24)
    coeffs = np.ones(23)
    val, grad = qg.adjoint_grad(circ, masks, coeffs, 480, "c128")
    rv, rg = oracle.adjoint_grad(circ, 480, masks, coeffs)
    assert abs(val.item() - rv) < 1e-12 * 23
    assert np.max(np.abs(grad.cpu().numpy() - rg)) < 1e-10


def test_autograd_function_and_gradcheck(qg):
    n, L = 6, 2
    rng = np.random.default_rng(0)
    ang = rng.uniform(-np.pi, np.pi, 2 * n * L)
    circ = W.ansatz(n, ang, L)
    masks = W.zz_chain_masks(n)
    coeffs = np.ones(n - 1)
    params = torch.tensor(ang, dtype=torch.float64, device="cuda", requires_grad=True)
    f = qg.QGExpval.apply(params, circ, masks, coeffs, "c128")
    f.backward()
    _, rg = oracle.adjoint_grad(circ, 2 * n * L, masks, coeffs)
    assert np.max(np.abs(params.grad.cpu().numpy() - rg)) < 1e-10
    with torch.no_grad():
        f2 = qg.QGExpval.apply(params.detach(), circ, masks, coeffs, "c128")
    assert abs(f2.item() - f.item()) < 1e-12
    fn = lambda p: qg.QGExpval.apply(p, circ, masks, coeffs, "c128")
    assert torch.autograd.gradcheck(fn, (params.detach().clone().requires_grad_(True),), eps=1e-6, atol=1e-6)


def test_adjoint_validation(qg):
    circ = W.config5(n=6, layers=1)
    masks = W.zz_chain_masks(6)
    with pytest.raises(qg.QGError):
        qg.adjoint_grad(circ, masks, np.ones(5), 3, "c128")  # slots >= n_params
    bad = W.CircuitBuilder(4).g1(W.U3, 0, 1, 2, 3, pidx=0).build()
    with pytest.raises(qg.QGError):
        qg.adjoint_grad(bad, [3], [1.0], 1, "c128")
