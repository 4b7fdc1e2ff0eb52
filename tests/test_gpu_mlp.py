"""Cost-model MLP kernels (FP32, on the GPU) against the FP64 reference."""
import numpy as np
import pytest
import torch

from oracle import mlp as ref
from paper_2504_03967_amd import workloads as W

pytestmark = pytest.mark.gpu

F = 24


@pytest.fixture(scope="module")
def qg():
    from paper_2504_03967_amd import qg as lib
    assert torch.cuda.is_available()
    return lib


def rand_model(qg, seed):
    m = qg.MLP(F, seed=seed)
    rng = np.random.default_rng(seed)
    theta = (rng.normal(scale=0.2, size=m.n_params)).astype(np.float32)
    m.set_params(theta)
    return m, theta.astype(np.float64), rng


@pytest.mark.parametrize("B", [1, 7, 300])
def test_forward_matches_reference(qg, B):
    m, theta, rng = rand_model(qg, B)
    X = rng.normal(size=(B, F)).astype(np.float32)
    y = m.forward(X)
    yr, _ = ref.forward(theta, X.astype(np.float64), F, 64)
    assert np.all(np.abs(y - yr) <= 1e-4 * np.maximum(1, np.abs(yr)))


@pytest.mark.parametrize("B", [1, 33, 256])
def test_gradient_matches_reference(qg, B):
    m, theta, rng = rand_model(qg, 100 + B)
    X = rng.normal(size=(B, F)).astype(np.float32)
    t = rng.normal(size=B).astype(np.float32)
    loss, g = m.grad(X, t)
    lr_, gr = ref.grad(theta, X.astype(np.float64), t.astype(np.float64), F, 64)
    assert abs(loss - lr_) <= 1e-4 * max(1, lr_)
    assert np.max(np.abs(g - gr)) <= 1e-3 * max(1e-3, np.max(np.abs(gr)))


def test_adam_matches_reference(qg):
    m, theta, rng = rand_model(qg, 5)
    m_ = np.zeros_like(theta)
    v_ = np.zeros_like(theta)
    th = theta.copy()
    for step in range(1, 4):
        g = rng.normal(size=theta.size).astype(np.float32)
        m.adam_step(g, 1e-3)
        th, m_, v_ = ref.adam_step(th, g.astype(np.float64), m_, v_, step, 1e-3)
    got = m.get_params()
    assert np.max(np.abs(got - th)) < 1e-6


def test_training_on_gpu_reduces_loss(qg):
    rng = np.random.default_rng(8)
    X = rng.normal(size=(2048, F)).astype(np.float32)
    t = (np.sin(X[:, 0]) + 0.3 * X[:, 1] * X[:, 2]).astype(np.float32)
    m = qg.MLP(F, seed=3)
    losses = m.train(X, t, epochs=40, batch=128, lr=3e-3, seed=1)
    assert losses[-1] < 0.2 * losses[0]
    y = m.forward(X)
    assert np.mean((y - t) ** 2) < 0.3 * np.var(t)
