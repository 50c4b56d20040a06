"""Surrogate network: the FP64 reference is pinned by finite differences (CPU); the
library's hand-written forward/backward/Adam kernels are checked against it (GPU)."""
import numpy as np
import pytest

from oracle import mlp_ref


def test_reference_gradient_finite_differences():
    """Central differences of the reference loss match its chain-rule gradient (catches a
    missing activation derivative, a transposed weight or a wrong loss term)."""
    rng = np.random.default_rng(0)
    nin, width, depth = 5, 7, 4
    _, n = mlp_ref.layout(nin, width, depth)
    p = rng.standard_normal(n) * 0.5
    X = rng.standard_normal((9, nin))
    y = rng.standard_normal(9)
    L, g = mlp_ref.loss_grad(p, X, y, nin, width, depth)
    assert L == pytest.approx(mlp_ref.loss(p, X, y, nin, width, depth), rel=1e-14)
    h = 1e-6
    for k in rng.choice(n, 40, replace=False):
        e = np.zeros(n)
        e[k] = h
        fd = (mlp_ref.loss(p + e, X, y, nin, width, depth) - mlp_ref.loss(p - e, X, y, nin, width, depth)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_reference_layout_counts():
    _, n = mlp_ref.layout(10, 128, 5)
    assert n == 10 * 128 + 128 + 3 * (128 * 128 + 128) + 128 * 2 + 2


@pytest.fixture(scope="module")
def fp4():
    import paper_2104_04895_amd as m
    return m


@pytest.mark.gpu
def test_gpu_loss_and_gradient_against_reference(fp4):
    """The library's FP32 forward/backward kernels against the FP64 reference on the same
    parameters and data: loss to 1e-5, every gradient entry to 1e-4 of the largest."""
    rng = np.random.default_rng(1)
    nin, width, depth = 10, 128, 5
    with fp4.Mlp(0, nin, width, depth, seed=3) as net:
        p = net.get_params()
        X = rng.standard_normal((300, nin)).astype(np.float32)
        y = rng.standard_normal(300).astype(np.float32)
        L, g = net.loss_grad(X, y)
    Lr, gr = mlp_ref.loss_grad(p.astype(np.float64), X, y, nin, width, depth)
    assert L == pytest.approx(Lr, rel=1e-5)
    assert np.max(np.abs(g - gr)) <= 1e-4 * np.max(np.abs(gr))


@pytest.mark.gpu
def test_gpu_training_and_bf16_inference(fp4):
    """Adam on the GPU fits a smooth target (loss falls by >10x); BF16 inference agrees with
    FP32 inference to BF16 precision."""
    rng = np.random.default_rng(2)
    nin = 4
    X = rng.uniform(-1, 1, (4096, nin)).astype(np.float32)
    y = (np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2] - 0.5 * X[:, 3] ** 2).astype(np.float32)
    with fp4.Mlp(0, nin, 64, 4, seed=5) as net:
        losses = net.train(X, y, epochs=60, batch=256, lr=3e-3, seed=7)
        assert losses[-1] < losses[0] - 2.0      # NLL: log-sigma drops as the fit tightens
        out32, _ = net.predict(X, bf16=False)
        out16, _ = net.predict(X, bf16=True)
    assert np.sqrt(np.mean((out32[:, 0] - y) ** 2)) < 0.05
    assert np.max(np.abs(out16[:, 0] - out32[:, 0])) < 0.05
