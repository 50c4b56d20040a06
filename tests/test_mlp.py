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


def _bf16(x):
    """Round to nearest even BF16 (as float64)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.gpu
def test_gpu_bf16_mfma_inference_against_bf16_reference(fp4):
    """BF16 inference on the matrix cores against a host evaluation with the same roundings
    (BF16 inputs, weights and hidden activations, wide accumulation): the MFMA operand
    layouts, the zero padding of K = 18 and of the 2-wide output layer, and a ragged row
    count (1000 rows, not a multiple of 64) are all exercised."""
    rng = np.random.default_rng(4)
    nin, width, depth = 18, 128, 5
    X = rng.standard_normal((1000, nin)).astype(np.float32)
    with fp4.Mlp(0, nin, width, depth, seed=11) as net:
        p = net.get_params().astype(np.float64)
        out, _ = net.predict(X, bf16=True)
    dims, _ = mlp_ref.layout(nin, width, depth)
    h = _bf16(X)
    for l, (i, o, wo, bo) in enumerate(dims):
        W = _bf16(p[wo:wo + i * o].reshape(o, i).astype(np.float32))
        z = h @ W.T + p[bo:bo + o]
        h = _bf16(z / (1.0 + np.exp(-z))) if l + 1 < depth else z
    err = np.abs(out - h)
    scale = np.max(np.abs(h))
    assert np.median(err) <= 1e-3 * scale
    assert np.max(err) <= 3e-2 * scale
