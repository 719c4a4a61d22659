"""Pins of the warm-start network oracle (CPU): BF16 rounding against an
independent conversion, gradients against finite differences, the rounded
backward against the exact one, and Adam's update rule."""
import numpy as np
import pytest
import torch

from oracle import mlp


def test_layout_counts():
    assert mlp.N_PARAMS == 593408
    names = [n for n, _, _ in mlp.layout()]
    assert names == ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]
    v = np.arange(mlp.N_PARAMS, dtype=np.float64)
    np.testing.assert_array_equal(mlp.pack(mlp.unpack(v)), v)


def test_bf16_round_matches_torch_conversion():
    """Round to nearest even from FP32, checked against torch's float32 ->
    bfloat16 conversion (another implementation), including exact ties."""
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.uniform(-6, 6, size=20000),
                        [0.0, -0.0, 1.0, -2.5, 3.0e-39]]).astype(np.float32)
    # ties: FP32 values exactly half-way between two BF16 values
    base = rng.integers(0x3F000000, 0x40000000, size=2000, dtype=np.uint32) & 0xFFFF0000
    ties = (base | 0x8000).view(np.float32)
    for arr in (x, ties):
        want = torch.from_numpy(arr.copy()).to(torch.bfloat16).to(torch.float64).numpy()
        np.testing.assert_array_equal(mlp.bf16_round(arr), want)


def _loss(p, x, t, bf16):
    y, _ = mlp.forward(p, x, bf16=bf16)
    return mlp.mse(y, t)[0]


def test_gradient_matches_finite_differences():
    """Exact (FP64) backward against central differences, on sampled
    entries of every weight and bias tensor."""
    rng = np.random.default_rng(1)
    p = mlp.init_params(2) + 0.01 * rng.normal(size=mlp.N_PARAMS)  # nonzero biases
    x = rng.normal(size=(6, 4))
    t = rng.normal(size=(6, mlp.N_OUT))
    y, cache = mlp.forward(p, x, bf16=False)
    _, dy = mlp.mse(y, t)
    g = mlp.backward(p, cache, dy, bf16=False)
    h = 1e-6
    for name, shape, off in mlp.layout():
        idx = off + rng.choice(int(np.prod(shape)), size=12, replace=False)
        for i in idx:
            e = np.zeros_like(p)
            e[i] = h
            fd = (_loss(p + e, x, t, False) - _loss(p - e, x, t, False)) / (2 * h)
            assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-10), (name, i)


def test_rounded_backward_close_to_exact():
    """The BF16-operand backward differs from the exact one by BF16 rounding
    only: 2^-9 per operand, compounded through the layers (relative
    Frobenius norm per tensor below 5 %, the first layer's being largest)."""
    rng = np.random.default_rng(3)
    p = mlp.init_params(4)
    x = rng.normal(size=(64, 4))
    t = rng.normal(size=(64, mlp.N_OUT))
    y64, c64 = mlp.forward(p, x, bf16=False)
    y16, c16 = mlp.forward(p, x, bf16=True)
    assert np.linalg.norm(y16 - y64) / np.linalg.norm(y64) < 0.02
    g64 = mlp.unpack(mlp.backward(p, c64, mlp.mse(y64, t)[1], bf16=False))
    g16 = mlp.unpack(mlp.backward(p, c16, mlp.mse(y16, t)[1], bf16=True))
    for k in g64:
        assert np.linalg.norm(g16[k] - g64[k]) / np.linalg.norm(g64[k]) < 0.05, k


def test_adam_first_step_and_convergence():
    """First step moves every parameter by lr against the gradient's sign
    (bias-corrected moments equal g and g^2); repeated steps minimise a
    convex quadratic."""
    g = np.array([3.0, -0.5, 1e-3, -7.0])
    p = np.zeros(4)
    m, v = np.zeros(4), np.zeros(4)
    mlp.adam(p, m, v, g, step=1, lr=0.01)
    np.testing.assert_allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    a = np.array([1.0, 10.0, 0.1, 3.0])
    p = np.array([1.0, -2.0, 3.0, 0.5])
    m, v = np.zeros(4), np.zeros(4)
    for k in range(1, 3001):
        mlp.adam(p, m, v, a * p, step=k, lr=0.01)
    assert np.abs(p).max() < 0.02
