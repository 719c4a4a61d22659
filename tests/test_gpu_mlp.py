"""The warm-start network's HIP kernels against the NumPy oracle on the same
BF16 operands: forward outputs, gradients per tensor, one Adam step, and a
short training run through the library."""
import numpy as np
import pytest

from oracle import mlp
from parity_util import print_case

pytestmark = pytest.mark.gpu


def _data(B, seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed) + 0.02 * rng.normal(size=mlp.N_PARAMS)
    p = p.astype(np.float32).astype(np.float64)  # the FP32 master values
    x = rng.normal(size=(B, 4)).astype(np.float32)
    t = rng.normal(size=(B, mlp.N_OUT)).astype(np.float32)
    return p, x, t


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("B", [16, 64, 256])
def test_forward_matches_oracle(gpu_lib, B):
    p, x, t = _data(B, 1)
    net = gpu_lib.Mlp(p, B)
    y = net.forward(x).cpu().numpy().astype(np.float64)
    yo, _ = mlp.forward(p, x.astype(np.float64), bf16=True)
    err = np.abs(y - yo).max() / np.abs(yo).max()
    print_case(f"mlp forward B={B}: max rel err {err:.2e}")
    # FP32 accumulation vs FP64 on identical BF16 operands; a hidden value
    # whose FP32 sum lands on the other side of a BF16 rounding boundary
    # moves by one BF16 ulp (2^-8 relative)
    assert err < 2e-3
    assert _rel(y, yo) < 1e-3


@pytest.mark.parametrize("B", [64, 256])
def test_backward_matches_oracle(gpu_lib, B):
    p, x, t = _data(B, 2)
    net = gpu_lib.Mlp(p, B)
    y = net.forward(x).cpu().numpy().astype(np.float64)
    _, dy = mlp.mse(y, t.astype(np.float64))
    g = net.backward(dy.astype(np.float32)).cpu().numpy().astype(np.float64)
    yo, cache = mlp.forward(p, x.astype(np.float64), bf16=True)
    go = mlp.backward(p, cache, dy, bf16=True)
    for name, shape, off in mlp.layout():
        n = int(np.prod(shape))
        e = _rel(g[off:off + n], go[off:off + n])
        print_case(f"mlp grad {name} B={B}: rel Frobenius {e:.2e}")
        assert e < 0.02, name


def test_adam_step_matches_oracle(gpu_lib):
    p, x, t = _data(64, 3)
    net = gpu_lib.Mlp(p, 64)
    rng = np.random.default_rng(4)
    g = rng.normal(size=mlp.N_PARAMS).astype(np.float32)
    net.grads.copy_(__import__("torch").from_numpy(g))
    p32, m, v = p.copy(), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS)
    for k in (1, 2, 3):
        net.adam(1e-3)
        mlp.adam(p32, m, v, g.astype(np.float64), step=k, lr=1e-3)
    got = net.p32.cpu().numpy().astype(np.float64)
    assert np.abs(got - p32).max() < 1e-6
    bf = net.pbf16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    np.testing.assert_array_equal(bf.view(np.float32).astype(np.float64),
                                  mlp.bf16_round(got.astype(np.float32)))


def test_training_reduces_loss(gpu_lib):
    """A few hundred Adam steps on a smooth synthetic map: the loss falls."""
    rng = np.random.default_rng(5)
    B = 256
    x = rng.normal(size=(B, 4)).astype(np.float32)
    A = rng.normal(size=(4, mlp.N_OUT)) / 2
    t = np.tanh(x.astype(np.float64) @ A).astype(np.float32)
    net = gpu_lib.Mlp(mlp.init_params(6), B)
    losses = []
    for k in range(300):
        net.forward(x)
        if k == 0:  # the library's loss and gradient against the oracle's
            y = net.y.cpu().numpy().astype(np.float64)
            lo, dyo = mlp.mse(y, t.astype(np.float64))
        losses.append(net.mse_backward(t))
        if k == 0:
            assert losses[0] == pytest.approx(lo, rel=1e-5)
            np.testing.assert_allclose(net._dy.cpu().numpy(), dyo, rtol=1e-6, atol=1e-12)
        net.adam(1e-3)
    print_case(f"mlp training loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.2 * losses[0]
