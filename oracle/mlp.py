"""FP64 NumPy oracle of the warm-start network -- TEST INFRASTRUCTURE ONLY.

The learned part is not in the paper: it is a small fully connected network
that maps four sheath parameters (ln Te/Ti, ln A, u/v_ti, ln L/lambda_D,
standardised) to steady profiles on 256 points of x/L (phi, n_e, n_i,
Gamma_e, Gamma_i, T_e, T_i; 1792 outputs, standardised), so that a new run
can be loaded near its steady state instead of cold.

Model: 4 -> 256 -> 256 -> 256 -> 1792, ReLU after the three hidden layers,
mean squared error, Adam (beta1 0.9, beta2 0.999, eps 1e-8).  The GPU keeps
weights, biases, inputs and stored activations in BF16 and accumulates in
FP32; this oracle computes in FP64 and, with ``bf16=True``, rounds exactly
those operands to BF16 (round to nearest even from FP32), so that it sees the
same operands as the GPU.  The backward pass uses the same rounded operands:
the output gradient and the hidden-layer gradients are rounded to BF16
before they enter a product.

Parameter vector (element offsets, the same in the BF16 and FP32 copies):
W1 [256][4], b1 [256], W2 [256][256], b2 [256], W3 [256][256], b3 [256],
W4 [1792][256], b4 [1792]; 593,408 values.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 4, 256, 1792
LAYERS = [(N_HID, N_IN), (N_HID, N_HID), (N_HID, N_HID), (N_OUT, N_HID)]


def layout():
    """[(name, shape, offset)] of the parameter vector."""
    out, off = [], 0
    for l, (o, i) in enumerate(LAYERS, start=1):
        out.append((f"W{l}", (o, i), off))
        off += o * i
        out.append((f"b{l}", (o,), off))
        off += o
    return out


N_PARAMS = sum(int(np.prod(s)) for _, s, _ in layout())


def unpack(vec: np.ndarray) -> dict:
    return {name: vec[off:off + int(np.prod(shape))].reshape(shape) for name, shape, off in layout()}


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _, _ in layout()])


def bf16_round(x) -> np.ndarray:
    """Round to BF16 (8 exponent bits, 7 stored mantissa bits) to nearest,
    ties to even, from the FP32 value; returned as float64.  Finite inputs."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, FP32 values."""
    rng = np.random.default_rng(seed)
    d = {}
    for l, (o, i) in enumerate(LAYERS, start=1):
        bound = np.sqrt(6.0 / i)
        d[f"W{l}"] = rng.uniform(-bound, bound, size=(o, i)).astype(np.float32).astype(np.float64)
        d[f"b{l}"] = np.zeros(o)
    return pack(d)


def forward(params: np.ndarray, x: np.ndarray, bf16: bool = True):
    """y [B][1792] and the cache (x, h1, h2, h3 as seen by the next layer)."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    p = {k: rnd(v) for k, v in unpack(params).items()}
    h = rnd(x)
    cache = [h]
    for l in (1, 2, 3):
        h = rnd(np.maximum(h @ p[f"W{l}"].T + p[f"b{l}"], 0.0))
        cache.append(h)
    y = h @ p["W4"].T + p["b4"]
    return y, cache


def backward(params: np.ndarray, cache, dy: np.ndarray, bf16: bool = True) -> np.ndarray:
    """Gradient of sum(dy * y) with respect to the parameter vector."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    p = {k: rnd(v) for k, v in unpack(params).items()}
    x, h1, h2, h3 = cache
    g = {}
    d = rnd(dy)
    for l, hin in ((4, h3), (3, h2), (2, h1), (1, x)):
        g[f"W{l}"] = d.T @ hin
        g[f"b{l}"] = d.sum(axis=0)
        if l > 1:
            d = rnd((d @ p[f"W{l}"]) * (hin > 0))
    return pack(g)


def mse(y: np.ndarray, t: np.ndarray):
    """Mean squared error over all outputs and its gradient dL/dy."""
    diff = y - t
    return float(np.mean(diff * diff)), 2.0 * diff / diff.size


def adam(p32: np.ndarray, m: np.ndarray, v: np.ndarray, g: np.ndarray, step: int, lr: float,
         b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step counts from 1), in place; returns the BF16 copy."""
    m *= b1
    m += (1.0 - b1) * g
    v *= b2
    v += (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    p32 -= lr * mhat / (np.sqrt(vhat) + eps)
    return bf16_round(p32)
