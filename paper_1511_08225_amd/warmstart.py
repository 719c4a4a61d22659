"""Learned warm start (not in the paper): a network trained on steady sheath
profiles that the batched sweep itself produces predicts, from four run
parameters, the steady potential and moments of a new run; the run is then
loaded from those profiles instead of cold (slpic_run_config.warm_profile).

The network's forward pass, loss gradient, backward pass and Adam step run in
the library's kernels (``slpic.Mlp``); this module is the data plumbing
around them: the input features, the resampling of moment rows onto 256
points of x/L, the standardisation of inputs and outputs, minibatching.

Profiles: 7 rows of 256 values on x/L = k/255: phi, n_e, n_i, Gamma_e,
Gamma_i, T_e, T_i (physical, f = beta g, Eq. 5; T = (2K/n - m V^2)/3 from the
kinetic energy density K and the drift V = Gamma/n).  The network learns the
densities and temperatures as logarithms (they span orders of magnitude and
are positive), the potential and the fluxes as they are.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import slpic

N_POINTS = 256
N_ROWS = 7      # phi, n_e, n_i, Gamma_e, Gamma_i, T_e, T_i
LOG_ROWS = (1, 2, 5, 6)  # rows the network sees as logarithms
MOMENT_ROWS = (0, 1, 4, 2, 5)  # phi, n_e, n_i, Gamma_e, Gamma_i in the slpic_moments layout
N_FLOOR = 1e-6  # density floor of the logarithm (n0 = 1)


def features(cfg: dict) -> np.ndarray:
    """(ln Te/Ti, ln A, u/v_ti, ln L/lambda_D) of a sheath configuration."""
    return np.array([math.log(cfg["te_over_ti"]), math.log(cfg["ion_amu"]), cfg["u_over_vti"],
                     math.log(cfg["nx"] * cfg["dx"])], dtype=np.float64)


def temperatures(m: np.ndarray, cfg: dict) -> np.ndarray:
    """(2, nodes) temperatures T_e, T_i from a (7, nodes) moment array
    (phi, then per species n, Gamma_x, kinetic energy density): the three
    velocity components' mean thermal energy about the drift, in T_e units;
    where a species is (almost) absent, its source temperature."""
    out = []
    for s, (rn, rg, rk) in enumerate(((1, 2, 3), (4, 5, 6))):
        mass = cfg["species"][s]["mass"]
        T0 = cfg["species"][s]["temperature"]
        n = m[rn]
        ok = n > N_FLOOR
        nn = np.where(ok, n, 1.0)
        T = (2.0 * m[rk] / nn - mass * (m[rg] / nn) ** 2) / 3.0
        out.append(np.where(ok & (T > 1e-3 * T0), T, T0))
    return np.stack(out)


def profiles_from_moments(m: np.ndarray, cfg: dict) -> np.ndarray:
    """(7, 256) profiles from a (7, nx+1) moment array (node j at x/L = j/nx)."""
    nodes = m.shape[1]
    xn = np.arange(nodes) / (nodes - 1)
    xi = np.arange(N_POINTS) / (N_POINTS - 1)
    T = temperatures(m, cfg)
    rows = [np.interp(xi, xn, m[row]) for row in MOMENT_ROWS] + [np.interp(xi, xn, T[s]) for s in range(2)]
    return np.stack(rows)


def collect_profiles(cfgs: list[dict], steps: int, sample_every: int = 64, sample_last: int = 2048,
                     precision: str = "f32", tuning: dict | None = None):
    """Advance the runs together from cold for `steps` steps, averaging the
    moments over the last `sample_last` steps (a sample every `sample_every`).
    Returns the (N, 7, 256) profiles and the sampled-window mean of Phi_w."""
    tuning = tuning or {"chunk": 512, "block": 64, "sort_every": 64, "sort_bucket": 1}
    se = tuning["sort_every"]
    g = max(16, se)
    sim = slpic.Sim(cfgs, precision=precision, sort_every=se, sort_bucket=tuning["sort_bucket"],
                    chunk=tuning["chunk"], block=tuning["block"], graph_steps=g,
                    push_order=tuning.get("push_order", 0), sort_tile=tuning.get("sort_tile", 0))
    first = max(0, steps - sample_last)
    sim.step(first)
    done = first
    while done < steps:
        sim.step(sample_every)
        done += sample_every
        sim.moments_sample(-1)
    torch.cuda.synchronize()
    prof = np.stack([profiles_from_moments(sim.moments_window(r).cpu().numpy(), cfgs[r]) for r in range(len(cfgs))])
    phi_w = prof[:, 0, 0] - prof[:, 0, -1]
    sim.close()
    return prof, phi_w


def to_net(Y: np.ndarray) -> np.ndarray:
    """Profiles (N, 7, 256) as the network learns them: logarithms of the
    densities (floored) and temperatures."""
    Z = np.array(Y, dtype=np.float64, copy=True).reshape(len(Y), N_ROWS, N_POINTS)
    for r in LOG_ROWS:
        Z[:, r] = np.log(np.maximum(Z[:, r], N_FLOOR))
    return Z


def from_net(Z: np.ndarray) -> np.ndarray:
    Y = np.array(Z, dtype=np.float64, copy=True).reshape(len(Z), N_ROWS, N_POINTS)
    for r in LOG_ROWS:
        Y[:, r] = np.exp(Y[:, r])
    return Y


class Standardizer:
    """Inputs: per-feature mean and standard deviation.  Outputs (in the
    network's form, see to_net): per-point mean, one standard deviation per
    profile row (so rows with a pinned value, such as phi at the wall, stay
    finite)."""

    def __init__(self, X: np.ndarray, Y: np.ndarray):
        self.xm, self.xs = X.mean(axis=0), X.std(axis=0) + 1e-12
        Z = to_net(Y)
        self.ym = Z.mean(axis=0)
        self.ys = Z.std(axis=(0, 2)) + 1e-12

    def x(self, X):
        return ((X - self.xm) / self.xs).astype(np.float32)

    def y(self, Y):
        Z = to_net(Y)
        return ((Z - self.ym) / self.ys[None, :, None]).reshape(len(Z), -1).astype(np.float32)

    def y_inv(self, Z):
        Z = np.asarray(Z, dtype=np.float64).reshape(len(Z), N_ROWS, N_POINTS)
        return from_net(Z * self.ys[None, :, None] + self.ym)


def _init_params(seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in ((256, 4), (256, 256), (256, 256), (N_ROWS * N_POINTS, 256)):
        b = math.sqrt(6.0 / i)
        parts.append(rng.uniform(-b, b, size=o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def train(X: np.ndarray, Y: np.ndarray, epochs: int = 400, lr: float = 1e-3, batch: int = 256, seed: int = 0,
          log=None):
    """Train on (features, profiles); returns (network, standardizer, losses)."""
    std = Standardizer(X, Y)
    xs, ys = std.x(X), std.y(Y)
    net = slpic.Mlp(_init_params(seed), batch)
    rng = np.random.default_rng(seed + 1)
    n = len(xs)
    losses = []
    for ep in range(epochs):
        if n >= batch:
            order = rng.permutation(n)
            batches = [order[k * batch:(k + 1) * batch] for k in range(n // batch)]
        else:  # fewer samples than a batch: draw with replacement
            batches = [rng.integers(0, n, size=batch)]
        tot = 0.0
        for idx in batches:
            net.forward(xs[idx])
            tot += net.mse_backward(ys[idx])
            net.adam(lr)
        losses.append(tot / len(batches))
        if log and (ep % 50 == 0 or ep == epochs - 1):
            log(f"epoch {ep}: loss {losses[-1]:.4f}")
    return net, std, losses


def predict(net, std: Standardizer, cfgs: list[dict]) -> np.ndarray:
    """(N, 7, 256) predicted profiles for the configurations."""
    X = std.x(np.stack([features(c) for c in cfgs]))
    out = []
    B = net.batch
    for k in range(0, len(X), B):
        xb = X[k:k + B]
        pad = np.zeros((B, 4), dtype=np.float32)
        pad[:len(xb)] = xb
        y = net.forward(pad).cpu().numpy()[:len(xb)]
        out.append(std.y_inv(y))
    return np.concatenate(out)


def quasi_neutral(prof: np.ndarray) -> np.ndarray:
    """The load profile made from a prediction: electrons take the ion
    density and flux (n_e = n_i, Gamma_e = Gamma_i).  In the steady state of
    a floating wall fed by a pair source both species carry the same flux
    everywhere, and outside the thin sheath n_e = n_i; loading the predicted
    densities as they are would put their independent errors (a percent or
    more) into the net charge and start a strong potential transient, while
    the sheath itself re-forms within a few steps."""
    out = np.array(prof, dtype=np.float64, copy=True)
    out[..., 1, :] = out[..., 2, :]
    out[..., 3, :] = out[..., 4, :]
    return out


def steady_index(phi_w: np.ndarray, window: int, reference: float, tol: float = 0.02) -> int:
    """First step count at which a window of Phi_w means lies within tol of
    the reference and the next two windows do too (-1 if never)."""
    nw = len(phi_w) // window
    if nw < 3:
        return -1
    means = phi_w[:nw * window].reshape(nw, window).mean(axis=1)
    ok = np.abs(means - reference) <= tol * abs(reference)
    for k in range(nw - 2):
        if ok[k] and ok[k + 1] and ok[k + 2]:
            return (k + 1) * window
    return -1
