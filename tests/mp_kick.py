"""The frozen-field velocity map of Eq. (A2a) in 40-digit arithmetic
(mpmath): the same segments as the closed form (beta = 1 inside the band of
Eq. 11b, the antiderivative G_c(p) = (p sqrt(p^2 + c^2) + c^2 asinh(p/c))/2
outside it, c^2 -> c^2 + u^2 for Eq. 11a), each root found by bisection to
1e-35.  Tests use it to measure the rounding error of the FP64 maps; it
shares nothing with the oracle or the library."""
import math

import mpmath as mp
import numpy as np

DIGITS = 40


def _G(cc, p):
    if cc == 0:
        return p * abs(p) / 2
    return (p * mp.sqrt(p * p + cc) + cc * mp.asinh(p / mp.sqrt(cc))) / 2


def _advance(cc, p, K):
    """p1 >= p with G(p1) - G(p) = K."""
    if K <= 0:
        return p
    target = _G(cc, p) + K
    q = p * abs(p) / 2 + K
    hi = mp.sqrt(2 * q) if q >= 0 else -mp.sqrt(-2 * q)
    if cc > 0:
        hi = min(hi, p + K / mp.sqrt(cc))
    lo = p
    tol = mp.mpf(10) ** -35
    for _ in range(400):
        mid = (lo + hi) / 2
        if _G(cc, mid) < target:
            lo = mid
        else:
            hi = mid
        if hi - lo < tol * max(1, abs(hi)):
            break
    return (lo + hi) / 2


def kick(kind: str, u: float, dt: float, vx: float, c2: float, a: float) -> float:
    """v_x after one step for v = (vx, sqrt(c2), 0) and a = (a, 0, 0)."""
    with mp.workdps(DIGITS):
        vx, c2, a, dt = mp.mpf(vx), mp.mpf(c2), mp.mpf(a), mp.mpf(dt)
        if a == 0:
            return float(vx)
        if math.isinf(u):
            return float(vx + a * dt)
        u = mp.mpf(u)
        A, sg = abs(a), (1 if a > 0 else -1)
        p0 = vx * sg
        if kind == "smooth":
            return float(sg * _advance(c2 + u * u, p0, A * u * dt))
        if c2 >= u * u:
            return float(sg * _advance(c2, p0, A * u * dt))
        ps = mp.sqrt(u * u - c2)
        p, rem = p0, dt
        if p < -ps:  # fast, up to the band
            need, avail = _G(c2, -ps) - _G(c2, p), A * u * rem
            if need >= avail:
                return float(sg * _advance(c2, p, avail))
            rem -= need / (A * u)
            p = -ps
        if p <= ps:  # slow, across the band
            tb = (ps - p) / A
            if tb >= rem:
                return float(sg * (p + A * rem))
            rem -= tb
            p = ps
        return float(sg * _advance(c2, p, A * u * rem))


def hard_cases(n: int = 600, seed: int = 0):
    """Random (vx, c^2, a) over six decades, with a fifth of the cases
    slowed through v_x = 0 with perpendicular speeds of 1e-8 to 1e-3 (where
    the inversion of G is worst conditioned)."""
    rng = np.random.default_rng(seed)
    vx = rng.normal(size=n) * 10 ** rng.uniform(-2, 0.7, size=n)
    c2 = (rng.normal(size=n) * 10 ** rng.uniform(-3, 0.5, size=n)) ** 2
    c2[: n // 20] = 0.0
    a = rng.normal(size=n) * 10 ** rng.uniform(-4, 0.5, size=n)
    m = n // 5
    a[-m:] = rng.uniform(0.5, 2.0, m) * np.sign(rng.normal(size=m))
    vx[-m:] = -a[-m:] * rng.uniform(0.2, 2.0, m)
    c2[-m:] = (10 ** rng.uniform(-8, -3, m)) ** 2
    return vx, c2, a
