"""Pins of the oracle's mid-run change of the speed limit (the limit may
vary in time): the resampling keeps f = beta g.  A uniform box loaded as
g0 = f0/beta at one limit and raised to u = inf must hold a Maxwellian (the
PIC distribution); raised or lowered to another finite limit, the same
distribution as a fresh load there; the beta-weighted charge is kept within
its sampling noise; an unchanged limit changes nothing."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads


def _box(u, ppc=400, seed=50):
    return workloads.langmuir_box(u, nx=64, ppc=ppc, seed=seed, sort_every=0)


def _speeds(run, s):
    _, vx, vy, vz = run.particles(s)
    return np.sqrt(vx * vx + vy * vy + vz * vz)


def test_same_limit_is_identity():
    cfg = _box(0.5)
    run = oracle.Run(cfg)
    before = [run.particles(s) for s in range(2)]
    w = [run.weight(s) for s in range(2)]
    run.set_speed_limit(cfg["u"], cfg["dt"])
    for s in range(2):
        for a, b in zip(before[s], run.particles(s)):
            assert np.array_equal(a, b)
        assert run.weight(s) == w[s]
    for bad in ((0.0, cfg["dt"]), (-1.0, cfg["dt"]), (0.25, 0.0)):
        with pytest.raises(ValueError):
            run.set_speed_limit(*bad)


def test_raise_to_pic_gives_maxwellian():
    """From g0 = f0/beta at u = 0.5 v_te (speeds weighted by 1/beta, far
    from Maxwellian) to u = inf: the electrons' speeds follow the Maxwell
    distribution of unit thermal speed again, and the weight becomes dx/ppc."""
    cfg = _box(0.5, ppc=600)
    run = oracle.Run(cfg)
    sp0 = _speeds(run, 0)
    assert stats.kstest(sp0, stats.maxwell.cdf).pvalue < 1e-6  # g0 is not f0
    run.set_speed_limit(math.inf, cfg["dx"] / 5.0)
    sp = _speeds(run, 0)
    assert stats.kstest(sp, stats.maxwell.cdf).pvalue > 1e-3
    assert run.weight(0) == pytest.approx(cfg["dx"] / 600, rel=1e-14)
    # the expected count is that of a fresh load (the weight's normalisation)
    n = run.nslots(0)
    assert abs(n - 64 * 600) < 6 * math.sqrt(64 * 600)


def test_raise_matches_fresh_load():
    """From u = 0.3 to u = 1.0 v_te: the resampled electron speeds and a
    fresh load at u = 1.0 come from the same distribution (two-sample KS)."""
    a = oracle.Run(_box(0.3, ppc=600, seed=51))
    a.set_speed_limit(1.0, 0.5)
    b = oracle.Run(_box(1.0, ppc=600, seed=52))
    assert stats.ks_2samp(_speeds(a, 0), _speeds(b, 0)).pvalue > 1e-3
    assert a.weight(0) == pytest.approx(b.weight(0), rel=1e-14)


def test_charge_kept_within_noise():
    """The beta-weighted charge of each species before and after a rise from
    u = 0.2 to u = 2 v_te: equal totals within 5 sigma of the resampling
    noise (each particle's charge share is resampled independently)."""
    cfg = _box(0.2, ppc=400, seed=53)
    run = oracle.Run(cfg)
    q0 = run.grid()["Q"].copy()
    run.set_speed_limit(2.0, 0.25)
    q1 = run.grid()["Q"]
    for s in range(2):
        tot0, tot1 = q0[s].sum(), q1[s].sum()
        # a particle of charge share c = q w' beta' copied floor(p) or ceil(p)
        # times: variance c^2 frac(p)(1 - frac(p)) <= c^2 / 4 per particle
        c = abs(q1[s]).sum() / max(run.nslots(s), 1)
        sigma = c * math.sqrt(run.nslots(s)) / 2.0
        assert abs(tot1 - tot0) <= 5 * sigma + 1e-12 * abs(tot0), (s, tot0, tot1, sigma)


def test_lower_matches_fresh_load():
    """From u = 1.0 down to u = 0.3 v_te: the resampled electron speeds and
    a fresh load at u = 0.3 come from the same distribution (two-sample KS),
    with the fresh load's weight and, within noise, its count."""
    a = oracle.Run(_box(1.0, ppc=600, seed=54))
    a.set_speed_limit(0.3, 1.0)
    b = oracle.Run(_box(0.3, ppc=600, seed=55))
    assert stats.ks_2samp(_speeds(a, 0), _speeds(b, 0)).pvalue > 1e-3
    assert a.weight(0) == pytest.approx(b.weight(0), rel=1e-14)
    assert abs(a.nslots(0) - b.nslots(0)) < 6 * math.sqrt(b.nslots(0))


@pytest.mark.parametrize("u_new", [0.5, 0.05])
def test_lowering_keeps_f_within_noise(u_new):
    """Lowering from u = 2 v_te: the beta-weighted totals of w and of w |v|^2
    per species equal their values before within 5 sigma of the resampling
    noise, sigma^2 = sum over particles of (w' beta')^2 frac(p) (1 -
    frac(p)) (times |v|^4 for the energy), p = beta w / (beta' w')."""
    cfg = _box(2.0, ppc=300, seed=56)
    run = oracle.Run(cfg)

    def beta(u, s2):
        return np.minimum(1.0, u / np.sqrt(s2))

    before = []
    for s in range(2):
        _, vx, vy, vz = run.particles(s)
        before.append((vx * vx + vy * vy + vz * vz, run.weight(s)))
    run.set_speed_limit(u_new, 0.5)
    for s in range(2):
        s2, w = before[s]
        w1 = run.weight(s)
        p = beta(2.0, s2) * w / (beta(u_new, s2) * w1)
        fr = p - np.floor(p)
        c = w1 * beta(u_new, s2)
        _, vx, vy, vz = run.particles(s)
        s2n = vx * vx + vy * vy + vz * vz
        for k in (0, 1):  # moments |v|^0 and |v|^2
            m0 = np.sum(w * beta(2.0, s2) * s2 ** k)
            m1 = np.sum(w1 * beta(u_new, s2n) * s2n ** k)
            sigma = math.sqrt(np.sum((c * s2 ** k) ** 2 * fr * (1 - fr)))
            assert abs(m1 - m0) <= 5 * sigma + 1e-12 * m0, (s, k, m0, m1, sigma)
        assert np.all(p < 255)
