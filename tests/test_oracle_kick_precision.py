"""The oracle's FP64 velocity map (Eq. A2a, exact frozen-field integral)
against the same map in 40-digit arithmetic: its worst absolute error over
random and worst-conditioned cases (slowed through zero with a tiny
perpendicular speed) stays at a few ulps of the speeds involved, a thousand
times below the 1e-11 floor the GPU parity tests allow."""
import math

import numpy as np
import pytest

import mp_kick
import oracle


@pytest.mark.parametrize("kind", ["step", "smooth"])
@pytest.mark.parametrize("u,dt", [(0.05, 3.0), (1.0, 0.7)])
def test_oracle_velocity_map_rounding_error(kind, u, dt):
    vx, c2, a = mp_kick.hard_cases(400, seed=1)
    worst = 0.0
    for i in range(len(vx)):
        got = oracle.kick_exact(kind, u, dt, [vx[i], math.sqrt(c2[i]), 0.0], [a[i], 0.0, 0.0])[0]
        want = mp_kick.kick(kind, u, dt, vx[i], c2[i], a[i])
        scale = max(1.0, abs(want), abs(vx[i]))
        worst = max(worst, abs(got - want) / scale)
    assert worst <= 1e-14, worst
