"""Pins of the oracle's exact Riemann solver (used for the shock-tube checks, Sec. 3.1)."""
import os

import numpy as np
import pytest

from oracle import riemann

GOLD = os.path.join(os.path.dirname(__file__), 'golden', 'toro_star_states.txt')


def _rows():
    return np.loadtxt(GOLD, comments='#')


@pytest.mark.parametrize('row', list(range(5)))
def test_star_state_matches_textbook_table(row):
    r = _rows()[row]
    left, right = tuple(r[0:3]), tuple(r[3:6])
    ps, us = riemann.star_state(left, right, 1.4)
    # printed to 5-6 significant digits
    assert abs(ps - r[6]) <= 6e-5 * max(1.0, abs(r[6]))
    assert abs(us - r[7]) <= 6e-5 * max(1.0, abs(r[7]))
    assert abs(riemann.residual(ps, left, right, 1.4)) < 1e-13 * max(1.0, abs(r[7]) + 1)


def test_single_shock_is_reproduced():
    """Mach-3 post/pre-shock states (Rankine-Hugoniot closed form) are joined by one right
    shock: the star state equals the post-shock state."""
    g = 1.4
    rho2 = 2.4 * 9.0 / 5.6          # (g+1) M^2 / ((g-1) M^2 + 2), M = 3
    p2 = (2 * g * 9.0 - (g - 1)) / (g + 1)
    u_s = 3.0 * np.sqrt(g)          # shock speed into rest gas with c = sqrt(g)
    u2 = u_s * (1.0 - 1.0 / rho2)
    assert abs(rho2 - 3.857142857) < 1e-9 and abs(p2 - 10.33333333) < 1e-8
    assert abs(u2 - 2.629368792) < 1e-9
    ps, us = riemann.star_state((rho2, u2, p2), (1.0, 0.0, 1.0), g)
    assert abs(ps - p2) < 1e-10 * p2 and abs(us - u2) < 1e-10
    # sampled: post state left of the shock, rest gas right of it
    s = np.array([u_s - 1e-6, u_s + 1e-6])
    out = riemann.sample((rho2, u2, p2), (1.0, 0.0, 1.0), g, s)
    assert np.allclose(out[:, 0], [rho2, u2, p2], rtol=1e-9)
    assert np.allclose(out[:, 1], [1.0, 0.0, 1.0], rtol=1e-9)


def test_sampled_solution_is_continuous_through_rarefaction():
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    s = np.linspace(-1.3, -0.05, 400)
    out = riemann.sample(left, right, 1.4, s)
    assert np.max(np.abs(np.diff(out[0]))) < 0.01
    # isentropic: p / rho^gamma constant in the fan
    ent = out[2] / out[0] ** 1.4
    assert np.allclose(ent, 1.0, rtol=1e-12)
