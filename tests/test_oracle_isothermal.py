"""Pins of the oracle's no-slip isothermal wall (reading R32; the M2.9 ramp's wall,
Sec. 4): ghost images with velocity odd, pressure even and temperature odd about the
wall temperature, density from the equation of state."""
import numpy as np
import pytest

from oracle import derivatives as D, grid as gr, rhs as R
from paper_2511_18042_amd import cases

IT, NS, P = cases.NOSLIP_ISOTHERMAL, cases.NOSLIP, cases.PERIODIC


def _gas():
    return R.Gas(gamma=1.4, viscous=True, Re=500.0, Mref=0.7, Pr=0.72)


def _temperature(Q, gas):
    W = R.primitives(Q, gas.gamma)
    return gas.gamma * gas.Mref ** 2 * W[4] / W[0], W


def _wall_case(T_lo, T_hi, seed=3):
    c = cases.Case(2, (12, 10, 1), [(P, P), (IT, IT)], h=(0.1, 0.1, 1.0))
    cases.random_rough_state(c, seed=seed)
    c.wall_T = [(0.0, 0.0), (T_lo, T_hi)]
    return c


def test_ghost_pairs_mirror_velocity_and_pressure_and_average_to_the_wall_temperature():
    gas = _gas()
    c = _wall_case(2.5, 3.5)
    g = gr.Grid(c.ndim, c.n, c.bc, c.h, wall_T=c.wall_T)
    Q = c.Q.copy()
    gr.fill_ghosts_conserved(Q, g, gas)
    T, W = _temperature(Q, gas)
    gj, n = g.g[1], g.n[1]
    for side, Tw in ((0, 2.5), (1, 3.5)):
        for m in range(gj):
            dst = gj - 1 - m if side == 0 else gj + n + m
            src = gj + m if side == 0 else gj + n - 1 - m
            for q in (1, 2):
                np.testing.assert_allclose(W[q][:, dst], -W[q][:, src], rtol=1e-14, atol=1e-15)
            np.testing.assert_allclose(W[4][:, dst], W[4][:, src], rtol=1e-13)
            np.testing.assert_allclose(0.5 * (T[:, dst] + T[:, src]), Tw, rtol=1e-13)


def test_wall_at_the_local_temperature_gives_the_adiabatic_images():
    """Where the interior temperature equals the wall temperature, the isothermal and the
    adiabatic no-slip images coincide."""
    gas = _gas()
    c = _wall_case(1.0, 1.0, seed=5)
    W = R.primitives(c.Q, gas.gamma)
    Tw = 1.7
    rho = W[0]
    p = rho * Tw / (gas.gamma * gas.Mref ** 2)
    c.Q = cases.conserved(rho, W[1], W[2], W[3], p, gas.gamma)
    c.wall_T = [(0.0, 0.0), (Tw, Tw)]
    iso = c.Q.copy()
    gr.fill_ghosts_conserved(iso, gr.Grid(c.ndim, c.n, c.bc, c.h, wall_T=c.wall_T), gas)
    adi = c.Q.copy()
    gr.fill_ghosts_conserved(adi, gr.Grid(c.ndim, c.n, [(P, P), (NS, NS)], c.h))
    np.testing.assert_allclose(iso, adi, rtol=1e-13, atol=1e-15)


def test_linear_temperature_continues_through_the_ghosts():
    """Fluid at rest with T linear in y and the wall temperatures taken from that line at
    the wall faces (cell-centred nodes: the faces lie half a spacing outside the first and
    last nodes): the images continue the line, so the E4 derivative of T is the slope at
    every node, ghosts included."""
    gas = _gas()
    ny, h = 16, 0.05
    c = cases.Case(2, (8, ny, 1), [(P, P), (IT, IT)], h=(0.1, h, 1.0))
    _, y, _ = cases.cartesian_mesh(c)
    a, b = 2.0, 3.0                      # T = a + b y
    T = a + b * y
    p = np.full_like(T, 0.9)
    rho = gas.gamma * gas.Mref ** 2 * p / T
    z = np.zeros_like(T)
    c.Q = cases.conserved(rho, z, z, z, p, gas.gamma)
    y_lo, y_hi = c.x0[1], c.x0[1] + ny * h
    c.wall_T = [(0.0, 0.0), (a + b * y_lo, a + b * y_hi)]
    g = gr.Grid(c.ndim, c.n, c.bc, c.h, wall_T=c.wall_T)
    Q = c.Q.copy()
    gr.fill_ghosts_conserved(Q, g, gas)
    Tq, _ = _temperature(Q, gas)
    _, yy, _ = cases.cartesian_mesh(c)
    np.testing.assert_allclose(Tq, a + b * yy, rtol=1e-13)
    dT = D.e4(Tq, 1) / h
    sl = (slice(None), slice(2, -2), slice(None))
    np.testing.assert_allclose(dT[sl], b, rtol=1e-11)


def test_an_isothermal_wall_needs_the_gas_model():
    c = _wall_case(2.0, 2.0)
    with pytest.raises(ValueError):
        gr.fill_ghosts_conserved(c.Q.copy(), gr.Grid(c.ndim, c.n, c.bc, c.h, wall_T=c.wall_T))
