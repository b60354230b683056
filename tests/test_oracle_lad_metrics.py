"""Pins of the oracle's LAD coefficients / Gaussian filter (Sec. 2.2) and grid metrics (Sec. 2.1)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import grid as gr, lad, rhs as R
from oracle.derivatives import gradient
from paper_2511_18042_amd import cases


def test_gaussian_weights_sum_and_nyquist_exact():
    w = lad.GAUSS_FRAC
    assert w[0] + 2 * sum(w[1:]) == Fraction(1)
    assert w[0] + 2 * sum(((-1) ** k) * w[k] for k in range(1, 5)) == Fraction(0)
    # second moment of the kernel is positive (a low-pass smoother)
    assert sum(2 * k * k * w[k] for k in range(1, 5)) > 0


def test_gaussian_pass_preserves_constants_and_kills_nyquist():
    g = gr.Grid(1, (32,), [(gr.BC_PERIODIC, gr.BC_PERIODIC)])
    f = np.full(g.shape, 3.0)
    assert np.allclose(lad.gaussian_pass(f, 0, g), 3.0, atol=1e-15)
    i = np.arange(g.shape[-1])
    f = np.cos(np.pi * (i - 5))[None, None, :].astype(float)
    assert np.max(np.abs(lad.gaussian_pass(f, 0, g))) < 1e-15


def _lin_case(ndim, n):
    c = cases.Case(ndim, tuple(list(n) + [1] * (3 - len(n))), [(cases.TRANSMISSIVE,) * 2] * ndim,
                   h=tuple([1.0 / 16] * ndim + [1.0] * (3 - ndim)))
    x, y, z = cases.cartesian_mesh(c)
    return c, x, y, z


@pytest.mark.parametrize('ndim', [1, 2, 3])
def test_lad_coefficients_vanish_on_linear_fields(ndim):
    """All fourth differences of a field linear in x vanish, so mu*, beta*, kappa* = 0."""
    c, x, y, z = _lin_case(ndim, [12] * ndim)
    g = gr.Grid(ndim, c.n, [(gr.BC_PERIODIC,) * 2] * ndim, c.h)
    rho = 1.0 + 0.1 * x
    u = 0.2 - 0.3 * x + (0.1 * y if ndim > 1 else 0)
    v = 0.1 + 0.2 * x if ndim > 1 else 0 * x
    p = 1.0 + 0.05 * x
    W = np.stack([rho, u, v, 0 * x, p])
    # linear p/rho is not linear; use e-linear check separately: here rho, u, v, p linear
    M = gr.node_metrics(g)
    G4 = {l: np.stack([gradient(W[q], l, 'E4', g) for q in range(5)]) for l in range(ndim)}
    coef = lad.lad_coefficients(W, G4, M, g, R.Gas(), R.Opts(C_mu=0.002), raw_only=True)
    inner = g.interior()
    assert np.max(np.abs(coef[0][inner])) < 1e-13     # |S| constant
    assert np.max(np.abs(coef[1][inner])) < 1e-13     # theta constant


def test_switch_is_zero_under_expansion_and_uniform_flow():
    c, x, _, _ = _lin_case(1, [24])
    g = gr.Grid(1, c.n, [(gr.BC_TRANSMISSIVE,) * 2], c.h)
    M = gr.node_metrics(g)
    # expansion: theta > 0 everywhere, large fourth differences in theta
    W = np.stack([1 + 0 * x, 0.5 * np.sin(3 * x) + 2 * x, 0 * x, 0 * x, 1 + 0 * x])
    G4 = {0: np.stack([gradient(W[q], 0, 'E4', g) for q in range(5)])}
    th = G4[0][1] * M[9] * M[0]
    assert np.all(th[g.interior()] > 0)
    coef = lad.lad_coefficients(W, G4, M, g, R.Gas(), R.Opts(), raw_only=True)
    assert np.all(coef[1] == 0.0)
    # uniform flow: all coefficients vanish
    W = np.stack([1 + 0 * x, 0.3 + 0 * x, 0 * x, 0 * x, 1 + 0 * x])
    G4 = {0: np.stack([gradient(W[q], 0, 'E4', g) for q in range(5)])}
    coef = lad.lad_coefficients(W, G4, M, g, R.Gas(), R.Opts(C_mu=0.002))
    assert all(np.all(cf == 0.0) for cf in coef)


def test_bulk_viscosity_switches_on_in_compression():
    c, x, _, _ = _lin_case(1, [40])
    g = gr.Grid(1, c.n, [(gr.BC_TRANSMISSIVE,) * 2], c.h)
    M = gr.node_metrics(g)
    s = np.tanh((x - 1.25) * 20)
    u = -s                                 # converging flow with a density rise
    W = np.stack([1.5 + 0.5 * s, u, 0 * x, 0 * x, 1 + 0 * x])
    G4 = {0: np.stack([gradient(W[q], 0, 'E4', g) for q in range(5)])}
    coef = lad.lad_coefficients(W, G4, M, g, R.Gas(), R.Opts())
    assert np.max(coef[1][g.interior()]) > 1e-4
    # with a uniform density the length scale Delta_beta = |dx . grad rho / |grad rho|| is zero
    W[0] = 1.0
    G4 = {0: np.stack([gradient(W[q], 0, 'E4', g) for q in range(5)])}
    assert np.all(lad.lad_coefficients(W, G4, M, g, R.Gas(), R.Opts())[1] == 0.0)


@pytest.mark.parametrize('ndim', [2, 3])
def test_metric_identity_on_wavy_periodic_grid(ndim):
    n = (16, 12, 10)[:ndim]
    c = cases.periodic_case(ndim, n, curvilinear=True, amp=0.08)
    g = gr.Grid(ndim, c.n, c.bc, c.h, c.coords)
    M = gr.node_metrics(g)
    sl = g.band(-3, 3)
    for j in range(3):
        s = sum(gr.d4(M[3 * l + j], l) for l in range(ndim))
        assert np.max(np.abs(s[g.band(-1, 1)])) < 1e-14
    # metrics of an affine map are exact: Jacobian determinant positive
    assert np.all(M[9][sl] > 0)


def test_cartesian_metrics_of_affine_coords_match_closed_form():
    c = cases.Case(3, (8, 7, 6), [(cases.PERIODIC,) * 2] * 3, h=(0.1, 0.2, 0.3))
    x, y, z = cases.cartesian_mesh(c)
    gc = gr.Grid(3, c.n, c.bc, c.h, np.stack([x, y, z]))
    gcart = gr.Grid(3, c.n, c.bc, c.h)
    Mc, M0 = gr.node_metrics(gc), gr.node_metrics(gcart)
    sl = gc.band(-3, 3)
    assert np.allclose(Mc[(slice(None),) + sl], M0[(slice(None),) + sl], rtol=1e-13, atol=1e-15)
