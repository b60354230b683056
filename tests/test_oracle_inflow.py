"""Pins of the oracle's digital-filter inflow generator (reading R33; Sec. 4's inflow)."""
import math

import numpy as np
import pytest

from oracle import grid as gr, inflow as DF
from paper_2511_18042_amd import cases


def _spec(ny=9, nz=12, y_lim=0.35):
    dy = np.linspace(0.05, 0.15, ny)
    y = np.cumsum(dy) - 0.5 * dy
    mean = np.stack([1.0 + 0.1 * y, 0.5 + y, 0.02 * y, 1.2 - 0.1 * y])
    R11 = 0.01 * (1.0 + y)
    R22 = 0.004 * (1.0 + y)
    R21 = -0.3 * np.sqrt(R11 * R22)
    R33 = 0.006 * (1.0 + y)
    return DF.DFSpec(dy, y, 0.1, y_lim, Iy=[(0.13, 0.23), (0.17, 0.3), (0.1, 0.13)], Iz=[0.15, 0.15, 0.3],
                     Ix=[0.7, 0.28, 0.28], U_ref=1.0, mean=mean, rey=np.stack([R11, R21, R22, R33]),
                     gamma=1.4, M_sra=2.9, p=1.0 / (1.4 * 2.9 ** 2))


@pytest.mark.parametrize('n', [0.3, 1.0, 2.5, 7.2])
def test_coefficients_unit_energy_symmetric_support(n):
    b = DF.df_coefficients(n)
    N = (b.size - 1) // 2
    assert N == math.ceil(2 * n)
    assert abs(np.sum(b * b) - 1.0) < 1e-14
    np.testing.assert_array_equal(b, b[::-1])
    assert np.all(np.diff(b[N:]) < 0)


def test_impulse_response_is_the_separable_product():
    """A unit impulse at padded row jp0, column k0 gives psi_new(j, k) =
    b_eta_j(jp0 - pad - j) b_zeta(k0 - k mod nz): the filters' indexing, padding and
    spanwise periodicity."""
    s = _spec()
    pad = s.pad()
    nz = 12
    for c in range(3):
        for jp0, k0 in ((pad + 2, 0), (pad + 4, 7), (3, 11)):
            r = np.zeros((3, s.ny + 2 * pad, nz))
            r[c, jp0, k0] = 1.0
            out = DF.filter_plane(s, r)
            assert np.all(out[[q for q in range(3) if q != c]] == 0.0)
            bz = DF.df_coefficients(s.Iz[c] / s.dz)
            Nz = (bz.size - 1) // 2
            for j, by in enumerate(s.eta_coefficients(c)):
                Ny = (by.size - 1) // 2
                for k in range(nz):
                    i = jp0 - pad - j
                    wz = sum(bz[l + Nz] for l in range(-Nz, Nz + 1) if (k + l - k0) % nz == 0)
                    want = (by[i + Ny] if abs(i) <= Ny else 0.0) * wz
                    assert abs(out[c, j, k] - want) <= 1e-15, (c, j, k)


def test_zones_pick_inner_and_outer_scales():
    s = _spec()
    for c in range(3):
        for j, b in enumerate(s.eta_coefficients(c)):
            I = s.Iy[c][0] if s.y[j] <= s.y_lim else s.Iy[c][1]
            np.testing.assert_array_equal(b, DF.df_coefficients(I / s.dy[j]))


def test_time_correlation_keeps_unit_variance():
    """psi <- psi e1 + new e2 with e1 = exp(-pi dt / 2T), e1^2 + e2^2 = 1: a stationary
    unit-variance field stays one with lag correlation e1."""
    s = _spec()
    dt = 0.013
    one = np.ones((3, s.ny, 4))
    e1 = DF.correlate(s, one, 0.0 * one, dt, first=False)
    e2 = DF.correlate(s, 0.0 * one, one, dt, first=False)
    for c in range(3):
        T = s.Ix[c] / s.U_ref
        assert abs(e1[c, 0, 0] - math.exp(-math.pi * dt / (2 * T))) < 1e-15
        assert abs(e1[c, 0, 0] ** 2 + e2[c, 0, 0] ** 2 - 1.0) < 1e-14
    np.testing.assert_array_equal(DF.correlate(s, one, 2 * one, dt, first=True), 2 * one)


def test_lund_transform_reproduces_the_reynolds_stresses():
    """Unit psi vectors map to the columns of the Cholesky factor: the covariance of
    (u', v', w') for uncorrelated unit psi is exactly R (R13 = R23 = 0)."""
    s = _spec(nz=1)
    base = DF.inflow_plane(s, np.zeros((3, s.ny, 1)))
    cols = []
    for c in range(3):
        psi = np.zeros((3, s.ny, 1))
        psi[c] = 1.0
        pl = DF.inflow_plane(s, psi)
        cols.append(np.stack([pl[1] - base[1], pl[2] - base[2], pl[3] - base[3]])[:, :, 0])
    A = np.stack(cols, axis=1)                      # (3 velocity, 3 psi, ny)
    cov = np.einsum('ipj,kpj->ikj', A, A)
    R11, R21, R22, R33 = s.rey
    np.testing.assert_allclose(cov[0, 0], R11, rtol=1e-13)
    np.testing.assert_allclose(cov[1, 0], R21, rtol=1e-13)
    np.testing.assert_allclose(cov[1, 1], R22, rtol=1e-13)
    np.testing.assert_allclose(cov[2, 2], R33, rtol=1e-13)
    assert np.all(cov[2, :2] == 0.0)


def test_strong_reynolds_analogy_and_uniform_pressure():
    """T'/T = -(gamma - 1) Mbar^2 u'/U with the local mean Mach number
    Mbar^2 = U^2 / c^2, c^2 = T / M_sra^2 (T in units of the reference temperature, the
    reference speed of sound U_ref / M_sra); density opposite at constant pressure."""
    s = _spec(nz=3)
    rng = np.random.default_rng(4)
    psi = rng.standard_normal((3, s.ny, 3))
    pl = DF.inflow_plane(s, psi)
    U, T = s.mean[1][:, None], s.mean[3][:, None]
    up = pl[1] - U
    c2 = T * (s.U_ref / s.M_sra) ** 2
    tr = -(s.gamma - 1.0) * (U ** 2 / c2) * up / U
    np.testing.assert_allclose(pl[0], s.mean[0][:, None] * (1.0 - tr), rtol=1e-13)
    assert np.all(pl[4] == s.p)


def test_ghost_write_touches_only_the_inflow_ghosts():
    c = cases.periodic_case(3, (10, 9, 12))
    c.bc = [(cases.FIXED, cases.TRANSMISSIVE), (cases.NOSLIP, cases.TRANSMISSIVE), (cases.PERIODIC, cases.PERIODIC)]
    cases.random_smooth_state(c, seed=2)
    g = gr.Grid(3, c.n, c.bc, c.h)
    s = _spec(ny=9, nz=12)
    Q = c.Q.copy()
    plane = DF.inflow_plane(s, np.random.default_rng(1).standard_normal((3, 9, 12)))
    DF.write_inflow_ghosts(Q, g, plane, 1.4)
    changed = np.any(Q != c.Q, axis=0)
    blk = np.zeros_like(changed)
    blk[5:17, 5:14, 0:5] = True
    assert np.all(changed <= blk) and changed[5:17, 5:14, 0:5].all()
    rho = Q[0, 5:17, 5:14, 0]
    np.testing.assert_allclose(rho, plane[0].T, rtol=1e-15)
