"""Pins of the oracle's time step, Runge-Kutta scheme, raw LAD coefficients and viscosity law
against closed forms that do not come from the oracle itself.

* CFL time step (reading R8): on a Cartesian grid the contravariant spectral radius of
  direction l is (|u_l| + c) / h_l; on an affine grid x = A xi it is |a_l . u| + c |a_l|
  with a_l the rows of A^-1.  dt = CFL / max over nodes of their sum.
* SSP-RK3 (Sec. 2.3, third-order TVD Runge-Kutta): applied to dQ/dt = lambda Q its
  amplification factor is the cubic Taylor polynomial 1 + z + z^2/2 + z^3/6 (z = lambda dt),
  and on the Euler equations the error of a fixed spatial discretisation falls as dt^3.
  Marched with dt ~ h^(4/3) the whole method keeps its fourth spatial order (R1).
* Raw mu*, beta*, kappa* (Sec. 2.2): on fields whose fourth differences are known exactly
  (quartic e, theta from a quintic velocity whose E4 derivative is exact up to a constant)
  each coefficient has a closed form in rho, c, T and the spacing.
* Sutherland's law (Sec. 2.1): the tabulated viscosity of air and the kinetic-theory limits
  mu ~ T^(1/2) far above and mu ~ T^(3/2) far below the Sutherland temperature.
"""
import numpy as np
import pytest

from oracle import grid as gr, lad, rhs as R
from oracle.derivatives import gradient
from paper_2511_18042_amd import cases


# ------------------------------------------------------------------ CFL time step
def _state_with_hot_node(c, seed):
    rng = np.random.default_rng(seed)
    shape = c.shape
    rho = 0.5 + rng.random(shape)
    u = rng.uniform(-1, 1, shape)
    v = rng.uniform(-1, 1, shape) if c.ndim > 1 else 0 * rho
    w = rng.uniform(-1, 1, shape) if c.ndim > 2 else 0 * rho
    p = 0.5 + rng.random(shape)
    # one interior node far faster than the rest decides the maximum
    idx = tuple(s // 2 for s in shape)
    u[idx] = 3.0
    p[idx] = 5.0
    return rho, u, v, w, p


@pytest.mark.parametrize('ndim,h', [(1, (0.05,)), (2, (0.05, 0.02)), (3, (0.1, 0.03, 0.07))])
def test_cfl_dt_cartesian_closed_form(ndim, h):
    n = (9, 7, 6)[:ndim]
    c = cases.Case(ndim, tuple(list(n) + [1] * (3 - ndim)), [(cases.TRANSMISSIVE,) * 2] * ndim,
                   h=tuple(list(h) + [1.0] * (3 - ndim)))
    rho, u, v, w, p = _state_with_hot_node(c, 11)
    gamma = 1.4
    c.Q = cases.conserved(rho, u, v, w, p, gamma)
    g = gr.Grid(ndim, c.n, c.bc, c.h)
    dt = R.cfl_dt(c.Q, g, R.Gas(gamma=gamma), 0.3)
    inner = g.interior()
    snd = np.sqrt(gamma * p / rho)
    vel = (u, v, w)
    s = sum((np.abs(vel[l]) + snd) / h[l] for l in range(ndim))
    assert dt == pytest.approx(0.3 / np.max(s[inner]), rel=1e-14)


def test_cfl_dt_affine_grid_closed_form():
    """Sheared, stretched 2D grid x = A (i, j): the metric terms are the rows of A^-1."""
    A = np.array([[0.04, 0.01], [-0.005, 0.02]])
    n = (10, 8)
    c = cases.Case(2, (n[0], n[1], 1), [(cases.TRANSMISSIVE,) * 2] * 2)
    i = np.arange(-cases.NG, n[0] + cases.NG)
    j = np.arange(-cases.NG, n[1] + cases.NG)
    J, I = np.meshgrid(j, i, indexing='ij')
    x = A[0, 0] * I + A[0, 1] * J
    y = A[1, 0] * I + A[1, 1] * J
    c.coords = np.stack([x, y, 0 * x])[:, None]
    rho, u, v, w, p = _state_with_hot_node(c, 5)
    gamma = 1.4
    c.Q = cases.conserved(rho, u, v, w, p, gamma)
    g = gr.Grid(2, c.n, c.bc, coords=c.coords)
    dt = R.cfl_dt(c.Q, g, R.Gas(gamma=gamma), 0.2)
    Ainv = np.linalg.inv(A)
    snd = np.sqrt(gamma * p / rho)
    s = sum(np.abs(Ainv[l, 0] * u + Ainv[l, 1] * v) + snd * np.hypot(Ainv[l, 0], Ainv[l, 1]) for l in range(2))
    assert dt == pytest.approx(0.2 / np.max(s[g.interior()]), rel=1e-12)


# ------------------------------------------------------------------ SSP-RK3
def test_ssp_rk3_amplification_is_cubic_taylor_polynomial(monkeypatch):
    """With L(Q) = lambda Q the three stages must give (1 + z + z^2/2 + z^3/6) Q exactly."""
    c = cases.entropy_wave(8)
    g = gr.Grid(1, c.n, c.bc, c.h)
    lam = -1.7
    monkeypatch.setattr(R, 'rhs', lambda Q, *a, **k: lam * Q)
    dt = 0.3
    U = c.Q
    for s in range(3):
        U = R.rk3_stage(c.Q, U, dt, s, g, R.Gas(), R.Opts(), 'lad')
    z = lam * dt
    amp = 1 + z + z * z / 2 + z ** 3 / 6
    inner = (slice(None),) + g.interior()
    assert np.allclose(U[inner], amp * c.Q[inner], rtol=1e-15, atol=0)


def _march_fixed_dt(c, scheme, opts, dt, t_end):
    g = gr.Grid(c.ndim, c.n, c.bc, c.h)
    M = gr.node_metrics(g)
    steps = int(round(t_end / dt))
    Q = c.Q.copy()
    for _ in range(steps):
        U = Q
        for s in range(3):
            U = R.rk3_stage(Q, U, dt, s, g, R.Gas(), opts, scheme, M)
        Q = U
    return Q, g


def test_ssp_rk3_error_is_third_order_in_dt():
    """Fixed grid (32 nodes, central E4 fluxes, no artificial terms): the state at t = 0.4
    differs from a 16x finer time march by O(dt^3)."""
    c = cases.entropy_wave(32)
    opts = R.Opts(C_beta=0.0, C_kappa=0.0, C_mu=0.0)
    ref, g = _march_fixed_dt(c, 'lad', opts, 0.4 / 320, 0.4)
    inner = (slice(None),) + g.interior()
    errs = []
    for nst in (10, 20, 40):
        Q, _ = _march_fixed_dt(c, 'lad', opts, 0.4 / nst, 0.4)
        errs.append(np.max(np.abs(Q[inner] - ref[inner])))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 3.0) < 0.25), (errs, orders)


def test_time_marched_entropy_wave_keeps_fourth_order_with_dt_h43():
    """MEG6 C-GBR marched to t = 0.25 with dt = 0.33 h^(4/3): L1 density error against the
    exact advected wave falls at fourth order (R1: the flux difference is fourth order)."""
    errs = []
    for n in (16, 32, 64):
        c = cases.entropy_wave(n)
        h = 1.0 / n
        nst = int(np.ceil(0.25 / (0.33 * h ** (4.0 / 3.0))))
        Q, g = _march_fixed_dt(c, 'cgbr', R.Opts(grad='E6'), 0.25 / nst, 0.25)
        ex = cases.entropy_wave(n, t=0.25).Q
        inner = g.interior()
        errs.append(np.mean(np.abs(Q[0][inner] - ex[0][inner])))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 3.6), (errs, orders)


# ------------------------------------------------------------------ raw LAD coefficients
def _line(n, h, bc=cases.TRANSMISSIVE):
    c = cases.Case(1, (n, 1, 1), [(bc, bc)], h=(h, 1.0, 1.0))
    x, _, _ = cases.cartesian_mesh(c)
    return c, x


def _raw(W, g, gas, opts):
    M = gr.node_metrics(g)
    G4 = {l: np.stack([gradient(W[q], l, 'E4', g) for q in range(5)]) for l in range(g.ndim)}
    return lad.lad_coefficients(W, G4, M, g, gas, opts, raw_only=True)


def test_raw_kappa_star_closed_form():
    """rho uniform, p quartic in x: e = p / ((gamma-1) rho) has fourth difference
    24 a4 h^4 / ((gamma-1) rho) and Delta_kappa = |Delta x . grad e / |grad e|| = h, so
    kappa*_raw = C_kappa (rho c / T) 24 |a4| h^5 / ((gamma-1) rho), T = gamma M^2 p / rho."""
    h, gamma, Mref, a4, rho0 = 0.05, 1.4, 2.0, 3.0, 0.8
    c, x = _line(24, h)
    g = gr.Grid(1, c.n, c.bc, c.h)
    p = 1.0 + 0.5 * x + a4 * x ** 4
    rho = rho0 + 0 * x
    W = np.stack([rho, 0 * x, 0 * x, 0 * x, p])
    gas = R.Gas(gamma=gamma, Mref=Mref)
    kap = _raw(W, g, gas, R.Opts(C_kappa=0.01))[2]
    snd = np.sqrt(gamma * p / rho)
    T = gamma * Mref ** 2 * p / rho
    expect = 0.01 * rho * snd / T * 24.0 * a4 * h ** 5 / ((gamma - 1.0) * rho0)
    inner = g.band(2, -2)        # the fourth difference reaches two nodes
    assert np.allclose(kap[inner], expect[inner], rtol=1e-9, atol=0)


def test_raw_beta_and_mu_star_closed_form():
    """u = a x^5 + b x with theta < 0: E4 returns u' - (h^4/30) u''''' = 5a x^4 + b - 4a h^4
    exactly, so delta^4 theta = 120 a h^4 (index space); in 1D f_sw = 1 where theta < 0 and
    |S| = |theta|.  With rho linear, Delta_beta = Delta_mu = h:
    beta*_raw = C_beta rho 120 |a| h^6 and mu*_raw = C_mu rho 120 |a| h^6."""
    h, a, b = 0.04, -2.0, -0.5
    c, x = _line(30, h)
    g = gr.Grid(1, c.n, c.bc, c.h)
    u = a * x ** 5 + b * x
    rho = 1.0 + 0.3 * x
    W = np.stack([rho, u, 0 * x, 0 * x, 1.0 + 0 * x])
    mu, beta, _ = _raw(W, g, R.Gas(), R.Opts(C_mu=0.002, C_beta=1.75, C_kappa=0.0))
    inner = g.band(2, -2)
    assert np.allclose(beta[inner], (1.75 * rho * 120 * abs(a) * h ** 6)[inner], rtol=1e-7, atol=0)
    assert np.allclose(mu[inner], (0.002 * rho * 120 * abs(a) * h ** 6)[inner], rtol=1e-7, atol=0)


def test_raw_coefficients_along_second_direction_use_its_spacing():
    """The same quartic pressure along y on a grid with h_x != h_y: Delta_kappa = h_y."""
    hx, hy, a4 = 0.1, 0.03, 2.0
    c = cases.Case(2, (7, 26, 1), [(cases.TRANSMISSIVE,) * 2] * 2, h=(hx, hy, 1.0))
    _, y, _ = cases.cartesian_mesh(c)
    g = gr.Grid(2, c.n, c.bc, c.h)
    p = 1.0 + 0.2 * y + a4 * y ** 4
    W = np.stack([1.0 + 0 * y, 0 * y, 0 * y, 0 * y, p])
    gas = R.Gas(gamma=1.4)
    kap = _raw(W, g, gas, R.Opts(C_kappa=0.01))[2]
    snd = np.sqrt(1.4 * p)
    T = 1.4 * p
    expect = 0.01 * snd / T * 24.0 * a4 * hy ** 5 / 0.4
    inner = g.band(2, -2)
    assert np.allclose(kap[inner], expect[inner], rtol=1e-9, atol=0)


# ------------------------------------------------------------------ Sutherland
def test_sutherland_matches_tabulated_air_viscosity():
    """Air: mu(273.15 K) = 1.716e-5 Pa s, S = 110.4 K; tabulated mu(300 K) = 1.846e-5 and
    mu(500 K) = 2.671e-5 Pa s (four significant digits)."""
    Tref, S = 273.15, 110.4
    for T, mu in ((300.0, 1.846e-5), (500.0, 2.671e-5)):
        ratio = lad.sutherland(T / Tref, S / Tref)
        assert ratio * 1.716e-5 == pytest.approx(mu, rel=1.5e-3)


def test_sutherland_kinetic_theory_limits():
    S = 110.4 / 108.0
    hot = lad.sutherland(4e6, S) / lad.sutherland(1e6, S)
    cold = lad.sutherland(4e-7, S) / lad.sutherland(1e-7, S)
    assert hot == pytest.approx(2.0, rel=1e-5)        # mu ~ T^(1/2) for T >> S
    assert cold == pytest.approx(8.0, rel=1e-5)       # mu ~ T^(3/2) for T << S
    assert lad.sutherland(1.0, S) == 1.0


# ------------------------------------------------------------------ classic RK4 (R38)
def test_rk4_amplification_is_quartic_taylor_polynomial(monkeypatch):
    """With L(Q) = lambda Q the four stages must give (1 + z + z^2/2 + z^3/6 + z^4/24) Q."""
    c = cases.entropy_wave(8)
    g = gr.Grid(1, c.n, c.bc, c.h)
    lam = -1.3
    monkeypatch.setattr(R, 'rhs', lambda Q, *a, **k: lam * Q)
    dt = 0.4
    U, _ = R.rk4_stages(c.Q, dt, g, R.Gas(), R.Opts(filter_alpha=0.5), 'lad')
    z = lam * dt
    amp = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    inner = (slice(None),) + g.interior()
    assert np.allclose(U[inner], amp * c.Q[inner], rtol=1e-15, atol=0)


def test_rk4_error_is_fourth_order_in_dt():
    """Fixed grid (32 nodes, central E4 fluxes, no artificial terms, no filter): the state at
    t = 0.4 differs from a 16x finer RK4 march by O(dt^4)."""
    c = cases.entropy_wave(32)
    opts = R.Opts(C_beta=0.0, C_kappa=0.0, C_mu=0.0, filter_alpha=0.5)
    g = gr.Grid(c.ndim, c.n, c.bc, c.h)
    M = gr.node_metrics(g)

    def march(nst):
        Q = c.Q.copy()
        for _ in range(nst):
            Q, _ = R.rk4_stages(Q, 0.4 / nst, g, R.Gas(), opts, 'lad', M)
        return Q
    ref = march(160)
    inner = (slice(None),) + g.interior()
    errs = [np.max(np.abs(march(n)[inner] - ref[inner])) for n in (5, 10, 20)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 4.0) < 0.3), (errs, orders)


def test_rk4_step_filters_once_after_the_fourth_stage():
    """The LAD-C6 RK4 step equals the unfiltered RK4 step followed by one filter pass, and
    RK4 refuses the other schemes."""
    from oracle.implicit_filter import filter_state
    c = cases.random_smooth_state(cases.periodic_case(2, (24, 16, 1)), seed=5)
    g = gr.Grid(c.ndim, c.n, c.bc, c.h)
    M = gr.node_metrics(g)
    gas = R.Gas()
    opts = R.Opts(lad='C6', time_scheme='rk4')
    Qf, _, dt, bad = R.time_step(c.Q, 0.0, 1.0, g, gas, opts, 'lad', M)
    assert bad == 0
    Qu, _ = R.rk4_stages(c.Q, dt, g, gas, R.Opts(lad='C6', filter_alpha=0.5), 'lad', M)
    inner = (slice(None),) + g.interior()
    want = filter_state(Qu, g, opts.filter_alpha, gas=gas)
    assert np.array_equal(Qf[inner], want[inner])
    assert np.max(np.abs(Qf[inner] - Qu[inner])) > 0
    with pytest.raises(ValueError):
        R.rk4_step(c.Q, 0.0, 1.0, g, gas, opts, 'cgbr', M)
