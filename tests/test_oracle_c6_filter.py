"""Pins of the LAD-C6 pieces of the oracle: C6 gradients, compact interface fluxes and
the tenth-order implicit filter (readings R27-R29).

Each pin is fixed by mathematics that the oracle does not use itself: the modified
wavenumber of the compact scheme, the closed-form transfer function of the
maximal-order filter, polynomial exactness, telescoping sums and brute-force dense
solves of the bounded systems.
"""
import numpy as np
import pytest

from oracle import derivatives as D, implicit_filter as IF, lad, rhs as R
from oracle.grid import Grid, BC_PERIODIC, BC_TRANSMISSIVE, BC_REFLECTIVE, fill_ghosts_conserved
from paper_2511_18042_amd import cases


# ----------------------------------------------------------------- C6 gradients
def c6_wavenumber(k):
    """Modified wavenumber of the sixth-order compact first derivative (unit spacing):
    [a sin k + (b/2) sin 2k] / (1 + 2 alpha cos k), alpha = 1/3, a = 14/9, b = 1/9."""
    return (14.0 / 9.0 * np.sin(k) + 1.0 / 18.0 * np.sin(2 * k)) / (1.0 + 2.0 / 3.0 * np.cos(k))


@pytest.mark.parametrize('n,m', [(16, 1), (16, 3), (24, 7), (40, 11)])
def test_c6_periodic_sine_has_the_compact_modified_wavenumber(n, m):
    g = Grid(1, (n,), [(BC_PERIODIC, BC_PERIODIC)])
    k = 2 * np.pi * m / n
    x = np.arange(-5, n + 5, dtype=float)
    f = np.sin(k * x + 0.3)[None, None, :]
    got = D.gradient(f, 0, 'C6', g)[0, 0]
    ref = c6_wavenumber(k) * np.cos(k * x + 0.3)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_c6_observed_order_on_periodic_sines():
    errs = []
    for n in (16, 32, 64):
        g = Grid(1, (n,), [(BC_PERIODIC, BC_PERIODIC)], h=(1.0 / n,))
        x = (np.arange(-5, n + 5) + 0.5) / n
        got = D.gradient(np.sin(2 * np.pi * x)[None, None, :], 0, 'C6', g)[0, 0, 5:5 + n] * n
        errs.append(np.max(np.abs(got - 2 * np.pi * np.cos(2 * np.pi * x[5:5 + n]))))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 6) < 0.25), orders


def _dense_c6_bounded(N):
    A = np.eye(N)
    for i in range(1, N - 1):
        a = 0.25 if i in (1, N - 2) else 1.0 / 3.0
        A[i, i - 1] = A[i, i + 1] = a
    return A


@pytest.mark.parametrize('N', [6, 7, 9, 14, 23])
def test_c6_bounded_matches_dense_solve(N):
    rng = np.random.default_rng(N)
    f = rng.normal(size=(N, 3))
    rhs = np.empty_like(f)
    for i in range(N):
        if i == 0:
            rhs[i] = (-3 * f[0] + 4 * f[1] - f[2]) / 2
        elif i == N - 1:
            rhs[i] = (3 * f[N - 1] - 4 * f[N - 2] + f[N - 3]) / 2
        elif i in (1, N - 2):
            rhs[i] = 0.75 * (f[i + 1] - f[i - 1])
        else:
            rhs[i] = 7 / 9 * (f[i + 1] - f[i - 1]) + (f[i + 2] - f[i - 2]) / 36
    ref = np.linalg.solve(_dense_c6_bounded(N), rhs)
    assert np.max(np.abs(D.c6_bounded_lines(f) - ref)) <= 1e-14 * max(1.0, np.abs(ref).max())


def test_c6_bounded_line_exact_on_quadratics():
    x = np.linspace(-1.3, 2.1, 31)
    h = x[1] - x[0]
    for k in range(3):
        got = D.c6_bounded_lines((x ** k)[:, None])[:, 0] / h
        ref = k * x ** (k - 1) if k else 0 * x
        assert np.allclose(got, ref, atol=1e-12)


def test_c6_bounded_centre_matches_the_modified_wavenumber():
    """Far from the closure rows (decay 0.38197 per node) a bounded line is the periodic
    scheme: the centre of a long line sees the modified wavenumber."""
    N, k = 161, 0.7
    x = np.arange(N, dtype=float)
    got = D.c6_bounded_lines(np.sin(k * x)[:, None])[:, 0]
    c = N // 2
    assert abs(got[c] - c6_wavenumber(k) * np.cos(k * x[c])) < 1e-14


# ----------------------------------------------------------------- compact fluxes
def _line_grid(n, periodic):
    bc = (BC_PERIODIC, BC_PERIODIC) if periodic else (BC_TRANSMISSIVE, BC_TRANSMISSIVE)
    return Grid(1, (n,), [bc])


@pytest.mark.parametrize('n,m', [(16, 2), (32, 5)])
def test_c6_face_differences_are_the_c6_derivative_on_periodic_lines(n, m):
    g = _line_grid(n, True)
    k = 2 * np.pi * m / n
    x = np.arange(-5, n + 5, dtype=float)
    F = np.sin(k * x - 0.2)[None, None, None, :]
    Fh = lad.c6_faces(F, 0, g)[0, 0, 0]
    dF = Fh[5:5 + n] - Fh[4:4 + n]
    assert np.max(np.abs(dF - c6_wavenumber(k) * np.cos(k * x[5:5 + n] - 0.2))) < 1e-13


def test_c6_faces_bounded_telescope_to_the_boundary_i4_fluxes():
    """Conservation: the interior sum of the differences is F_{n-1/2} - F_{-1/2}, and the
    two boundary faces are the I4 values of the node fluxes."""
    n = 23
    g = _line_grid(n, False)
    rng = np.random.default_rng(5)
    F = rng.normal(size=(2, 1, 1, n + 10))
    Fh = lad.c6_faces(F, 0, g)
    dF = Fh[..., 5:5 + n] - Fh[..., 4:4 + n]
    i4 = lambda i: (7 * (F[..., 5 + i] + F[..., 6 + i]) - (F[..., 4 + i] + F[..., 7 + i])) / 12  # noqa: E731
    assert np.allclose(Fh[..., 4], i4(-1), rtol=0, atol=1e-15)
    assert np.allclose(Fh[..., 4 + n], i4(n - 1), rtol=0, atol=1e-15)
    assert np.allclose(dF.sum(axis=-1), i4(n - 1) - i4(-1), rtol=0, atol=1e-13)


def test_c6_faces_bounded_matches_dense_solve():
    n = 13
    g = _line_grid(n, False)
    rng = np.random.default_rng(8)
    F = rng.normal(size=n + 10)
    P = lambda i: F[5 + i]  # noqa: E731
    faces = list(range(-1, n))           # face i+1/2
    A = np.eye(len(faces))
    b = np.zeros(len(faces))
    for r, i in enumerate(faces):
        if i in (-1, n - 1):
            b[r] = (7 * (P(i) + P(i + 1)) - (P(i - 1) + P(i + 2))) / 12
        else:
            A[r, r - 1] = A[r, r + 1] = 1 / 3
            b[r] = 29 / 36 * (P(i) + P(i + 1)) + (P(i - 1) + P(i + 2)) / 36
    ref = np.linalg.solve(A, b)
    got = lad.c6_faces(F[None, None, None, :], 0, g)[0, 0, 0, 4:5 + n]
    assert np.max(np.abs(got - ref)) < 1e-14


def test_c6_faces_exact_derivative_of_cubics_on_bounded_lines():
    """Both the I4 ends and the compact rows are exact for low-degree polynomials, so the
    face differences reproduce F' of a cubic at every interior node."""
    n = 20
    g = _line_grid(n, False)
    x = np.arange(-5, n + 5, dtype=float) * 0.1 - 0.4
    for k in range(4):
        F = (x ** k)[None, None, None, :]
        Fh = lad.c6_faces(F, 0, g)[0, 0, 0]
        dF = (Fh[5:5 + n] - Fh[4:4 + n]) / 0.1
        ref = k * x[5:5 + n] ** (k - 1) if k else 0 * x[5:5 + n]
        assert np.max(np.abs(dF - ref)) < 1e-11, k


# ----------------------------------------------------------------- implicit filter
@pytest.mark.parametrize('alpha', [0.0, 0.3, 0.45, 0.49, 0.499])
def test_filter_transfer_function_closed_form(alpha):
    """The maximal-order tenth-order filter has T(w) = 1 - (1 - 2 alpha) sin^10(w/2) /
    (1 + 2 alpha cos w): a cosine polynomial of degree 5 over the tridiagonal symbol,
    zero at w = pi and flat to O(w^10) at w = 0."""
    w = np.linspace(0.0, np.pi, 41)
    coef = IF.gv_coefficients(alpha)
    ref = 1.0 - (1.0 - 2 * alpha) * np.sin(w / 2) ** 10 / (1.0 + 2 * alpha * np.cos(w))
    assert np.max(np.abs(IF.transfer(w, alpha, coef) - ref)) < 1e-13


def test_filter_identity_at_alpha_one_half():
    assert IF.gv_coefficients(0.5) == (1.0, 1.0, 0.0, 0.0, 0.0, 0.0)


def test_filter_explicit_member_is_the_tenth_difference():
    """alpha = 0: phi^ = phi - 2^-10 delta^10 phi (binomial weights, alternating)."""
    coef = IF.gv_coefficients(0.0)
    from math import comb
    ref = [1 - comb(10, 5) / 1024.0] + [(-1) ** (k + 1) * 2 * comb(10, 5 - k) / 1024.0 for k in range(1, 6)]
    assert np.allclose(coef, ref, rtol=0, atol=1e-16)


@pytest.mark.parametrize('n,m', [(32, 1), (32, 7), (32, 16), (48, 13)])
def test_filter_scales_periodic_modes_by_the_transfer_function(n, m):
    g = Grid(1, (n,), [(BC_PERIODIC, BC_PERIODIC)])
    w = 2 * np.pi * m / n
    x = np.arange(-5, n + 5, dtype=float)
    Q = np.zeros((5, 1, 1, n + 10))
    Q[0] = 2.0 + 0.1 * np.cos(w * x + 0.4)
    Q[4] = 3.0
    out = IF.filter_state(Q, g, 0.49)
    T = 1 - 0.02 * np.sin(w / 2) ** 10 / (1 + 0.98 * np.cos(w))
    ref = 2.0 + 0.1 * T * np.cos(w * x + 0.4)
    # the tridiagonal symbol 1 + 2 alpha cos w falls to 0.02 at the Nyquist mode
    assert np.max(np.abs(out[0, 0, 0, 5:5 + n] - ref[5:5 + n])) < 1e-13


def test_filter_keeps_degree_nine_polynomials_on_bounded_lines():
    """Interior rows are exact for degree < 10 and the boundary neighbours enter with
    their own (ghost) values, so a polynomial filled into the ghosts is a fixed point."""
    n = 30
    g = Grid(1, (n,), [(cases.FIXED, cases.FIXED)])
    x = (np.arange(-5, n + 5) - 17.0) / 20.0
    Q = np.zeros((5, 1, 1, n + 10))
    Q[0] = 1.0 + 0.3 * x ** 9 - 0.2 * x ** 4 + x
    Q[4] = 2.0 - x ** 7
    out = IF.filter_state(Q, g, 0.49)
    assert np.max(np.abs(out - Q)) < 1e-13
    # degree 10 is changed: (1 - 2 alpha) 2^-10 10! / 17^10 = 3.5e-11 in the interior
    xi = np.arange(-5, n + 5) - 17.0
    Q[0] = 1.0 + (xi / 17.0) ** 10
    out = IF.filter_state(Q, g, 0.49)
    assert np.max(np.abs(out[0] - Q[0])) > 1e-11


def test_filter_bounded_matches_dense_solve():
    n = 12
    rng = np.random.default_rng(3)
    col = rng.normal(size=(n + 10, 2))
    coef = IF.gv_coefficients(0.45)
    A = np.eye(n)
    b = np.zeros((n, 2))
    for i in range(n):
        p = 5 + i
        b[i] = coef[0] * col[p] + sum(0.5 * coef[k] * (col[p + k] + col[p - k]) for k in range(1, 6))
        if i > 0:
            A[i, i - 1] = 0.45
        else:
            b[i] -= 0.45 * col[4]
        if i < n - 1:
            A[i, i + 1] = 0.45
        else:
            b[i] -= 0.45 * col[5 + n]
    ref = np.linalg.solve(A, b)
    got = IF.filter_lines(col, 5, n, False, 0.45, coef)
    assert np.max(np.abs(got - ref)) < 1e-14


def test_filter_state_conserves_periodic_totals_and_uniform_states():
    c = cases.random_smooth_state(cases.periodic_case(2, (24, 24)), seed=4)
    g = Grid(2, c.n, c.bc, h=c.h)
    fill_ghosts_conserved(c.Q, g)
    out = IF.filter_state(c.Q, g, 0.49)
    inner = (slice(None),) + g.interior()
    # sum of a periodic filtered line = T(0) times the sum (T(0) = 1)
    assert np.allclose(out[inner].sum(axis=(1, 2, 3)), c.Q[inner].sum(axis=(1, 2, 3)), rtol=1e-14)
    u = cases.uniform_state(cases.periodic_case(2, (24, 24))).Q
    assert np.max(np.abs(IF.filter_state(u, g, 0.49)[inner] - u[inner])) < 1e-14


# ----------------------------------------------------------------- LAD-C6 RHS
def test_lad_c6_rhs_uniform_flow_is_steady_on_cartesian_grids():
    c = cases.uniform_state(cases.periodic_case(2, (20, 20)))
    Q = c.Q
    g = Grid(2, c.n, c.bc, h=c.h)
    L = R.rhs(Q, g, R.Gas(), R.Opts(lad='C6'), 'lad')
    assert np.max(np.abs(L)) < 1e-12


def test_lad_c6_rhs_observed_order_on_an_entropy_wave():
    """Smooth inviscid advection: the artificial coefficients vanish to round-off, so the
    RHS error of LAD-C6 falls at sixth order (LAD-E4: fourth)."""
    errs = {'E4': [], 'C6': []}
    for n in (16, 32):
        c = cases.entropy_wave(n)
        g = Grid(1, c.n, c.bc, h=c.h)
        x = (np.arange(-5, n + 5) + 0.5) / n
        for sch in errs:
            L = R.rhs(c.Q, g, R.Gas(), R.Opts(lad=sch, C_beta=0.0, C_kappa=0.0), 'lad')
            rho_x = 2 * np.pi * 0.2 * np.cos(2 * np.pi * x)   # d rho / dx of the wave
            ref = -rho_x[5:5 + n]                               # u = 1, p const
            errs[sch].append(np.max(np.abs(L[0, 0, 0, 5:5 + n] - ref)))
    for sch, order in (('E4', 4), ('C6', 6)):
        o = np.log2(errs[sch][0] / errs[sch][1])
        assert abs(o - order) < 0.35, (sch, o)


def test_lad_c6_bounded_rhs_conserves_up_to_boundary_fluxes():
    """Sum over the interior of dQ/dt / J = -(F_{n-1/2} - F_{-1/2}) with the I4 faces."""
    c = cases.sod(40)
    g = Grid(1, c.n, c.bc, h=c.h)
    L = R.rhs(c.Q, g, R.Gas(), R.Opts(lad='C6'), 'lad')
    tot = L[:, 0, 0, 5:45].sum(axis=-1) * c.h[0]
    # far-field states are uniform and at rest except the pressure jump: net flux of
    # momentum p_L - p_R through the ends, none of mass or energy
    assert np.allclose(tot, [0.0, 1.0 - 0.1, 0.0, 0.0, 0.0], atol=1e-12)


def test_lad_c6_step_applies_the_filter_once_after_the_last_stage():
    c = cases.random_smooth_state(cases.periodic_case(1, (32,)), seed=9)
    g = Grid(1, c.n, c.bc, h=c.h)
    gas = R.Gas()
    o = R.Opts(lad='C6')
    Qf, t, dt, bad = R.rk3_step(c.Q.copy(), 0.0, 1.0, g, gas, o, 'lad')
    o_nf = R.Opts(lad='C6', filter_alpha=0.5)
    Qn, t2, dt2, _ = R.rk3_step(c.Q.copy(), 0.0, 1.0, g, gas, o_nf, 'lad')
    assert dt == dt2 and bad == 0
    inner = (slice(None),) + g.interior()
    ref = IF.filter_state(Qn, g, 0.49)
    assert np.max(np.abs(Qf[inner] - ref[inner])) < 1e-15
    assert np.max(np.abs(Qf[inner] - Qn[inner])) > 0.0


def test_filter_leaves_fixed_ghosts_to_the_caller():
    """FIXED ghost values are never rewritten (R13): a pass along x does not touch the
    FIXED ghost rows of y, whose values enter the y pass as given."""
    T, NS, FX = cases.TRANSMISSIVE, cases.NOSLIP, cases.FIXED
    c = cases.random_rough_state(cases.Case(2, (6, 40, 1), [(T, T), (NS, FX)], h=(0.05 / 6, 1 / 40, 1)), seed=24)
    g = Grid(2, c.n, c.bc, h=c.h)
    out = IF.filter_state(c.Q, g, 0.49)
    assert np.array_equal(out[:, :, 45:, 5:11], c.Q[:, :, 45:, 5:11])
    # and the y pass sees them: changing a FIXED ghost changes the filtered interior next to it
    Q2 = c.Q.copy()
    Q2[0, 0, 45, 5:11] += 0.1
    out2 = IF.filter_state(Q2, g, 0.49)
    assert np.max(np.abs(out2[0, 0, 44, 5:11] - out[0, 0, 44, 5:11])) > 1e-3
