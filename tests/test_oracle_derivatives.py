"""Pins of the oracle's E6 / E4 / C4 first derivatives (MEG6 / MIG4 gradients, LAD-E4)."""
import numpy as np
import pytest

from oracle import derivatives as D
from oracle.grid import Grid, BC_PERIODIC, BC_TRANSMISSIVE


def _line(N):
    return np.arange(N, dtype=float)[None, None, :]


@pytest.mark.parametrize('kind,deg', [('E6', 6), ('E4', 4)])
def test_explicit_exact_on_polynomials(kind, deg):
    x = _line(30) * 0.37 - 3.0
    f = D.e6 if kind == 'E6' else D.e4
    for k in range(deg + 1):
        got = f(x ** k, 0)[0, 0, 4:-4] / 0.37
        ref = k * x[0, 0, 4:-4] ** (k - 1) if k else 0 * x[0, 0, 4:-4]
        assert np.allclose(got, ref, rtol=1e-11, atol=1e-9)
    got = f(x ** (deg + 1), 0)[0, 0, 4:-4] / 0.37
    assert not np.allclose(got, (deg + 1) * x[0, 0, 4:-4] ** deg, rtol=1e-9, atol=1e-7)


def _dense_c4(N, cyclic):
    A = np.eye(N)
    for i in range(N):
        if cyclic or 0 < i < N - 1:
            A[i, (i - 1) % N] += 0.25
            A[i, (i + 1) % N] += 0.25
    return A


@pytest.mark.parametrize('N', list(range(5, 17)))
def test_c4_bounded_matches_dense_solve(N):
    rng = np.random.default_rng(N)
    f = rng.normal(size=(N, 3))
    rhs = np.empty_like(f)
    rhs[1:-1] = 0.75 * (f[2:] - f[:-2])
    rhs[0] = (-3 * f[0] + 4 * f[1] - f[2]) / 2
    rhs[-1] = (3 * f[-1] - 4 * f[-2] + f[-3]) / 2
    ref = np.linalg.solve(_dense_c4(N, False), rhs)
    got = D.c4_bounded_lines(f)
    assert np.max(np.abs(got - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize('N', list(range(5, 17)))
def test_c4_cyclic_matches_dense_solve(N):
    rng = np.random.default_rng(100 + N)
    f = rng.normal(size=(N, 2))
    rhs = 0.75 * (np.roll(f, -1, 0) - np.roll(f, 1, 0))
    ref = np.linalg.solve(_dense_c4(N, True), rhs)
    got = D.c4_cyclic_lines(f)
    assert np.max(np.abs(got - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref)))


def test_c4_inverse_decay_factor():
    """The interior influence of a unit impulse decays by 2 - sqrt(3) = 0.26795 per node."""
    N = 41
    A = _dense_c4(N, True)
    col = np.linalg.inv(A)[:, 0]
    ratios = -col[1:6] / col[0:5]
    assert np.allclose(ratios, 2 - np.sqrt(3), rtol=1e-6)


@pytest.mark.parametrize('kind,order', [('E6', 6), ('E4', 4), ('C4', 4)])
def test_observed_order_on_periodic_sines(kind, order):
    errs = []
    for n in (16, 32, 64):
        g = Grid(1, (n,), [(BC_PERIODIC, BC_PERIODIC)], h=(1.0 / n,))
        x = (np.arange(-5, n + 5) + 0.5) / n
        f = np.sin(2 * np.pi * x)[None, None, :]
        got = D.gradient(f, 0, kind, g)[0, 0, 5:5 + n] * n
        errs.append(np.max(np.abs(got - 2 * np.pi * np.cos(2 * np.pi * x[5:5 + n]))))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - order) < 0.2), orders


def test_c4_bounded_line_exact_on_quadratics():
    """With one-sided second-order end rows, the bounded C4 line is exact for degree <= 2."""
    g = Grid(1, (20,), [(BC_TRANSMISSIVE, BC_TRANSMISSIVE)])
    x = np.arange(30, dtype=float)[None, None, :]
    f = 0.3 * x ** 2 - 2 * x + 1
    got = D.c4(f, 0, g)
    assert np.allclose(got, 0.6 * x - 2, rtol=1e-12, atol=1e-12)


def test_modified_wavenumbers():
    """Fourier symbols k* h of the three operators (the truncation-error pins of the
    gradient orders): E6, E4 and C4 against their stencils applied to exp(i k x)."""
    n = 64
    g = Grid(1, (n,), [(BC_PERIODIC, BC_PERIODIC)])
    x = np.arange(-5, n + 5, dtype=float)
    for m in (1, 3, 7, 13):
        k = 2 * np.pi * m / n
        sym = {'E6': (45 * np.sin(k) - 9 * np.sin(2 * k) + np.sin(3 * k)) / 30,
               'E4': (8 * np.sin(k) - np.sin(2 * k)) / 6,
               'C4': 1.5 * np.sin(k) / (1 + 0.5 * np.cos(k))}
        for kind in ('E6', 'E4', 'C4'):
            re = D.gradient(np.cos(k * x)[None, None, :], 0, kind, g)[0, 0, 5:5 + n]
            assert np.allclose(re, -sym[kind] * np.sin(k * x[5:5 + n]), atol=1e-12)
        if m > 3:
            continue
        # leading errors at small k h: E6 ~ k^7/140, E4 ~ k^5/30, C4 ~ k^5/180
        assert abs(sym['E6'] - k) < 1.05 * k ** 7 / 140
        assert abs(sym['E4'] - k) < 1.05 * k ** 5 / 30
        assert abs(sym['C4'] - k) < 1.05 * k ** 5 / 180
