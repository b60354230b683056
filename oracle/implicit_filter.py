"""Low-pass implicit (Pade-type) filter of the LAD-C6 scheme (oracle; test infrastructure only).

Paper: Sec. 2.1 (the in-house solver damps the dispersion errors of its central
schemes with the low-pass implicit filter of Gaitonde & Visbal) and Alg. 1
(FILTER_CALLS: after the solution update of the last Runge-Kutta stage, the filter is
applied along i, j and k; C-GBR runs use no filter).

The filter of one line is the tridiagonal system

    alpha_f phi^_{i-1} + phi^_i + alpha_f phi^_{i+1} = sum_{k=0}^{K} (a_k / 2) (phi_{i+k} + phi_{i-k})

with transfer function T(w) = sum_k a_k cos(k w) / (1 + 2 alpha_f cos w).  The K + 1
coefficients of the order-2K member are fixed by T(pi) = 0 (the odd-even mode is
removed) and 1 - T(w) = O(w^{2K}) (the filter leaves polynomials of degree < 2K
unchanged); they are obtained here by solving those K + 1 moment conditions in exact
rational arithmetic.

Readings used here:
  R29  tenth order (K = 5, eleven points, which the five ghost layers hold) and
       alpha_f = 0.49 (the paper gives neither); the conserved state Q is filtered,
       once per time step, after the third stage of SSP-RK3, along xi, eta, zeta in
       turn.  Before each direction the ghost layers are refilled with the boundary
       images of the current field; the filtered lines are those through interior
       nodes, and the unknowns of a bounded line are its interior nodes, whose
       neighbours across the boundary enter unfiltered (ghost values, never written:
       FIXED ghosts stay the caller's); a periodic line is cyclic over its interior
       nodes.  Alternative placement (option): after every stage.
"""
from fractions import Fraction

import numpy as np
import scipy.linalg

from . import grid as gr

FILTER_ORDER = 10
FILTER_ALPHA = 0.49


def gv_coefficients(alpha, order=FILTER_ORDER):
    """(a_0, .., a_K) of the order-``order`` filter for alpha_f = ``alpha`` (exact rationals
    of the binary value of alpha, returned as floats)."""
    K = order // 2
    al = Fraction(alpha)
    # unknowns a_0..a_K; rows: T(pi) = 0, then the w^{2m} Taylor terms, m = 0..K-1, of
    # sum_k a_k cos(k w) - (1 + 2 alpha cos w)
    A = [[Fraction((-1) ** k) for k in range(K + 1)]]
    b = [Fraction(0)]
    for m in range(K):
        A.append([Fraction(k ** (2 * m)) if (k or m == 0) else Fraction(0) for k in range(K + 1)])
        b.append((1 + 2 * al) if m == 0 else 2 * al)
    # Gauss-Jordan elimination over the rationals
    n = K + 1
    M = [row[:] + [rhs] for row, rhs in zip(A, b)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [vr - f * vc for vr, vc in zip(M[r], M[c])]
    return tuple(float(M[k][n]) for k in range(n))


def transfer(w, alpha, coef):
    """T(w) of the filter with coefficients ``coef``."""
    num = sum(a * np.cos(k * w) for k, a in enumerate(coef))
    return num / (1.0 + 2.0 * alpha * np.cos(w))


def _rhs(cols, lo, hi, coef):
    """sum_k a_k / 2 (phi_{i+k} + phi_{i-k}) for rows lo..hi-1 of cols (N, m)."""
    out = coef[0] * cols[lo:hi]
    for k in range(1, len(coef)):
        out = out + 0.5 * coef[k] * (cols[lo + k:hi + k] + cols[lo - k:hi - k])
    return out


def filter_lines(cols, g, n, periodic, alpha, coef):
    """Filtered interior of each column of cols (N, m) (lines along axis 0, ghosts filled)."""
    if periodic:
        inner = cols[g:g + n]
        rhs = coef[0] * inner
        for k in range(1, len(coef)):
            rhs = rhs + 0.5 * coef[k] * (np.roll(inner, -k, axis=0) + np.roll(inner, k, axis=0))
        c = np.zeros(n)
        c[0] = 1.0
        c[1] = alpha
        c[n - 1] += alpha
        return np.real(scipy.linalg.solve_circulant(c, rhs, singular='raise'))
    rhs = _rhs(cols, g, g + n, coef)
    rhs[0] = rhs[0] - alpha * cols[g - 1]
    rhs[n - 1] = rhs[n - 1] - alpha * cols[g + n]
    ab = np.zeros((3, n))
    ab[1, :] = 1.0
    ab[0, 1:] = alpha
    ab[2, :n - 1] = alpha
    return scipy.linalg.solve_banded((1, 1), ab, rhs, check_finite=False)


def filter_direction(Q, d, grid, alpha, coef):
    """One pass along d of the filter over the lines of Q (5, Nz, Ny, Nx) through interior
    nodes: their interior nodes are replaced; ghost values, the caller's FIXED ghosts
    included (R13), are read and never written."""
    ax = gr.axis_of(Q, d)
    g, n = grid.g[d], grid.n[d]
    inner = np.zeros(grid.shape, bool)
    inner[grid.interior()] = True
    lines = np.moveaxis(np.broadcast_to(inner, Q.shape), ax, 0)[g].reshape(-1)
    Qm = np.moveaxis(Q, ax, 0)
    N = Qm.shape[0]
    cols = Qm.reshape(N, -1)
    out = cols.copy()
    out[g:g + n, lines] = filter_lines(cols[:, lines], g, n, grid.periodic(d), alpha, coef)
    return np.moveaxis(out.reshape(Qm.shape), 0, ax)


def filter_state(Q, grid, alpha=FILTER_ALPHA, order=FILTER_ORDER, gas=None, keep=None):
    """FILTER_CALLS of Alg. 1 on the conserved state (R29); returns the filtered copy with
    its ghost layers refilled (isothermal walls need the gas model).

    keep (bool, field shape, optional): nodes that keep their value through every pass
    (the C-GBR nodes of a per-cell hybrid stage, R35); the lines are still solved whole,
    and the other nodes take their filtered values."""
    coef = gv_coefficients(alpha, order)
    Q = Q.copy()
    for d in range(grid.ndim):
        gr.fill_ghosts_conserved(Q, grid, gas)
        out = filter_direction(Q, d, grid, alpha, coef)
        Q = out if keep is None else np.where(keep[None], Q, out)
    gr.fill_ghosts_conserved(Q, grid, gas)
    return Q
