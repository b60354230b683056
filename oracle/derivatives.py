"""First derivatives along one computational direction (oracle; test infrastructure only).

Paper: Sec. 2.3 (MEG6 uses explicit sixth-order gradients, MIG4 implicit fourth-order
gradients, one tridiagonal solve per line and primitive, Sec. 4.2) and the
LAD-E4 variant of Sec. 4.2 / Sec. 5 (explicit fourth-order central differences).
Unit computational spacing (Delta xi = 1, Sec. 2.2).

  E6: f'_i = [45 (f_{i+1} - f_{i-1}) - 9 (f_{i+2} - f_{i-2}) + (f_{i+3} - f_{i-3})] / 60
  E4: f'_i = [ 8 (f_{i+1} - f_{i-1}) -   (f_{i+2} - f_{i-2})] / 12
  C4: (1/4) f'_{i-1} + f'_i + (1/4) f'_{i+1} = (3/4) (f_{i+1} - f_{i-1})
  C6: (1/3) f'_{i-1} + f'_i + (1/3) f'_{i+1} = (7/9) (f_{i+1} - f_{i-1}) + (1/36) (f_{i+2} - f_{i-2})
      (the sixth-order tridiagonal member of the compact central family; LAD-C6, Sec. 3)

C4 closure (reading R10): a non-periodic line is solved over all its nodes
including ghosts, with second-order one-sided end rows
f'_0 = (-3 f_0 + 4 f_1 - f_2)/2 and f'_{N-1} = (3 f_{N-1} - 4 f_{N-2} + f_{N-3})/2;
a periodic line is solved cyclically over the interior nodes and its ghost
derivatives are the periodic images.  C6 closure (reading R27): the same end rows,
and the C4 row at the second and second-to-last nodes, where the C6 stencil does not
fit.  The banded and circulant solves are the library routines
scipy.linalg.solve_banded / solve_circulant.

Explicit results are NaN where the stencil leaves the array.
"""
import numpy as np
import scipy.linalg

from .grid import shift, axis_of


def e6(f, d):
    return (45.0 * (shift(f, 1, d) - shift(f, -1, d))
            - 9.0 * (shift(f, 2, d) - shift(f, -2, d))
            + (shift(f, 3, d) - shift(f, -3, d))) / 60.0


def e4(f, d):
    return (8.0 * (shift(f, 1, d) - shift(f, -1, d)) - (shift(f, 2, d) - shift(f, -2, d))) / 12.0


def c4_line_matrix_banded(N):
    """Banded storage (3, N) of the bounded C4 system with one-sided end rows."""
    ab = np.zeros((3, N))
    ab[1, :] = 1.0
    ab[0, 2:] = 0.25          # super-diagonal a[i, i+1] for rows 1..N-2
    ab[2, :N - 2] = 0.25      # sub-diagonal a[i, i-1] for rows 1..N-2
    return ab


def c4_bounded_lines(F):
    """C4 derivative of each column of F (N, m) (lines along axis 0), bounded closure."""
    N = F.shape[0]
    rhs = np.empty_like(F)
    rhs[1:N - 1] = 0.75 * (F[2:] - F[:N - 2])
    rhs[0] = (-3.0 * F[0] + 4.0 * F[1] - F[2]) / 2.0
    rhs[N - 1] = (3.0 * F[N - 1] - 4.0 * F[N - 2] + F[N - 3]) / 2.0
    return scipy.linalg.solve_banded((1, 1), c4_line_matrix_banded(N), rhs)


def c4_cyclic_lines(F):
    """C4 derivative of each column of F (n, m), periodic lines of n nodes."""
    n = F.shape[0]
    rhs = 0.75 * (np.roll(F, -1, axis=0) - np.roll(F, 1, axis=0))
    c = np.zeros(n)
    c[0] = 1.0
    c[1] = 0.25
    c[n - 1] += 0.25
    return np.real(scipy.linalg.solve_circulant(c, rhs, singular='raise'))


def c4(f, d, grid):
    """Compact fourth-order derivative of a scalar field along direction d (R10)."""
    ax = axis_of(f, d)
    fm = np.moveaxis(f, ax, 0)
    N = fm.shape[0]
    cols = fm.reshape(N, -1)
    if grid.periodic(d):
        g, n = grid.g[d], grid.n[d]
        inner = c4_cyclic_lines(cols[g:g + n])
        out = np.empty_like(cols)
        out[g:g + n] = inner
        for e in range(0, g):
            out[e] = inner[(e - g) % n]
        for e in range(g + n, N):
            out[e] = inner[(e - g) % n]
    else:
        out = c4_bounded_lines(cols)
    return np.moveaxis(out.reshape(fm.shape), 0, ax)


C6_ALPHA = 1.0 / 3.0
C6_A = 7.0 / 9.0      # weight of (f_{i+1} - f_{i-1})
C6_B = 1.0 / 36.0     # weight of (f_{i+2} - f_{i-2})


def c6_bounded_lines(F):
    """C6 derivative of each column of F (N, m) (lines along axis 0), bounded closure (R27)."""
    N = F.shape[0]
    rhs = np.empty_like(F)
    rhs[2:N - 2] = C6_A * (F[3:N - 1] - F[1:N - 3]) + C6_B * (F[4:] - F[:N - 4])
    rhs[1] = 0.75 * (F[2] - F[0])
    rhs[N - 2] = 0.75 * (F[N - 1] - F[N - 3])
    rhs[0] = (-3.0 * F[0] + 4.0 * F[1] - F[2]) / 2.0
    rhs[N - 1] = (3.0 * F[N - 1] - 4.0 * F[N - 2] + F[N - 3]) / 2.0
    ab = np.zeros((3, N))
    ab[1, :] = 1.0
    ab[0, 3:N - 1] = C6_ALPHA     # a[i, i+1] for rows 2..N-3
    ab[2, 1:N - 3] = C6_ALPHA     # a[i, i-1] for rows 2..N-3
    ab[0, 2] = 0.25               # row 1 (C4)
    ab[2, 0] = 0.25
    ab[0, N - 1] = 0.25           # row N-2 (C4)
    ab[2, N - 3] = 0.25
    return scipy.linalg.solve_banded((1, 1), ab, rhs)


def c6_cyclic_lines(F):
    """C6 derivative of each column of F (n, m), periodic lines of n nodes."""
    n = F.shape[0]
    rhs = C6_A * (np.roll(F, -1, axis=0) - np.roll(F, 1, axis=0)) \
        + C6_B * (np.roll(F, -2, axis=0) - np.roll(F, 2, axis=0))
    c = np.zeros(n)
    c[0] = 1.0
    c[1] = C6_ALPHA
    c[n - 1] += C6_ALPHA
    return np.real(scipy.linalg.solve_circulant(c, rhs, singular='raise'))


def _compact(f, d, grid, bounded, cyclic):
    ax = axis_of(f, d)
    fm = np.moveaxis(f, ax, 0)
    N = fm.shape[0]
    cols = fm.reshape(N, -1)
    if grid.periodic(d):
        g, n = grid.g[d], grid.n[d]
        inner = cyclic(cols[g:g + n])
        out = np.empty_like(cols)
        out[g:g + n] = inner
        for e in range(0, g):
            out[e] = inner[(e - g) % n]
        for e in range(g + n, N):
            out[e] = inner[(e - g) % n]
    else:
        out = bounded(cols)
    return np.moveaxis(out.reshape(fm.shape), 0, ax)


def c6(f, d, grid):
    """Compact sixth-order derivative of a scalar field along direction d (R27)."""
    return _compact(f, d, grid, c6_bounded_lines, c6_cyclic_lines)


def gradient(f, d, kind, grid):
    """Derivative of f along d with scheme ``kind`` in {'E6', 'E4', 'C4', 'C6'}."""
    if kind == 'E6':
        return e6(f, d)
    if kind == 'E4':
        return e4(f, d)
    if kind == 'C4':
        return c4(f, d, grid)
    if kind == 'C6':
        return c6(f, d, grid)
    raise ValueError(kind)
