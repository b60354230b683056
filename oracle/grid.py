"""Grid layout, ghost layers, boundary images and metrics (oracle; test infrastructure only).

Paper: Sec. 2.1 (governing equations in generalised curvilinear coordinates,
Eq. eq:3.1.1; metrics normalised by the Jacobian, xi_hat = xi_x / J) and the
boundary conditions listed with each test case of Sec. 3.

Readings used here (see the design notes for the full list):
  R13  five ghost layers per active direction; transmissive = zeroth-order
       copy; reflective = mirror with the normal momentum negated; no-slip
       adiabatic = mirror with all momentum negated; fixed (Dirichlet inflow) =
       ghost values owned by the caller and never rewritten.  Directions are
       filled in the order x, y, z over the full extended extent, so corner
       ghosts are defined.  Scalar intermediate fields are filled with the
       same images and even parity.
  R14  nodes are cell centres.
  R6   node metrics in conservative form with the fourth-order explicit
       difference D4 as the outer operator; interface metrics by fourth-order
       interpolation I4 of the node metrics.

Array layout: a scalar field is ``(Nz, Ny, Nx)``; a stack of fields is
``(nvar, Nz, Ny, Nx)``.  Direction d (0 = xi/x, 1 = eta/y, 2 = zeta/z) is numpy
axis ``ndim_of_array - 1 - d``.  Inactive directions have one node and no ghosts.
"""
import numpy as np

NG = 5
BC_PERIODIC, BC_TRANSMISSIVE, BC_REFLECTIVE, BC_NOSLIP, BC_FIXED, BC_NOSLIP_T = 0, 1, 2, 3, 4, 5


class Grid:
    """Structured grid with ``ndim`` active directions.

    n      : interior node counts (nx, ny, nz); inactive directions must be 1.
    bc     : bc[d] = (lo, hi) boundary codes for each active direction d.
    h      : Cartesian spacings (hx, hy, hz) when ``coords`` is None.
    coords : (3, Nz, Ny, Nx) node coordinates including ghost nodes, for a
             curvilinear grid (None for Cartesian).
    wall_T : wall_T[d][side], the wall temperature (T_ref = 1) of a no-slip isothermal
             face (BC_NOSLIP_T); unused elsewhere.
    """

    def __init__(self, ndim, n, bc, h=(1.0, 1.0, 1.0), coords=None, wall_T=None):
        n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
        assert 1 <= ndim <= 3
        for d in range(ndim, 3):
            assert n[d] == 1, "inactive directions must have one node"
        self.ndim = ndim
        self.n = n
        self.g = tuple(NG if d < ndim else 0 for d in range(3))
        self.N = tuple(n[d] + 2 * self.g[d] for d in range(3))
        bc = [tuple(b) for b in bc] + [(BC_TRANSMISSIVE, BC_TRANSMISSIVE)] * (3 - len(bc))
        self.bc = bc[:3]
        self.h = tuple(float(v) for v in h) + (1.0,) * (3 - len(h))
        self.coords = coords
        wt = [tuple(float(v) for v in w) for w in (wall_T or [])]
        self.wall_T = (wt + [(0.0, 0.0)] * 3)[:3]

    @property
    def shape(self):
        return (self.N[2], self.N[1], self.N[0])

    def interior(self):
        """Slices (k, j, i) of the interior nodes of a scalar field."""
        return tuple(slice(self.g[d], self.g[d] + self.n[d]) for d in (2, 1, 0))

    def band(self, lo, hi):
        """Slices of the nodes whose position lies in [lo, n + hi) in every active direction
        (position 0 is the first interior node)."""
        out = []
        for d in (2, 1, 0):
            if d < self.ndim:
                out.append(slice(self.g[d] + lo, self.g[d] + self.n[d] + hi))
            else:
                out.append(slice(0, 1))
        return tuple(out)

    def periodic(self, d):
        return self.bc[d][0] == BC_PERIODIC


def axis_of(f, d):
    return f.ndim - 1 - d


def shift(f, s, d, fill=np.nan):
    """g[..., i, ...] = f[..., i + s, ...] along direction d; ``fill`` outside the array."""
    ax = axis_of(f, d)
    g = np.full_like(f, fill)
    n = f.shape[ax]
    if abs(s) >= n:
        return g
    src = [slice(None)] * f.ndim
    dst = [slice(None)] * f.ndim
    if s >= 0:
        src[ax] = slice(s, n)
        dst[ax] = slice(0, n - s)
    else:
        src[ax] = slice(0, n + s)
        dst[ax] = slice(-s, n)
    g[tuple(dst)] = f[tuple(src)]
    return g


def _take(f, ax, idx):
    sl = [slice(None)] * f.ndim
    sl[ax] = slice(idx, idx + 1)
    return tuple(sl)


def _ghost_pairs(grid, d, side):
    """(destination index, source index, mirrored?) for each ghost layer on one side (R13)."""
    g, n = grid.g[d], grid.n[d]
    t = grid.bc[d][side]
    pairs = []
    for m in range(g):
        dst = g - 1 - m if side == 0 else g + n + m
        if t == BC_PERIODIC:
            src = dst + n if side == 0 else dst - n
            pairs.append((dst, src, False))
        elif t == BC_TRANSMISSIVE:
            pairs.append((dst, g if side == 0 else g + n - 1, False))
        elif t in (BC_REFLECTIVE, BC_NOSLIP, BC_NOSLIP_T):
            pairs.append((dst, g + m if side == 0 else g + n - 1 - m, True))
        elif t == BC_FIXED:
            pass
        else:
            raise ValueError("unknown boundary code %r" % t)
    return pairs


def _isothermal_image(Qs, T_w, gas):
    """Ghost state mirroring the conserved state Qs across a no-slip wall held at T_w
    (R32): velocity odd (zero at the wall), pressure even (no normal gradient),
    temperature odd about T_w (the pair's mean is T_w), density from p = rho T /
    (gamma Mref^2)."""
    gamma = gas.gamma
    gM2 = gamma * gas.Mref ** 2
    rho = Qs[0]
    u = Qs[1:4] / rho
    ke = 0.5 * rho * (u ** 2).sum(axis=0)
    p = (gamma - 1.0) * (Qs[4] - ke)
    T_g = 2.0 * T_w - gM2 * p / rho
    rho_g = gM2 * p / T_g
    out = np.empty_like(Qs)
    out[0] = rho_g
    out[1:4] = -rho_g * u
    out[4] = p / (gamma - 1.0) + 0.5 * rho_g * (u ** 2).sum(axis=0)
    return out


def fill_ghosts_conserved(Q, grid, gas=None):
    """Fill the ghost layers of the conserved state Q (5, Nz, Ny, Nx) in place (R13).

    Reflective walls negate the momentum component normal to the wall (the
    Cartesian component of the sweep direction; walls are grid lines aligned
    with that axis).  No-slip adiabatic walls negate all momentum, so the wall
    velocity is zero while density and energy (hence temperature) are even.
    No-slip isothermal walls (R32) need the gas (gamma, Mref) for the equation of
    state.
    """
    for d in range(grid.ndim):
        ax = axis_of(Q, d)
        for side in (0, 1):
            t = grid.bc[d][side]
            if t == BC_NOSLIP_T and gas is None:
                raise ValueError('an isothermal wall needs the gas model')
            for dst, src, mirrored in _ghost_pairs(grid, d, side):
                if t == BC_NOSLIP_T:
                    Q[_take(Q, ax, dst)] = _isothermal_image(Q[_take(Q, ax, src)], grid.wall_T[d][side], gas)
                    continue
                Q[_take(Q, ax, dst)] = Q[_take(Q, ax, src)]
                if mirrored:
                    comps = [1 + d] if t == BC_REFLECTIVE else [1, 2, 3]
                    for c in comps:
                        sl = list(_take(Q, ax, dst))
                        sl[0] = slice(c, c + 1)
                        Q[tuple(sl)] *= -1.0
    return Q


def fill_ghosts_scalar(f, grid):
    """Fill the ghost layers of a scalar intermediate field (Nz, Ny, Nx) in place with the
    boundary images and even parity (R13); fixed boundaries use the zeroth-order copy."""
    for d in range(grid.ndim):
        ax = axis_of(f, d)
        g, n = grid.g[d], grid.n[d]
        for side in (0, 1):
            t = grid.bc[d][side]
            for m in range(g):
                dst = g - 1 - m if side == 0 else g + n + m
                if t == BC_PERIODIC:
                    src = dst + n if side == 0 else dst - n
                elif t in (BC_TRANSMISSIVE, BC_FIXED):
                    src = g if side == 0 else g + n - 1
                else:
                    src = g + m if side == 0 else g + n - 1 - m
                f[_take(f, ax, dst)] = f[_take(f, ax, src)]
    return f


def d4(f, d):
    """Fourth-order explicit central difference along d (unit computational spacing)."""
    return (8.0 * (shift(f, 1, d) - shift(f, -1, d)) - (shift(f, 2, d) - shift(f, -2, d))) / 12.0


def node_metrics(grid):
    """Node metrics (10, Nz, Ny, Nx) = (xi_x, xi_y, xi_z, eta_x, eta_y, eta_z, zeta_x, zeta_y, zeta_z)/J
    and J, i.e. the normalised metric terms of Sec. 2.1 (xi_hat = xi_x / J).

    Cartesian grids: xi_hat = (hy hz, 0, 0), eta_hat = (0, hx hz, 0),
    zeta_hat = (0, 0, hx hy), J = 1 / (hx hy hz) (unit computational spacing).

    Curvilinear grids (R6): conservative form with D4 as the outer operator,
      2D: xi_hat = ( y_eta, -x_eta), eta_hat = (-y_xi, x_xi), zeta_hat_z = x_xi y_eta - x_eta y_xi
      3D: xi_hat_x = (y_eta z)_zeta - (y_zeta z)_eta and cyclic permutations,
    so that sum_l D4_l(l_hat) = 0 to round-off (discrete geometric conservation).
    1/J is the determinant of the D4 coordinate Jacobian.
    Values are defined where the stencils fit (positions -3 .. n+2); NaN elsewhere.
    """
    shape = grid.shape
    M = np.zeros((10,) + shape)
    if grid.coords is None:
        hx, hy, hz = grid.h
        M[0] = hy * hz
        M[4] = hx * hz
        M[8] = hx * hy
        M[9] = 1.0 / (hx * hy * hz)
        return M
    x, y, z = grid.coords
    nd = grid.ndim
    if nd == 1:
        xx = d4(x, 0)
        M[0] = 1.0
        M[4] = xx
        M[8] = xx
        M[9] = 1.0 / xx
        return M
    if nd == 2:
        x_xi, x_eta = d4(x, 0), d4(x, 1)
        y_xi, y_eta = d4(y, 0), d4(y, 1)
        M[0] = y_eta
        M[1] = -x_eta
        M[3] = -y_xi
        M[4] = x_xi
        det = x_xi * y_eta - x_eta * y_xi
        M[8] = det
        M[9] = 1.0 / det
        return M
    D = lambda f, d: d4(f, d)  # noqa: E731
    # inner derivatives
    xe, xz, xx_ = D(x, 1), D(x, 2), D(x, 0)
    ye, yz, yx = D(y, 1), D(y, 2), D(y, 0)
    ze, zz, zx = D(z, 1), D(z, 2), D(z, 0)
    M[0] = D(ye * z, 2) - D(yz * z, 1)
    M[1] = D(ze * x, 2) - D(zz * x, 1)
    M[2] = D(xe * y, 2) - D(xz * y, 1)
    M[3] = D(yz * z, 0) - D(yx * z, 2)
    M[4] = D(zz * x, 0) - D(zx * x, 2)
    M[5] = D(xz * y, 0) - D(xx_ * y, 2)
    M[6] = D(yx * z, 1) - D(ye * z, 0)
    M[7] = D(zx * x, 1) - D(ze * x, 0)
    M[8] = D(xx_ * y, 1) - D(xe * y, 0)
    det = (xx_ * (ye * zz - yz * ze) - xe * (yx * zz - yz * zx) + xz * (yx * ze - ye * zx))
    M[9] = 1.0 / det
    return M


def interface_metrics(M, d):
    """xi_tilde at the interface i+1/2 along d, stored at node i (R6):
    I4(a) = [7 (a_i + a_{i+1}) - (a_{i-1} + a_{i+2})] / 12 applied to the three
    normalised metric components of direction d."""
    a = M[3 * d:3 * d + 3]
    return (7.0 * (a + shift(a, 1, d)) - (shift(a, -1, d) + shift(a, 2, d))) / 12.0


def i4(f, d):
    """Fourth-order mid-point interpolation to i+1/2 (stored at node i)."""
    return (7.0 * (f + shift(f, 1, d)) - (shift(f, -1, d) + shift(f, 2, d))) / 12.0


def delta_x(grid, d):
    """Local displacement vector along direction d at every node (Sec. 2.2):
    0.5 (x_{i+1} - x_{i-1}) componentwise; (h_d e_d) on a Cartesian grid."""
    out = np.zeros((3,) + grid.shape)
    if grid.coords is None:
        out[d] = grid.h[d]
        return out
    for c in range(3):
        out[c] = 0.5 * (shift(grid.coords[c], 1, d) - shift(grid.coords[c], -1, d))
    return out
