"""Localized artificial diffusivity and central fluxes (oracle; test infrastructure only).

Paper: Sec. 2.2 (artificial transport coefficients mu*, beta*, kappa* added to the
physical ones; switching function f_sw; truncated-Gaussian over-bar; length
scales Delta_{l,mu}, Delta_{l,beta}, Delta_{l,kappa} from the local displacement
vector Delta x_l), Eq. tauij (viscous stress and heat flux in curvilinear
coordinates) and Sec. 2.1 (viscous flux vectors, Sutherland law, Stokes
hypothesis, kappa_hat = mu_hat / ((gamma-1) Pr M^2), p = rho T / (gamma M^2)).
The LAD form of the hybrid uses explicit fourth-order central differences (E4,
Sec. 5); written in flux form, the E4 derivative of a node flux is the difference
of its fourth-order interface interpolation I4.  The paper's stand-alone LAD scheme
uses sixth-order compact central differences (LAD-C6, Sec. 3 and Alg. 1), whose flux
form is a tridiagonal system for the interface fluxes (R28).

Readings used here:
  R9   5-point fourth difference for d^4/dxi^4 Delta xi^4; |S| = sqrt(S_ij S_ij);
       unit vectors of grad(rho), grad(e) regularised with +1e-32; H(0) = 0;
       over-bar = Kawai & Lele's 9-point truncated Gaussian applied along
       xi, eta, zeta in turn, computed at interior nodes with ghost images
       refilled before every pass; starred coefficients add directly to the
       non-dimensional mu_hat, beta and kappa_hat.
  R11  viscous fluxes: node values of -xi_hat . [0, tau, phi] from the scheme's
       gradients, I4 to the interface, then differenced.
  R13  ghost images of intermediate scalar fields (even parity).
  R15  T = gamma M^2 p / rho with M = 1 for inviscid runs.
  R28  LAD-C6: the primitives' gradients are C6 (R27); the interface fluxes F_{i+1/2}
       of a line solve
         (1/3) F_{i-1/2} + F_{i+1/2} + (1/3) F_{i+3/2}
             = (29/36) (F_i + F_{i+1}) + (1/36) (F_{i-1} + F_{i+2}),
       whose differences satisfy the C6 relation for the node derivative exactly
       (subtract the rows of i+1/2 and i-1/2).  A bounded line takes the two
       boundary faces -1/2 and n-1/2 from I4 (known values of the system), so the
       scheme stays conservative; a periodic line is cyclic over its n faces.
"""
from fractions import Fraction

import numpy as np
import scipy.linalg

from .grid import shift, fill_ghosts_scalar, delta_x, i4, axis_of

# Truncated-Gaussian weights for offsets 0, +-1, ..., +-4 (Kawai & Lele 2008).
GAUSS_FRAC = (Fraction(3565, 10368), Fraction(3091, 12960), Fraction(1997, 25920),
              Fraction(149, 12960), Fraction(107, 103680))
GAUSS_W = tuple(float(w) for w in GAUSS_FRAC)


def physical_gradients(G, M, grid):
    """d q / d x_j = sum_l J l_hat_j d q / d xi_l (chain rule, Sec. 2.1).

    G : dict l -> (nq, ...) derivatives along xi_l for active l.
    Returns (nq, 3, ...)."""
    some = next(iter(G.values()))
    D = np.zeros((some.shape[0], 3) + some.shape[1:])
    for l, Gl in G.items():
        for j in range(3):
            D[:, j] += M[9] * M[3 * l + j] * Gl
    return D


def sutherland(T, S):
    """mu / mu_inf for non-dimensional T = T/T_inf and S = S_suth / T_inf."""
    return T ** 1.5 * (1.0 + S) / (T + S)


def temperature(W, gas):
    return gas.gamma * gas.Mref ** 2 * W[4] / W[0]


def physical_transport(W, gas):
    """(mu_hat, kappa_hat) of the fluid (zero for inviscid runs)."""
    if not gas.viscous:
        z = np.zeros_like(W[0])
        return z, z
    mu = sutherland(temperature(W, gas), gas.suth) / gas.Re
    kappa = mu / ((gas.gamma - 1.0) * gas.Pr * gas.Mref ** 2)
    return mu, kappa


def viscous_node_flux(W, D, M, d, gas, mu, beta, kappa):
    """-l_hat . [0, tau, phi] at every node for direction d (Eq. tauij).

    D = physical gradients (5, 3, ...) of (rho, u, v, w, p)."""
    rho, p = W[0], W[4]
    du = D[1:4]                                   # du[i][j] = d u_i / d x_j
    theta = du[0][0] + du[1][1] + du[2][2]
    g2 = gas.gamma * gas.Mref ** 2
    dT = [g2 * (D[4][j] / rho - p * D[0][j] / (rho * rho)) for j in range(3)]
    tau = [[mu * (du[i][j] + du[j][i]) + ((beta - (2.0 / 3.0) * mu) * theta if i == j else 0.0)
            for j in range(3)] for i in range(3)]
    vel = W[1:4]
    phi = [vel[0] * tau[i][0] + vel[1] * tau[i][1] + vel[2] * tau[i][2] + kappa * dT[i]
           for i in range(3)]
    m = M[3 * d:3 * d + 3]
    F = np.zeros_like(W)
    for i in range(3):
        F[1 + i] = -(m[0] * tau[i][0] + m[1] * tau[i][1] + m[2] * tau[i][2])
    F[4] = -(m[0] * phi[0] + m[1] * phi[1] + m[2] * phi[2])
    return F


def convective_node_flux(W, M, d, gamma):
    """F^c(W, l_hat) at every node for direction d (Eq. eq:3.1.1)."""
    rho, u, v, w, p = W
    m = M[3 * d:3 * d + 3]
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    U = m[0] * u + m[1] * v + m[2] * w
    return np.stack([rho * U, rho * u * U + m[0] * p, rho * v * U + m[1] * p,
                     rho * w * U + m[2] * p, (E + p) * U])


def delta4(f, d):
    return (shift(f, -2, d) - 4.0 * shift(f, -1, d) + 6.0 * f
            - 4.0 * shift(f, 1, d) + shift(f, 2, d))


def gaussian_pass(f, d, grid):
    """One truncated-Gaussian pass along d at interior nodes, then ghost images (R9)."""
    out = GAUSS_W[0] * f
    for s in range(1, 5):
        out = out + GAUSS_W[s] * (shift(f, s, d) + shift(f, -s, d))
    res = np.zeros_like(f)
    inner = grid.interior()
    res[inner] = out[inner]
    return fill_ghosts_scalar(res, grid)


def lad_coefficients(W, G4, M, grid, gas, opts, raw_only=False):
    """Artificial (mu*, beta*, kappa*) at every node (interior + ghost images) (Sec. 2.2).

    G4 : dict l -> E4 derivatives (5, ...) of the primitives along xi_l."""
    gamma = gas.gamma
    D = physical_gradients(G4, M, grid)
    rho, p = W[0], W[4]
    du = D[1:4]
    S2 = np.zeros_like(rho)
    for i in range(3):
        for j in range(3):
            sij = 0.5 * (du[i][j] + du[j][i])
            S2 = S2 + sij * sij
    Smag = np.sqrt(S2)
    theta = du[0][0] + du[1][1] + du[2][2]
    w1 = du[2][1] - du[1][2]
    w2 = du[0][2] - du[2][0]
    w3 = du[1][0] - du[0][1]
    om2 = w1 * w1 + w2 * w2 + w3 * w3
    e = p / ((gamma - 1.0) * rho)
    de = [(D[4][j] / rho - p * D[0][j] / (rho * rho)) / (gamma - 1.0) for j in range(3)]
    grho = [D[0][j] for j in range(3)]
    nr = np.sqrt(grho[0] ** 2 + grho[1] ** 2 + grho[2] ** 2) + 1e-32
    ne = np.sqrt(de[0] ** 2 + de[1] ** 2 + de[2] ** 2) + 1e-32
    T = temperature(W, gas)
    c = np.sqrt(gamma * p / rho)
    fsw = np.where(theta < 0.0, theta * theta / (theta * theta + om2 + 1e-32), 0.0)

    s_mu = np.zeros_like(rho)
    s_beta = np.zeros_like(rho)
    s_kap = np.zeros_like(rho)
    for l in range(grid.ndim):
        dx = delta_x(grid, l)
        dmu2 = dx[0] ** 2 + dx[1] ** 2 + dx[2] ** 2
        dbeta = (dx[0] * grho[0] + dx[1] * grho[1] + dx[2] * grho[2]) / nr
        dkap = np.abs(dx[0] * de[0] + dx[1] * de[1] + dx[2] * de[2]) / ne
        s_mu = s_mu + delta4(Smag, l) * dmu2
        s_beta = s_beta + delta4(theta, l) * dbeta * dbeta
        s_kap = s_kap + delta4(e, l) * dkap

    raws = [opts.C_mu * rho * np.abs(s_mu),
            opts.C_beta * rho * fsw * np.abs(s_beta),
            opts.C_kappa * rho * c / T * np.abs(s_kap)]
    inner = grid.interior()
    out = []
    for r in raws:
        f = np.zeros_like(rho)
        f[inner] = r[inner]
        fill_ghosts_scalar(f, grid)
        if not raw_only:
            for l in range(grid.ndim):
                f = gaussian_pass(f, l, grid)
        out.append(f)
    return out


C6F_ALPHA = 1.0 / 3.0
C6F_A = 29.0 / 36.0   # weight of (F_i + F_{i+1})
C6F_B = 1.0 / 36.0    # weight of (F_{i-1} + F_{i+2})


def c6_faces(Fn, d, grid):
    """Compact sixth-order interface fluxes along d (R28), stored at node i for the face
    i+1/2; defined on faces -1/2 .. n-1/2 (NaN elsewhere).  Fn: (m, ...) node fluxes,
    needed at positions -2 .. n+1 along d."""
    ax = axis_of(Fn, d)
    g, n = grid.g[d], grid.n[d]
    Fm = np.moveaxis(Fn, ax, 0)
    N = Fm.shape[0]
    cols = Fm.reshape(N, -1)
    out = np.full_like(cols, np.nan)
    F = lambda i: cols[g + i]  # noqa: E731  (position i of the line)
    if grid.periodic(d):
        inner = cols[g:g + n]
        rhs = C6F_A * (inner + np.roll(inner, -1, axis=0)) \
            + C6F_B * (np.roll(inner, 1, axis=0) + np.roll(inner, -2, axis=0))
        c = np.zeros(n)
        c[0] = 1.0
        c[1] = C6F_ALPHA
        c[n - 1] += C6F_ALPHA
        faces = np.real(scipy.linalg.solve_circulant(c, rhs, singular='raise'))
        out[g:g + n] = faces
        out[g - 1] = faces[n - 1]
    else:
        i4f = lambda i: (7.0 * (F(i) + F(i + 1)) - (F(i - 1) + F(i + 2))) / 12.0  # noqa: E731
        lo, hi = i4f(-1), i4f(n - 1)
        m = n - 1
        idx = np.arange(m)
        rhs = C6F_A * (cols[g + idx] + cols[g + idx + 1]) + C6F_B * (cols[g + idx - 1] + cols[g + idx + 2])
        rhs[0] -= C6F_ALPHA * lo
        rhs[m - 1] -= C6F_ALPHA * hi
        ab = np.zeros((3, m))
        ab[1, :] = 1.0
        ab[0, 1:] = C6F_ALPHA
        ab[2, :m - 1] = C6F_ALPHA
        # lines through ghost positions of the other directions may hold NaN node fluxes
        # (metrics undefined there); they are solved too but never used
        out[g:g + m] = scipy.linalg.solve_banded((1, 1), ab, rhs, check_finite=False)
        out[g - 1] = lo
        out[g + n - 1] = hi
    return np.moveaxis(out.reshape(Fm.shape), 0, ax)


def lad_interface_flux(W, Gl, M, d, grid, gas, coef, mu_f, kappa_f, order='E4'):
    """LAD interface flux along d at i+1/2 (stored at node i): I4 (LAD-E4) or the compact
    C6 faces (LAD-C6, R28) of the node convective + viscous flux with mu = mu_f + mu*,
    beta = beta*, kappa = kappa_f + kappa*.  Gl: the scheme's computational gradients
    of the primitives (E4 or C6)."""
    D = physical_gradients(Gl, M, grid)
    mu = mu_f + coef[0]
    beta = coef[1]
    kappa = kappa_f + coef[2]
    Fn = convective_node_flux(W, M, d, gas.gamma) + viscous_node_flux(W, D, M, d, gas, mu, beta, kappa)
    if order == 'C6':
        return c6_faces(Fn, d, grid)
    return i4(Fn, d)
