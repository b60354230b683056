"""Digital-filter inflow turbulence (Sec. 4, the 3D cases' inflow; reading R33).

Test infrastructure: a plain FP64 statement of the generator that the library's inflow
update is compared with.  The paper names the method family (digital filters, with
separate integral length scales per velocity component, two wall-normal zones, Table of
length scales, and the strong Reynolds analogy for temperature and density) but prints
none of its formulas; R33 takes the exponential-filter form with time correlation:

  1. per update, independent standard normal numbers r_c(j, k) for c = u, v, w on the
     inflow rows extended by the filter support along eta (k: spanwise, periodic) --
     drawn by the caller and passed in;
  2. filter coefficients b_i = exp(-pi |i| / n) / sqrt(sum_l exp(-2 pi |l| / n)),
     |i| <= N = ceil(2 n), with n = I / Delta the length scale in grid spacings: along
     eta per row (local spacing, the inner or outer scale by the row's wall distance
     against y_lim), along zeta per component;
     psi_new_c(j, k) = sum_i sum_l b^eta_{c,j}(i) b^zeta_c(l) r_c(j + i, k + l);
  3. time correlation over T_c = I_x,c / U_ref (Taylor's hypothesis):
     psi_c <- psi_c exp(-pi dt / (2 T_c)) + psi_new_c sqrt(1 - exp(-pi dt / T_c)),
     psi_c = psi_new_c on the first update;
  4. velocity fluctuations by the Cholesky factor of the Reynolds stresses (Lund):
     u' = a11 psi_u, v' = a21 psi_u + a22 psi_v, w' = a33 psi_w with a11 = sqrt(R11),
     a21 = R21 / a11, a22 = sqrt(R22 - a21^2), a33 = sqrt(R33) (zero where R11 = 0);
  5. strong Reynolds analogy with the local mean Mach number M^2 = M_sra^2 U^2 / (U_ref^2 T)
     (T in units of the reference temperature): T'/T = -(gamma - 1) M^2 u'/U
     = -(gamma - 1) M_sra^2 U u' / (U_ref^2 T); rho'/rho = -T'/T, pressure unchanged;
  6. every ghost layer of the low-xi face (FIXED) takes the plane's state
     (rho(1 + rho'/rho), U + u', V + v', w', p).
"""
import math

import numpy as np

from .grid import NG


def df_coefficients(n):
    """Filter coefficients b_i, i = -N..N, for a length scale of n grid spacings (step 2)."""
    n = max(float(n), 1e-12)
    N = int(math.ceil(2.0 * n))
    i = np.arange(-N, N + 1)
    b = np.exp(-math.pi * np.abs(i) / n)
    return b / math.sqrt(np.sum(b * b))


class DFSpec:
    """What the generator needs (all arrays over the ny interior inflow rows).

    dy, y      : row spacing and wall distance of each row
    dz         : spanwise spacing (uniform, periodic)
    y_lim      : inner / outer zone boundary (rows with y <= y_lim take the inner scale)
    Iy         : Iy[c] = (inner, outer) wall-normal length scales, c = u, v, w
    Iz, Ix     : spanwise and streamwise length scales per component
    U_ref      : convection velocity of Taylor's hypothesis and of the analogy
    mean       : (4, ny) mean rho, U, V, T
    rey        : (4, ny) R11, R21, R22, R33
    gamma, M_sra, p : gas ratio, Mach number of the analogy, the (uniform) pressure
    """

    def __init__(self, dy, y, dz, y_lim, Iy, Iz, Ix, U_ref, mean, rey, gamma, M_sra, p):
        self.dy, self.y = np.asarray(dy, float), np.asarray(y, float)
        self.dz, self.y_lim = float(dz), float(y_lim)
        self.Iy, self.Iz, self.Ix = [tuple(map(float, v)) for v in Iy], list(map(float, Iz)), list(map(float, Ix))
        self.U_ref = float(U_ref)
        self.mean, self.rey = np.asarray(mean, float), np.asarray(rey, float)
        self.gamma, self.M_sra, self.p = float(gamma), float(M_sra), float(p)
        self.ny = self.dy.size

    def eta_coefficients(self, c):
        """Per row j the coefficients along eta of component c (inner / outer zone)."""
        return [df_coefficients(self.Iy[c][0 if self.y[j] <= self.y_lim else 1] / self.dy[j])
                for j in range(self.ny)]

    def pad(self):
        """Rows of random numbers beyond the plane on each side (the largest eta support)."""
        return max((b.size - 1) // 2 for c in range(3) for b in self.eta_coefficients(c))


def filter_plane(spec, r):
    """Step 2: r (3, ny + 2 pad, nz) -> psi_new (3, ny, nz)."""
    pad = spec.pad()
    nz = r.shape[2]
    out = np.zeros((3, spec.ny, nz))
    for c in range(3):
        bz = df_coefficients(spec.Iz[c] / spec.dz)
        Nz = (bz.size - 1) // 2
        # along zeta (periodic) for every padded row
        rz = np.zeros_like(r[c])
        for l in range(-Nz, Nz + 1):
            rz += bz[l + Nz] * np.roll(r[c], -l, axis=1)
        for j, by in enumerate(spec.eta_coefficients(c)):
            Ny = (by.size - 1) // 2
            for i in range(-Ny, Ny + 1):
                out[c, j] += by[i + Ny] * rz[pad + j + i]
    return out


def correlate(spec, psi, psi_new, dt, first):
    """Step 3."""
    if first:
        return psi_new.copy()
    out = np.empty_like(psi)
    for c in range(3):
        T = spec.Ix[c] / spec.U_ref
        out[c] = psi[c] * math.exp(-math.pi * dt / (2.0 * T)) + psi_new[c] * math.sqrt(1.0 - math.exp(-math.pi * dt / T))
    return out


def inflow_plane(spec, psi):
    """Steps 4-5: the primitive inflow plane (rho, u, v, w, p) of shape (5, ny, nz)."""
    R11, R21, R22, R33 = spec.rey
    a11 = np.sqrt(R11)
    a21 = np.where(a11 > 0.0, R21 / np.where(a11 > 0.0, a11, 1.0), 0.0)
    a22 = np.sqrt(np.maximum(R22 - a21 * a21, 0.0))
    a33 = np.sqrt(R33)
    up = a11[:, None] * psi[0]
    vp = a21[:, None] * psi[0] + a22[:, None] * psi[1]
    wp = a33[:, None] * psi[2]
    rho, U, V, Tm = spec.mean
    tr = -(spec.gamma - 1.0) * spec.M_sra ** 2 * U[:, None] * up / (spec.U_ref ** 2 * Tm[:, None])   # T'/T
    out = np.empty((5,) + psi.shape[1:])
    out[0] = rho[:, None] * (1.0 - tr)
    out[1] = U[:, None] + up
    out[2] = V[:, None] + vp
    out[3] = wp
    out[4] = spec.p
    return out


def write_inflow_ghosts(Q, grid, plane, gamma):
    """Step 6: every ghost layer of the low-xi face takes the plane's state (conserved)."""
    rho, u, v, w, p = plane
    g1, n1, g2, n2 = grid.g[1], grid.n[1], grid.g[2], grid.n[2]
    cons = np.stack([rho, rho * u, rho * v, rho * w, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)])
    # plane indices (j, k) -> field axes (k, j): Q[q, g2 + k, g1 + j, i]
    for m in range(NG):
        Q[:, g2:g2 + n2, g1:g1 + n1, m] = np.transpose(cons, (0, 2, 1))
    return Q


def update(spec, Q, grid, psi, r, dt, first):
    """One inflow update (steps 2-6): returns the new psi; writes Q's inflow ghosts."""
    psi_new = filter_plane(spec, r)
    psi = correlate(spec, psi, psi_new, dt, first)
    write_inflow_ghosts(Q, grid, inflow_plane(spec, psi), spec.gamma)
    return psi
