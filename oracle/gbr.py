"""Centralised gradient-based reconstruction with HLLC fluxes (oracle; test infrastructure only).

Paper: Sec. 2.3 -- characteristic transformation of the primitives (waves
acoustic 1,5 / entropy 2 / shear 3,4), centralised interpolation
C^C = (C^{L,Lin} + C^{R,Lin}) / 2, the wave-appropriate selection rule with the
Omega^d sensor and the MP criterion (threshold 1e-20), fifth-order MP upwind
states, and the curvilinear HLLC flux with Roe-averaged wave speeds.

Readings used here:
  R1  GBR linear interface states from node values and gradients:
        C^{L,Lin}_{i+1/2} = C_i     + C'_i / 2     + C''_i / 12
        C^{R,Lin}_{i+1/2} = C_{i+1} - C'_{i+1} / 2 + C''_{i+1} / 12
        C''_j = 2 (C_{j+1} - 2 C_j + C_{j-1}) - (C'_{j+1} - C'_{j-1}) / 2
  R2  MP5 = Suresh & Huynh (1997) monotonicity-preserving fifth-order scheme,
      alpha = 4, beta = 4/3, test threshold 1e-20.
  R3  entropy wave (b = 2): when the MP test passes (product <= 1e-20) the
      central linear value is kept, otherwise the MP5 value is used.
  R4  acoustic "Linear" = the upwind GBR linear state.
  R5  frozen state of the characteristic transformation = the Roe average of nodes
      i and i+1 (the same average the HLLC wave speeds of Sec. 2.3 use):
      rho~ = sqrt(rho_i rho_{i+1}), u~ and H~ weighted by sqrt(rho), c~ from H~ and u~;
      basis n = xi~/|xi~|, t1 = normalise(n x e_m) with m = argmin |n_m| (lowest index
      on ties), t2 = n x t1.  (The arithmetic mean of the two nodes, read first, gives
      sound speeds that mix a dense cold state with a light hot one across strong
      contacts; the reconstructed acoustic fields then lose positivity on Le Blanc's
      shock tube within four steps, while the paper runs it stably.)
  R7  Omega = (pressure switch) x (Ducros ratio); the over-bar is the maximum over
      the node and its two neighbours along the sweep; the left state uses node i,
      the right state node i+1; strict "> 0.01".  The Ducros ratio is regularised
      as (theta^2 + eps) / (theta^2 + |omega|^2 + eps), eps = 1e-32, so that where
      the flow has neither dilatation nor vorticity (a pressure jump at rest) the
      pressure switch alone decides; with eps only in the denominator such a jump
      is never detected and the unlimited acoustic states go negative.
  R16 HLLC star flux F*_K = F_K + S_K (Q*_K - Q_K), |xi~| restored on the Roe
      wave speeds, E^K in the star state read as specific total energy.
  R36 positivity of the reconstructed states: the paper prints no safeguard, yet reports
      C-GBR stable (Sec. 4.1, stability table) on cases where the characteristic
      reconstruction, limited field by field, returns a negative density or pressure at a
      few interfaces (Le Blanc's shock tube, the triple point): there the side whose state
      is not positive takes its upwind node's primitive state (first order), the other side
      keeps its reconstruction.
"""
import numpy as np

from .grid import shift, interface_metrics


# ---------------------------------------------------------------- helpers
def minmod(a, b):
    return 0.5 * (np.sign(a) + np.sign(b)) * np.minimum(np.abs(a), np.abs(b))


def minmod4(w, x, y, z):
    sw = np.sign(w)
    return (0.125 * (sw + np.sign(x)) * np.abs((sw + np.sign(y)) * (sw + np.sign(z)))
            * np.minimum(np.minimum(np.abs(w), np.abs(x)), np.minimum(np.abs(y), np.abs(z))))


def product_test_margin(x1, x2, y1, y2, eps):
    """Distance of P = (x1 - x2)(y1 - y2) from the threshold eps, in units of the
    sensitivity of P to rounding of its four inputs."""
    a = x1 - x2
    b = y1 - y2
    scale = np.abs(a) * (np.abs(y1) + np.abs(y2)) + np.abs(b) * (np.abs(x1) + np.abs(x2)) + 1e-300
    return np.abs(a * b - eps) / scale


def mp5(vm2, vm1, v0, vp1, vp2, alpha=4.0, eps=1e-20):
    """Left-biased MP5 value at i+1/2 from v_{i-2..i+2} (Suresh & Huynh 1997, R2).

    Returns (value, margin of the MP acceptance test)."""
    vor = (2.0 * vm2 - 13.0 * vm1 + 47.0 * v0 + 27.0 * vp1 - 3.0 * vp2) / 60.0
    vmp = v0 + minmod(vp1 - v0, alpha * (v0 - vm1))
    accept = (vor - v0) * (vor - vmp) <= eps
    margin = product_test_margin(vor, v0, vor, vmp, eps)
    djm1 = vm2 - 2.0 * vm1 + v0
    dj = vm1 - 2.0 * v0 + vp1
    djp1 = v0 - 2.0 * vp1 + vp2
    dm4p = minmod4(4.0 * dj - djp1, 4.0 * djp1 - dj, dj, djp1)
    dm4m = minmod4(4.0 * dj - djm1, 4.0 * djm1 - dj, dj, djm1)
    vul = v0 + alpha * (v0 - vm1)
    vav = 0.5 * (v0 + vp1)
    vmd = vav - 0.5 * dm4p
    vlc = v0 + 0.5 * (v0 - vm1) + (4.0 / 3.0) * dm4m
    vmin = np.maximum(np.minimum(np.minimum(v0, vp1), vmd), np.minimum(np.minimum(v0, vul), vlc))
    vmax = np.minimum(np.maximum(np.maximum(v0, vp1), vmd), np.maximum(np.maximum(v0, vul), vlc))
    limited = vor + minmod(vmin - vor, vmax - vor)   # median(vor, vmin, vmax)
    return np.where(accept, vor, limited), margin


def roe_frozen_state(WL, WR, gamma):
    """(rho~, c~) of the Roe average of two primitive states (R5)."""
    rL, rR = WL[0], WR[0]
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    wL, wR = sL / (sL + sR), sR / (sL + sR)

    def enthalpy(Wk):
        q2 = Wk[1] ** 2 + Wk[2] ** 2 + Wk[3] ** 2
        return gamma / (gamma - 1.0) * Wk[4] / Wk[0] + 0.5 * q2

    u = [wL * WL[m] + wR * WR[m] for m in (1, 2, 3)]
    H = wL * enthalpy(WL) + wR * enthalpy(WR)
    c = np.sqrt((gamma - 1.0) * (H - 0.5 * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)))
    return sL * sR, c


def tangents(n):
    """Orthonormal tangents (t1, t2) for unit normals n (3, ...) (R5)."""
    m = np.argmin(np.abs(n), axis=0)
    zero = np.zeros_like(n[0])
    t1 = np.stack([
        np.where(m == 0, zero, np.where(m == 1, -n[2], n[1])),
        np.where(m == 0, n[2], np.where(m == 1, zero, -n[0])),
        np.where(m == 0, -n[1], np.where(m == 1, n[0], zero)),
    ])
    t1 = t1 / np.sqrt(t1[0] ** 2 + t1[1] ** 2 + t1[2] ** 2)
    t2 = np.stack([n[1] * t1[2] - n[2] * t1[1],
                   n[2] * t1[0] - n[0] * t1[2],
                   n[0] * t1[1] - n[1] * t1[0]])
    return t1, t2


def to_characteristic(V, n, t1, t2, rb, cb):
    """Primitive (rho, u, v, w, p) -> characteristic (C1..C5) with the frozen state (R5)."""
    un = n[0] * V[1] + n[1] * V[2] + n[2] * V[3]
    k = rb / (2.0 * cb)
    pc = V[4] / (2.0 * cb * cb)
    return np.stack([
        -k * un + pc,
        V[0] - V[4] / (cb * cb),
        t1[0] * V[1] + t1[1] * V[2] + t1[2] * V[3],
        t2[0] * V[1] + t2[1] * V[2] + t2[2] * V[3],
        k * un + pc,
    ])


def from_characteristic(C, n, t1, t2, rb, cb):
    """Inverse of :func:`to_characteristic`."""
    un = (cb / rb) * (C[4] - C[0])
    return np.stack([
        C[0] + C[1] + C[4],
        n[0] * un + t1[0] * C[2] + t2[0] * C[3],
        n[1] * un + t1[1] * C[2] + t2[1] * C[3],
        n[2] * un + t1[2] * C[2] + t2[2] * C[3],
        cb * cb * (C[0] + C[4]),
    ])


def gbr_linear_states(Cm1, C0, C1, C2, Dm1, D0, D1, D2):
    """Upwind GBR linear states at i+1/2 from values C_{i-1..i+2} and gradients D_{i-1..i+2} (R1)."""
    c2_i = 2.0 * (C1 - 2.0 * C0 + Cm1) - 0.5 * (D1 - Dm1)
    c2_ip = 2.0 * (C2 - 2.0 * C1 + C0) - 0.5 * (D2 - D0)
    return C0 + 0.5 * D0 + c2_i / 12.0, C1 - 0.5 * D1 + c2_ip / 12.0


# ---------------------------------------------------------------- HLLC
def euler_flux(Wk, xt, gamma):
    """Contravariant convective flux (Eq. eq:3.1.1) of primitive state Wk with metric xt."""
    rho, u, v, w, p = Wk
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    U = xt[0] * u + xt[1] * v + xt[2] * w
    return np.stack([rho * U,
                     rho * u * U + xt[0] * p,
                     rho * v * U + xt[1] * p,
                     rho * w * U + xt[2] * p,
                     (E + p) * U])


def hllc(WL, WR, xt, gamma):
    """HLLC flux at an interface with metric xt (3, ...) (Sec. 2.3, R16)."""
    with np.errstate(divide='ignore', invalid='ignore'):
        xn2 = xt[0] ** 2 + xt[1] ** 2 + xt[2] ** 2
        xn = np.sqrt(xn2)

        def parts(Wk):
            rho, u, v, w, p = Wk
            E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
            H = (E + p) / rho
            c = np.sqrt(gamma * p / rho)
            U = xt[0] * u + xt[1] * v + xt[2] * w
            return rho, (u, v, w), p, E, H, c, U

        rL, uL, pL, EL, HL, cL, UL = parts(WL)
        rR, uR, pR, ER, HR, cR, UR = parts(WR)
        R = np.sqrt(rR / rL)
        ub = [(uL[m] + R * uR[m]) / (1.0 + R) for m in range(3)]
        Hb = (HL + R * HR) / (1.0 + R)
        cb = np.sqrt((gamma - 1.0) * (Hb - 0.5 * (ub[0] ** 2 + ub[1] ** 2 + ub[2] ** 2)))
        Ub = xt[0] * ub[0] + xt[1] * ub[1] + xt[2] * ub[2]
        SL = np.minimum(UL - cL * xn, Ub - cb * xn)
        SR = np.maximum(UR + cR * xn, Ub + cb * xn)
        Ss = ((rR * UR * (SR - UR) - rL * UL * (SL - UL) + (pL - pR) * xn2)
              / (rR * (SR - UR) - rL * (SL - UL)))

        def star_flux(rho, u, p, E, U, S):
            F = np.stack([rho * U,
                          rho * u[0] * U + xt[0] * p,
                          rho * u[1] * U + xt[1] * p,
                          rho * u[2] * U + xt[2] * p,
                          (E + p) * U])
            Qk = np.stack([rho, rho * u[0], rho * u[1], rho * u[2], E])
            fac = rho * (S - U) / (S - Ss)
            Qs = np.stack([fac,
                           fac * (u[0] + xt[0] * (Ss - U) / xn2),
                           fac * (u[1] + xt[1] * (Ss - U) / xn2),
                           fac * (u[2] + xt[2] * (Ss - U) / xn2),
                           fac * (E / rho + (Ss - U) * (Ss / xn2 + p / (rho * (S - U))))])
            return F, F + S * (Qs - Qk)

        FL, FsL = star_flux(rL, uL, pL, EL, UL, SL)
        FR, FsR = star_flux(rR, uR, pR, ER, UR, SR)
        F = np.where(SL >= 0.0, FL, np.where(Ss >= 0.0, FsL, np.where(SR > 0.0, FsR, FR)))
        # undefined wave speeds (a state without a sound speed) give an undefined flux
        undefined = np.isnan(SL) | np.isnan(SR) | np.isnan(Ss)
        return np.where(undefined, np.nan, F)


# ---------------------------------------------------------------- sensor
def omega_sensor(W, dudx, grid):
    """Omega at every node (R7): pressure switch x Ducros ratio.

    W    : primitives (5, ...)
    dudx : dudx[i][j] = d u_i / d x_j (3, 3, ...) from the scheme's gradients.
    """
    p = W[4]
    phi = np.zeros_like(p)
    for d in range(grid.ndim):
        pp, pm = shift(p, 1, d), shift(p, -1, d)
        phi = np.maximum(phi, np.abs(pp - 2.0 * p + pm) / (pp + 2.0 * p + pm))
    theta = dudx[0][0] + dudx[1][1] + dudx[2][2]
    w1 = dudx[2][1] - dudx[1][2]
    w2 = dudx[0][2] - dudx[2][0]
    w3 = dudx[1][0] - dudx[0][1]
    om2 = w1 * w1 + w2 * w2 + w3 * w3
    return phi * ((theta * theta + 1e-32) / (theta * theta + om2 + 1e-32))


def omega_bar(Om, d):
    return np.maximum(np.maximum(shift(Om, -1, d), Om), shift(Om, 1, d))


# ---------------------------------------------------------------- interface flux
def gbr_interface_flux(W, G, Ob, M, d, gamma, omega_thr=0.01, mp_eps=1e-20, mp_alpha=4.0,
                       record=None):
    """C-GBR convective flux at every interface i+1/2 along d, stored at node i.

    W  : primitives (5, ...);  G : their derivatives along d (5, ...);
    Ob : Omega-bar along d, or None for inviscid flow, where Sec. 2.3 limits with the MP
         criterion alone: every field takes its linear state (upwind for the acoustic
         fields, central for the others) where the MP test of the entropy rule passes,
         MP5 where it fails (R26);
    M  : node metrics (10, ...).
    If ``record`` is a dict, the smallest decision margin per interface is stored
    under record['margin'] (used to excuse threshold flips, R22).
    """
    Ws = {s: shift(W, s, d) for s in range(-2, 4)}
    Gs = {s: shift(G, s, d) for s in range(-1, 3)}
    xt = interface_metrics(M, d)
    xn = np.sqrt(xt[0] ** 2 + xt[1] ** 2 + xt[2] ** 2)
    n = xt / xn
    t1, t2 = tangents(n)
    rb, cb = roe_frozen_state(Ws[0], Ws[1], gamma)

    C = {s: to_characteristic(Ws[s], n, t1, t2, rb, cb) for s in Ws}
    Cp = {s: to_characteristic(Gs[s], n, t1, t2, rb, cb) for s in Gs}

    CL_lin, CR_lin = gbr_linear_states(C[-1], C[0], C[1], C[2], Cp[-1], Cp[0], Cp[1], Cp[2])
    CC = 0.5 * (CL_lin + CR_lin)

    mpL, mL = mp5(C[-2], C[-1], C[0], C[1], C[2], mp_alpha, mp_eps)
    mpR, mR = mp5(C[3], C[2], C[1], C[0], C[-1], mp_alpha, mp_eps)

    cmpL = C[0] + minmod(C[1] - C[0], mp_alpha * (C[0] - C[-1]))
    cmpR = C[1] + minmod(C[0] - C[1], mp_alpha * (C[1] - C[2]))
    passL = (CL_lin - C[0]) * (CL_lin - cmpL) <= mp_eps
    passR = (CR_lin - C[1]) * (CR_lin - cmpR) <= mp_eps

    CL = np.empty_like(CL_lin)
    CR = np.empty_like(CR_lin)
    if Ob is None:                         # inviscid: MP criterion for every field (R26)
        for b in range(5):
            linL = CL_lin[b] if b in (0, 4) else CC[b]
            linR = CR_lin[b] if b in (0, 4) else CC[b]
            CL[b] = np.where(passL[b], linL, mpL[b])
            CR[b] = np.where(passR[b], linR, mpR[b])
        tested = range(5)
        om = np.inf
    else:
        ObL = Ob
        ObR = shift(Ob, 1, d)
        shockL = ObL > omega_thr
        shockR = ObR > omega_thr
        for b in (0, 4):                       # acoustic waves
            CL[b] = np.where(shockL, mpL[b], CL_lin[b])
            CR[b] = np.where(shockR, mpR[b], CR_lin[b])
        CL[1] = np.where(passL[1], CC[1], mpL[1])   # entropy wave (R3)
        CR[1] = np.where(passR[1], CC[1], mpR[1])
        for b in (2, 3):                       # shear waves
            CL[b] = np.where(shockL, mpL[b], CC[b])
            CR[b] = np.where(shockR, mpR[b], CC[b])
        tested = (1,)
        om = np.minimum(np.abs(ObL - omega_thr), np.abs(ObR - omega_thr)) / omega_thr

    if record is not None:
        t = np.inf
        for b in tested:
            t = np.minimum(t, product_test_margin(CL_lin[b], C[0][b], CL_lin[b], cmpL[b], mp_eps))
            t = np.minimum(t, product_test_margin(CR_lin[b], C[1][b], CR_lin[b], cmpR[b], mp_eps))
        mm = np.minimum(np.min(mL, axis=0), np.min(mR, axis=0))
        record['margin'] = np.minimum(np.minimum(om, mm), t)

    WL0 = from_characteristic(CL, n, t1, t2, rb, cb)
    WR0 = from_characteristic(CR, n, t1, t2, rb, cb)
    # R36: a reconstructed state without positive density and pressure is replaced by its
    # upwind node's own state (first order on that side)
    with np.errstate(invalid='ignore'):
        okL = (WL0[0] > 0.0) & (WL0[4] > 0.0)
        okR = (WR0[0] > 0.0) & (WR0[4] > 0.0)
    WL = np.where(okL, WL0, Ws[0])
    WR = np.where(okR, WR0, Ws[1])
    if record is not None:
        with np.errstate(divide='ignore', invalid='ignore'):
            pos = np.minimum(np.minimum(np.abs(WL0[0] / Ws[0][0]), np.abs(WL0[4] / Ws[0][4])),
                             np.minimum(np.abs(WR0[0] / Ws[1][0]), np.abs(WR0[4] / Ws[1][4])))
        record['margin'] = np.minimum(record['margin'], np.where(np.isfinite(pos), pos, 0.0))
        record['WL'], record['WR'] = WL, WR
    return hllc(WL, WR, xt, gamma)
