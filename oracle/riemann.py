"""Exact solution of the 1D Riemann problem for an ideal gas (oracle; test infrastructure only).

The 1D shock tubes of Sec. 3.1 are compared against the exact Riemann solution.
This is the textbook construction (Toro, "Riemann Solvers and Numerical Methods
for Fluid Dynamics", ch. 4): the star pressure solves
    f_L(p) + f_R(p) + (u_R - u_L) = 0,
with f_K the shock (Rankine-Hugoniot) branch for p > p_K and the rarefaction
(isentropic) branch otherwise; Newton iteration to a relative change < 1e-15;
u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2; the solution is then sampled on x/t.
"""
import numpy as np


def _f_and_df(p, rho, pk, c, gamma):
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        q = np.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
    r = p / pk
    f = 2.0 * c / (gamma - 1.0) * (r ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
    df = 1.0 / (rho * c) * r ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(left, right, gamma):
    """(p*, u*) for left/right primitive states (rho, u, p)."""
    rL, uL, pL = left
    rR, uR, pR = right
    cL = np.sqrt(gamma * pL / rL)
    cR = np.sqrt(gamma * pR / rR)
    p = max(1e-12, 0.5 * (pL + pR) - 0.125 * (uR - uL) * (rL + rR) * (cL + cR))
    for _ in range(200):
        fL, dL = _f_and_df(p, rL, pL, cL, gamma)
        fR, dR = _f_and_df(p, rR, pR, cR, gamma)
        pn = p - (fL + fR + uR - uL) / (dL + dR)
        pn = max(pn, 1e-14)
        done = abs(pn - p) / (0.5 * (pn + p)) < 1e-15
        p = pn
        if done:
            break
    fL, _ = _f_and_df(p, rL, pL, cL, gamma)
    fR, _ = _f_and_df(p, rR, pR, cR, gamma)
    return p, 0.5 * (uL + uR) + 0.5 * (fR - fL)


def residual(p, left, right, gamma):
    rL, uL, pL = left
    rR, uR, pR = right
    fL, _ = _f_and_df(p, rL, pL, np.sqrt(gamma * pL / rL), gamma)
    fR, _ = _f_and_df(p, rR, pR, np.sqrt(gamma * pR / rR), gamma)
    return fL + fR + uR - uL


def sample(left, right, gamma, s):
    """Primitive solution (rho, u, p) at similarity coordinates s = (x - x0) / t (array)."""
    rL, uL, pL = left
    rR, uR, pR = right
    ps, us = star_state(left, right, gamma)
    cL = np.sqrt(gamma * pL / rL)
    cR = np.sqrt(gamma * pR / rR)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    s = np.asarray(s, dtype=float)
    out = np.zeros((3,) + s.shape)
    for idx, x in np.ndenumerate(s):
        if x <= us:                                    # left of the contact
            if ps > pL:                                # left shock
                SL = uL - cL * np.sqrt((gamma + 1.0) / (2 * gamma) * ps / pL + (gamma - 1.0) / (2 * gamma))
                if x <= SL:
                    st = (rL, uL, pL)
                else:
                    st = (rL * (ps / pL + g1) / (g1 * ps / pL + 1.0), us, ps)
            else:                                      # left rarefaction
                csL = cL * (ps / pL) ** ((gamma - 1.0) / (2 * gamma))
                if x <= uL - cL:
                    st = (rL, uL, pL)
                elif x >= us - csL:
                    st = (rL * (ps / pL) ** (1.0 / gamma), us, ps)
                else:
                    c = 2.0 / (gamma + 1.0) * (cL + 0.5 * (gamma - 1.0) * (uL - x))
                    u = 2.0 / (gamma + 1.0) * (cL + 0.5 * (gamma - 1.0) * uL + x)
                    r = rL * (c / cL) ** (2.0 / (gamma - 1.0))
                    st = (r, u, pL * (c / cL) ** (2.0 * gamma / (gamma - 1.0)))
        else:                                          # right of the contact
            if ps > pR:                                # right shock
                SR = uR + cR * np.sqrt((gamma + 1.0) / (2 * gamma) * ps / pR + (gamma - 1.0) / (2 * gamma))
                if x >= SR:
                    st = (rR, uR, pR)
                else:
                    st = (rR * (ps / pR + g1) / (g1 * ps / pR + 1.0), us, ps)
            else:                                      # right rarefaction
                csR = cR * (ps / pR) ** ((gamma - 1.0) / (2 * gamma))
                if x >= uR + cR:
                    st = (rR, uR, pR)
                elif x <= us + csR:
                    st = (rR * (ps / pR) ** (1.0 / gamma), us, ps)
                else:
                    c = 2.0 / (gamma + 1.0) * (cR - 0.5 * (gamma - 1.0) * (uR - x))
                    u = 2.0 / (gamma + 1.0) * (-cR + 0.5 * (gamma - 1.0) * uR + x)
                    r = rR * (c / cR) ** (2.0 / (gamma - 1.0))
                    st = (r, u, pR * (c / cR) ** (2.0 * gamma / (gamma - 1.0)))
        out[(slice(None),) + idx] = st
    return out
