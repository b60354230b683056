"""Stage right-hand sides, CFL time step and SSP-RK3 (oracle; test infrastructure only).

Paper: Alg. 1 (LAD stage, with the implicit filter after the last stage of a
LAD-C6 step), Alg. 2 (C-GBR stage), Alg. 3 (hybrid: LAD unless
troubled cells exist), Sec. 5 (the hybrid uses LAD-E4 with MEG6 and a density /
pressure criterion for troubled cells; per-cell switching proposed as the
efficient form), Sec. 2.3 (conservative finite difference: node derivative =
difference of interface fluxes; third-order TVD Runge-Kutta).

The stage RHS is  dQ/dt = -J sum_l (F_hat_{l,i+1/2} - F_hat_{l,i-1/2})  on interior
nodes, with Q the physical conserved state (rho, rho u, rho v, rho w, E) and
F_hat the contravariant fluxes of Eq. eq:3.1.1 (convective + viscous).

Readings used here:
  R8   dt = CFL / max_i sum_l (|xi_l . u| + c |xi_l|), xi_l = J l_hat, from U^n,
       the last step clipped to t_end; no viscous limit.
  R11  C-GBR viscous fluxes use the GBR gradients and the physical coefficients.
  R12  per-cell hybrid: troubled flags f, dilated by a (2r+1)^ndim box (r = 3),
       interface flag g_{i+1/2} = f~_i or f~_{i+1}; g selects the C-GBR interface
       flux, otherwise the LAD flux.  The paper's global switch (any troubled
       interior node -> C-GBR everywhere) is kept as mode 'global'.
  R17  Shu-Osher SSP-RK3; flags re-evaluated every stage.
  R18  no fallback of the state: rho <= 0, p <= 0 or a non-finite value after a
       stage is reported (non-physical count).  (Reconstructed interface states have
       one, R36 in the gbr module; the hybrid's filter has one, R37.)
  R24  troubled if rho < rho_thr or p < p_thr (strict).
  R27-R29  LAD-C6: C6 gradients, compact interface fluxes (``Opts.lad = 'C6'``;
       derivatives and lad modules); the tenth-order implicit filter
       (implicit_filter module) after the third stage.
  R35  every stage that ran the LAD-based solver is followed by the filter when it is
       the step's last (Alg. 1 FILTER_CALLS; Alg. 3 runs that solver in the hybrid's LAD
       phases; Sec. 2.1: the solver's central schemes, explicit or compact, carry the
       filter): LAD-E4 and LAD-C6 alike, the global hybrid's LAD stages, and the nodes
       outside the dilated troubled set of a per-cell hybrid stage.  C-GBR stages are
       never filtered (Alg. 2).
  R38  LAD-C6 may march with the classic four-stage RK4 (Sec. 2.1 names RK4,4 beside the
       TVD RK3; Sec. 5 places LAD-C6's filter in the fourth Runge-Kutta stage), the filter
       after the fourth stage; C-GBR and the hybrid keep SSP-RK3 (Sec. 2.3, Sec. 5).
  R37  in a hybrid stage, a node whose filtered state would not be physical (density or
       pressure not positive, or not finite) keeps its unfiltered state.  The paper's
       criterion (Sec. 5) hands the troubled cells to C-GBR, which is never filtered; the
       filter's own ringing at a sharp jump the LAD phase has not yet smoothed (a strong
       contact at t = 0) is such a cell that only shows after the filter.  Pure LAD runs
       keep the plain filter, so the paper's LAD-C6 column of the stability table is not
       altered.
"""
from dataclasses import dataclass

import numpy as np

from . import grid as gr
from .derivatives import gradient
from .implicit_filter import filter_state
from .gbr import gbr_interface_flux, omega_sensor, omega_bar
from .lad import (lad_coefficients, lad_interface_flux, physical_gradients,
                  physical_transport, viscous_node_flux)


@dataclass
class Gas:
    gamma: float = 1.4
    Re: float = 1.0
    Pr: float = 0.72
    Mref: float = 1.0
    suth: float = 110.4 / 108.0
    viscous: bool = False


@dataclass
class Opts:
    grad: str = 'E6'              # 'E6' (MEG6) or 'C4' (MIG4)
    cfl: float = 0.2
    omega_thr: float = 0.01
    mp_eps: float = 1e-20
    mp_alpha: float = 4.0
    C_mu: float = 0.0
    C_beta: float = 1.75
    C_kappa: float = 0.01
    hybrid_mode: str = 'percell'  # 'percell' or 'global'
    rho_thr: float = -1.0
    p_thr: float = -1.0
    dilate: int = 3
    lad: str = 'E4'               # LAD central scheme: 'E4' or 'C6'
    filter_alpha: float = 0.49    # alpha_f of the LAD-C6 filter (0.5: no filter)
    filter_every_stage: bool = False   # R29 alternative: filter after every RK stage
    time_scheme: str = 'rk3'      # 'rk3' (SSP-RK3) or 'rk4' (classic RK4, the LAD scheme only; R38)


def primitives(Q, gamma):
    """(rho, u, v, w, p) from the conserved state (Sec. 2.1)."""
    rho = Q[0]
    u, v, w = Q[1] / rho, Q[2] / rho, Q[3] / rho
    p = (gamma - 1.0) * (Q[4] - 0.5 * rho * (u * u + v * v + w * w))
    return np.stack([rho, u, v, w, p])


def troubled_flags(W, opts):
    """R24: rho < rho_thr or p < p_thr (strict); a non-finite density or pressure is
    troubled too (the comparisons are written so that NaN fails them)."""
    return ~(W[0] >= opts.rho_thr) | ~(W[4] >= opts.p_thr)


def dilate(f, grid, r):
    """Box dilation of a boolean field by r nodes in every active direction."""
    out = f.copy()
    for d in range(grid.ndim):
        acc = out.copy()
        for s in range(1, r + 1):
            acc |= gr.shift(out, s, d, fill=False)
            acc |= gr.shift(out, -s, d, fill=False)
        out = acc
    return out


def interface_selectors(Q, W, grid, opts, scheme, force_flags=None):
    """Per direction boolean arrays g (at node i for the interface i+1/2): True -> C-GBR.
    ``force_flags`` (bool, field shape) replaces the troubled-cell criterion."""
    shape = grid.shape
    if scheme == 'cgbr':
        return [np.ones(shape, bool) for _ in range(grid.ndim)], None
    if scheme == 'lad':
        return [np.zeros(shape, bool) for _ in range(grid.ndim)], None
    f = troubled_flags(W, opts) if force_flags is None else force_flags.astype(bool)
    if opts.hybrid_mode == 'global':
        use = bool(f[grid.interior()].any())
        return [np.full(shape, use) for _ in range(grid.ndim)], f
    ft = dilate(f, grid, opts.dilate)
    return [ft | gr.shift(ft, 1, d, fill=False) for d in range(grid.ndim)], f


def rhs(Q, grid, gas, opts, scheme, M=None, info=None, force_flags=None):
    """dQ/dt (5, Nz, Ny, Nx) on interior nodes (zero on ghosts) for scheme in
    {'cgbr', 'lad', 'hybrid'}.  ``info`` (dict) receives diagnostics: the
    troubled flags, the selectors and, for C-GBR interfaces, the smallest decision
    margin per node (for excusing threshold flips)."""
    gamma = gas.gamma
    Q = Q.copy()
    gr.fill_ghosts_conserved(Q, grid, gas)
    W = primitives(Q, gamma)
    if M is None:
        M = gr.node_metrics(grid)
    sel, flags = interface_selectors(Q, W, grid, opts, scheme, force_flags)
    need_gbr = any(s.any() for s in sel)
    need_lad = any((~s).any() for s in sel)
    mu_f, kappa_f = physical_transport(W, gas)

    if need_gbr:
        G = {l: np.stack([gradient(W[q], l, opts.grad, grid) for q in range(5)])
             for l in range(grid.ndim)}
        Dg = physical_gradients(G, M, grid)
        Om = omega_sensor(W, Dg[1:4], grid) if gas.viscous else None   # R26
    if need_lad:
        G4 = {l: np.stack([gradient(W[q], l, opts.lad, grid) for q in range(5)])
              for l in range(grid.ndim)}
        coef = lad_coefficients(W, G4, M, grid, gas, opts)
        if info is not None:
            info['lad_coef'] = coef

    L = np.zeros_like(Q)
    inner = grid.interior()
    margin = np.full(grid.shape, np.inf)
    for d in range(grid.ndim):
        F = np.zeros_like(Q)
        if need_gbr:
            rec = {} if info is not None else None
            Ob = omega_bar(Om, d) if Om is not None else None
            Fg = gbr_interface_flux(W, G[d], Ob, M, d, gamma, opts.omega_thr,
                                    opts.mp_eps, opts.mp_alpha, record=rec)
            if gas.viscous:
                Fv = viscous_node_flux(W, Dg, M, d, gas, mu_f, np.zeros_like(mu_f), kappa_f)
                Fg = Fg + gr.i4(Fv, d)
            if rec is not None:
                m = np.where(sel[d], rec['margin'], np.inf)
                margin = np.fmin(margin, np.fmin(m, gr.shift(m, -1, d, fill=np.inf)))
            F = np.where(sel[d], Fg, F)
        if need_lad:
            Fl = lad_interface_flux(W, G4, M, d, grid, gas, coef, mu_f, kappa_f, opts.lad)
            F = np.where(sel[d], F, Fl)
        dF = F - gr.shift(F, -1, d)
        L[(slice(None),) + inner] -= M[9][inner] * dF[(slice(None),) + inner]
    if info is not None:
        info['flags'] = flags
        info['selectors'] = sel
        info['margin'] = margin
        info['W'] = W
    return L


def cfl_dt(Q, grid, gas, cfl, M=None):
    """Convective CFL time step from the interior of Q (R8)."""
    if M is None:
        M = gr.node_metrics(grid)
    inner = grid.interior()
    W = primitives(Q[(slice(None),) + inner], gas.gamma)
    Mi = M[(slice(None),) + inner]
    c = np.sqrt(gas.gamma * W[4] / W[0])
    s = np.zeros_like(c)
    for l in range(grid.ndim):
        xl = [Mi[9] * Mi[3 * l + j] for j in range(3)]
        s = s + np.abs(xl[0] * W[1] + xl[1] * W[2] + xl[2] * W[3]) \
            + c * np.sqrt(xl[0] ** 2 + xl[1] ** 2 + xl[2] ** 2)
    return cfl / np.max(s)


RK3_COEF = ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0))


def rk3_stage(Un, Us, dt, stage, grid, gas, opts, scheme, M=None, info=None, force_flags=None):
    """U^{(s+1)} = a U^n + b (U^{(s)} + dt L(U^{(s)})) on interior nodes; ghosts copied from U^n."""
    a, b = RK3_COEF[stage]
    L = rhs(Us, grid, gas, opts, scheme, M, info, force_flags)
    out = Un.copy()
    inner = (slice(None),) + grid.interior()
    out[inner] = a * Un[inner] + b * (Us[inner] + dt * L[inner])
    return out


def nonphysical_count(Q, grid, gamma):
    inner = (slice(None),) + grid.interior()
    W = primitives(Q[inner], gamma)
    bad = (~np.isfinite(Q[inner]).all(axis=0)) | (W[0] <= 0.0) | (W[4] <= 0.0)
    return int(bad.sum())


def stage_filter(U, info, grid, gas, opts, scheme):
    """FILTER_CALLS after a stage that ran the LAD-based solver (Alg. 1; Alg. 3 calls that
    solver in the hybrid's LAD phases; Sec. 2.1: the central schemes, explicit or compact,
    carry the low-pass implicit filter) (R29, R35).

    'lad'            : the whole field is filtered.
    'hybrid' global  : filtered when the stage found no troubled interior node (it ran
                       LAD everywhere), left alone otherwise (C-GBR, Alg. 2: no filter).
    'hybrid' percell : nodes outside the dilated troubled set take the filtered value,
                       the C-GBR nodes keep theirs.
    'cgbr'           : never filtered.
    ``info`` is the stage's RHS diagnostics (troubled flags)."""
    if not opts.filter_alpha < 0.5 or scheme == 'cgbr':
        return U
    if scheme == 'lad':
        return filter_state(U, grid, opts.filter_alpha, gas=gas)
    f = info['flags']
    if opts.hybrid_mode == 'global':
        if f[grid.interior()].any():
            return U
        return physical_or_unfiltered(filter_state(U, grid, opts.filter_alpha, gas=gas), U, grid, gas)
    if not f.any():          # the per-cell form's interface flags come from every node
        return physical_or_unfiltered(filter_state(U, grid, opts.filter_alpha, gas=gas), U, grid, gas)
    return physical_or_unfiltered(filter_state(U, grid, opts.filter_alpha, gas=gas, keep=dilate(f, grid, opts.dilate)),
                                  U, grid, gas)


def physical_or_unfiltered(Uf, U, grid, gas):
    """R37: interior nodes of the filtered state Uf whose density or pressure is not positive
    (or not finite) take the unfiltered state U; ghost layers are refilled afterwards."""
    inner = (slice(None),) + grid.interior()
    W = primitives(Uf[inner], gas.gamma)
    bad = (~np.isfinite(Uf[inner]).all(axis=0)) | ~(W[0] > 0.0) | ~(W[4] > 0.0)
    if not bad.any():
        return Uf
    out = Uf.copy()
    out[inner] = np.where(bad[None], U[inner], Uf[inner])
    gr.fill_ghosts_conserved(out, grid, gas)
    return out


def rk3_step(Q, t, t_end, grid, gas, opts, scheme, M=None):
    """One SSP-RK3 step (R8, R17); the third stage is followed by the implicit filter where
    it ran LAD (R29, R35; after every stage with ``opts.filter_every_stage``).
    Returns (Q_new, t_new, dt, nonphysical_count)."""
    if M is None:
        M = gr.node_metrics(grid)
    dt = min(cfl_dt(Q, grid, gas, opts.cfl, M), t_end - t)
    bad = 0
    U = Q
    for s in range(3):
        info = {} if scheme == 'hybrid' else None
        U = rk3_stage(Q, U, dt, s, grid, gas, opts, scheme, M, info=info)
        if s == 2 or opts.filter_every_stage:
            U = stage_filter(U, info, grid, gas, opts, scheme)
        bad += nonphysical_count(U, grid, gas.gamma)
    return U, t + dt, dt, bad


RK4_NODES = (0.5, 0.5, 1.0)                          # stage s + 1 input: U^n + c_s dt k_s
RK4_WEIGHTS = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)   # U^{n+1} = U^n + dt sum_s b_s k_s


def rk4_stages(Q, dt, grid, gas, opts, scheme, M=None):
    """The four stages of the classic RK4 (R38) with step dt; the filter follows the fourth
    stage (after every stage with ``opts.filter_every_stage``).  Returns (U^{n+1},
    non-physical count over the stage results)."""
    inner = (slice(None),) + grid.interior()
    acc = np.zeros_like(Q[inner])
    U = Q
    bad = 0
    for s in range(4):
        k = rhs(U, grid, gas, opts, scheme, M)
        acc = acc + (RK4_WEIGHTS[s] * dt) * k[inner]
        U = Q.copy()
        U[inner] = Q[inner] + (RK4_NODES[s] * dt * k[inner] if s < 3 else acc)
        if s == 3 or opts.filter_every_stage:
            U = stage_filter(U, None, grid, gas, opts, scheme)
        bad += nonphysical_count(U, grid, gas.gamma)
    return U, bad


def rk4_step(Q, t, t_end, grid, gas, opts, scheme, M=None):
    """One classic RK4 step (R38: the LAD scheme's alternative integrator, Sec. 2.1) with the
    time step of R8; returns (Q_new, t_new, dt, nonphysical_count)."""
    if scheme != 'lad':
        raise ValueError('RK4 marches the LAD scheme only (R38)')
    if M is None:
        M = gr.node_metrics(grid)
    dt = min(cfl_dt(Q, grid, gas, opts.cfl, M), t_end - t)
    U, bad = rk4_stages(Q, dt, grid, gas, opts, scheme, M)
    return U, t + dt, dt, bad


def time_step(Q, t, t_end, grid, gas, opts, scheme, M=None):
    """One step of the integrator ``opts.time_scheme`` names."""
    f = rk4_step if opts.time_scheme == 'rk4' else rk3_step
    return f(Q, t, t_end, grid, gas, opts, scheme, M)


def run(Q, t_end, grid, gas, opts, scheme, max_steps=10 ** 9):
    """March to t_end; returns (Q, steps, nonphysical_total)."""
    M = gr.node_metrics(grid)
    t = 0.0
    steps = 0
    bad = 0
    while t < t_end and steps < max_steps:
        Q, t, _, b = time_step(Q, t, t_end, grid, gas, opts, scheme, M)
        bad += b
        steps += 1
    return Q, steps, bad
