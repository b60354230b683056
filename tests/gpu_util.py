"""Helpers shared by the GPU parity tests: run a case through the C ABI and through the
oracle on the same seeded input, and compare them under the stated tolerance rule.

Tolerance rule (FP64 path):
  * per-stage state: max |U_gpu - U_oracle| <= 1e-12 * max |U_oracle| per conserved variable;
  * right-hand side: max |L_gpu - L_oracle| <= 1e-10 * max |L_oracle| per conserved variable
    (the RHS is a flux difference scaled by J; rounding of O(1e-16 |F|) in the fluxes
    becomes O(1e-15) of the largest RHS on data with O(1) jumps, so 1e-10 leaves margin);
  * every bound also carries an absolute floor of 1e-12 times the largest value over all
    five variables, so that a component that vanishes identically (e.g. the y-momentum RHS
    of a flow at rest) is not compared against its own round-off;
  * a node may exceed the bound only if the oracle recorded a threshold decision on one of
    its interfaces within 1e-10 of the threshold (R22); at most 0.1 % of nodes.
"""
import numpy as np

from oracle import grid as ogrid, rhs as orhs
from paper_2511_18042_amd import cases, lgbr

RHS_RTOL = 1e-10
STAGE_RTOL = 1e-12
MARGIN = 1e-10


def torch_mod():
    import torch
    return torch


def dev(a, dtype=None):
    torch = torch_mod()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def oracle_grid(c):
    return ogrid.Grid(c.ndim, c.n, c.bc, c.h, c.coords, wall_T=c.wall_T)


def gpu_context(c, gas, opts, precision='fp64', stream=None):
    """Context for case c; curvilinear metrics are computed on the GPU from the coordinates."""
    torch = torch_mod()
    curv = c.coords is not None
    g = lgbr.make_grid(c.ndim, c.n, c.bc, c.h, curvilinear=curv, wall_T=c.wall_T)
    metrics = coords = None
    if curv:
        coords = dev(c.coords)
        metrics = torch.zeros((10,) + tuple(c.shape), dtype=torch.float64, device='cuda')
        lgbr.metrics_from_coords(g, coords, metrics)
    ga = lgbr.make_gas(gas.gamma, gas.Re, gas.Pr, gas.Mref, gas.suth, gas.viscous)
    op = lgbr.make_opts(grad=opts.grad, precision=precision, cfl=opts.cfl, omega_thr=opts.omega_thr,
                        mp_eps=opts.mp_eps, mp_alpha=opts.mp_alpha, C_mu=opts.C_mu, C_beta=opts.C_beta,
                        C_kappa=opts.C_kappa, hybrid_mode=opts.hybrid_mode, rho_thr=opts.rho_thr,
                        p_thr=opts.p_thr, dilate=opts.dilate, lad=opts.lad, filter_alpha=opts.filter_alpha,
                        filter_every_stage=opts.filter_every_stage, time_scheme=opts.time_scheme)
    return lgbr.Context(g, ga, op, metrics, coords, stream), metrics


def gpu_rhs(ctx, c, scheme, Q=None, flags=None):
    torch = torch_mod()
    Qd = dev(c.Q if Q is None else Q)
    dQ = torch.zeros_like(Qd)
    fl = None if flags is None else dev(flags.astype(np.uint8))
    ctx.rhs(scheme, Qd, dQ, fl)
    torch.cuda.synchronize()
    return dQ.cpu().numpy()


def excused_mask(info, grid):
    m = info.get('margin')
    if m is None:
        return np.zeros(grid.shape, bool)
    return m <= MARGIN


def compare(gpu, ref, grid, rtol, excuse=None, label=''):
    """Per-variable max-norm relative comparison on interior nodes; returns the number of
    excused nodes.  Raises AssertionError with details otherwise."""
    inner = grid.interior()
    n_nodes = int(np.prod([s.stop - s.start for s in inner]))
    bad_any = np.zeros(grid.shape, bool)
    floor = 1e-12 * max(np.max(np.abs(ref[q][inner])) for q in range(ref.shape[0]))
    for q in range(ref.shape[0]):
        r = ref[q][inner]
        gv = gpu[q][inner]
        scale = np.max(np.abs(r))
        if scale == 0.0:
            scale = 1.0
        err = np.abs(gv - r)
        bad = ~(err <= rtol * scale + floor)
        full = np.zeros(grid.shape, bool)
        full[inner] = bad
        bad_any |= full
    if excuse is None:
        excuse = np.zeros(grid.shape, bool)
    unexcused = bad_any & ~excuse
    n_exc = int((bad_any & excuse).sum())
    if unexcused.any():
        idx = np.argwhere(unexcused)[:5]
        worst = []
        for q in range(ref.shape[0]):
            r = ref[q][inner]
            worst.append(float(np.max(np.abs(gpu[q][inner] - r)) / max(np.max(np.abs(r)), 1e-300)))
        raise AssertionError('%s: %d mismatching nodes (first %s); worst rel err per var %s'
                             % (label, int(unexcused.sum()), idx.tolist(), worst))
    assert n_exc <= max(1, int(1e-3 * n_nodes)), '%s: %d excused nodes > 0.1%%' % (label, n_exc)
    if n_exc:   # reported, so that a run shows every excusal it relied on
        print('EXCUSED %s: %d nodes (oracle margin <= %g)' % (label, n_exc, MARGIN), flush=True)
    return n_exc
