"""LAD-C6 along xi by the partition method, against the oracle's banded solves, through
LAD-C6 right-hand sides (FP64, the RHS tolerance of the other parity tests), beside the
kernels it replaces (LDS line tiles, PCR or one lane per line: mask bit 13):
  * interface fluxes (k_c6_faces_part: bounded lines of 129 to 2049 nodes of 2D and 3D
    problems, the n - 1 interior faces of the [1/3, 1, 1/3] system with the two
    fourth-order boundary faces on its right-hand side; segments per lane joined through
    their end unknowns);
  * gradients (k_grad_part: padded lines of 130 to 2050 nodes, the N - 2 unknowns between
    the decoupled end rows; the constant system by the same scans, the 1/4 neighbours of
    its first and last rows by a Woodbury correction).

Cases: the shortest lines they take (120 nodes: 128 gradient unknowns, 119 faces, which stay
on the tiles; 129 nodes: 128 faces), 300 nodes with reflective and transmissive walls, 1030
nodes with a FIXED inflow face, 2038 nodes (2046 gradient unknowns) and 2049 (2048 faces,
gradients on the PCR kernel), a 3D curvilinear block with a periodic zeta, a 1D line (its
gradients only: 1D faces stay on the PCR kernel) and a periodic line of 200 nodes, which
stays on the other kernels."""
import numpy as np
import pytest

import gpu_util as U
from oracle import rhs as orhs
from paper_2511_18042_amd import cases

pytestmark = pytest.mark.gpu

T, P, RF, NS, FX = cases.TRANSMISSIVE, cases.PERIODIC, cases.REFLECTIVE, cases.NOSLIP, cases.FIXED
NO_PART = 0xFFF | 0x2000


def _case(ndim, n, bc, seed):
    h = tuple(1.0 / m if m > 1 else 1.0 for m in n)
    c = cases.Case(ndim, n, bc, h=h)
    return cases.random_rough_state(c, seed=seed)


def _curv3d():
    c = cases.periodic_case(3, (160, 6, 8), curvilinear=True, amp=0.05)
    c.bc = [(RF, T), (NS, T), (P, P)]
    return cases.random_rough_state(c, seed=46)


CASES = {
    'x120': lambda: _case(2, (120, 8, 1), [(RF, T), (T, T)], 40),
    'x129': lambda: _case(2, (129, 8, 1), [(T, T), (RF, T)], 41),
    'x300_walls': lambda: _case(2, (300, 12, 1), [(RF, T), (T, RF)], 42),
    'x1030_fixed': lambda: _case(2, (1030, 6, 1), [(FX, T), (T, T)], 43),
    'x2038': lambda: _case(2, (2038, 5, 1), [(RF, FX), (T, T)], 49),
    'x2049': lambda: _case(2, (2049, 5, 1), [(T, RF), (T, T)], 44),
    'x160_3d_curv': _curv3d,
    'x200_periodic': lambda: _case(2, (200, 8, 1), [(P, P), (T, T)], 45),
    'x300_1d': lambda: _case(1, (300, 1, 1), [(T, RF)], 47),
}
UNCHANGED = ('x200_periodic',)   # periodic lines stay on the other kernels


def _gas(c):
    if c.ndim == 3:
        return orhs.Gas(gamma=1.4, viscous=True, Re=300.0, Mref=0.8, Pr=0.72)
    return orhs.Gas(gamma=c.gamma)


@pytest.mark.parametrize('name', list(CASES))
def test_c6_partition_parity_fp64(name):
    print('c6 partition', name, flush=True)
    c = CASES[name]()
    gas = _gas(c)
    opts = orhs.Opts(lad='C6', filter_alpha=0.49, C_mu=0.002)
    g = U.oracle_grid(c)
    ref = orhs.rhs(c.Q, g, gas, opts, 'lad')
    outs = []
    for mask in (-1, NO_PART):
        ctx, _ = U.gpu_context(c, gas, opts)
        ctx.set_line_tiles(mask)
        out = U.gpu_rhs(ctx, c, 'lad')
        ctx.close()
        U.compare(out, ref, g, U.RHS_RTOL, label='c6 part %s mask %d' % (name, mask))
        outs.append(out)
    inner = (slice(None),) + g.interior()
    a, b = outs[0][inner], outs[1][inner]
    scale = np.abs(b).reshape(5, -1).max(axis=1)
    scale = np.where(scale > 0, scale, scale.max())
    rel = np.abs(a - b).reshape(5, -1).max(axis=1) / scale
    print('partition vs other kernels', rel.tolist(), flush=True)
    assert rel.max() <= 1e-11
    if name in UNCHANGED:
        assert np.array_equal(a, b)


@pytest.mark.parametrize('precision', ['fp64', 'mixed'])
def test_c6_partition_rk3_steps(precision):
    """Two RK3 steps (three stages and the filter each) with and without the partition
    kernel on 300 x 12 nodes of near-square cells (LAD alone loses positivity within a step
    on the stretched cells of the RHS cases); FP64 also against the oracle's steps."""
    import torch
    from oracle import grid as ogrid
    c = cases.random_rough_state(cases.Case(2, (300, 12, 1), [(RF, T), (T, RF)], h=(1.0 / 300, 0.04 / 12, 1)),
                                 seed=48)
    gas = _gas(c)
    opts = orhs.Opts(lad='C6', filter_alpha=0.49, C_mu=0.002)
    g = U.oracle_grid(c)
    res = []
    for mask in (-1, NO_PART):
        ctx, _ = U.gpu_context(c, gas, opts, precision=precision)
        ctx.set_line_tiles(mask)
        Q = torch.from_numpy(np.ascontiguousarray(c.Q)).cuda()
        t = torch.zeros(1, dtype=torch.float64, device='cuda')
        for _ in range(2):
            ctx.rk3_step('lad', Q, 10.0, t)
        torch.cuda.synchronize()
        assert ctx.poll_status() == 0
        res.append((Q.cpu().numpy(), float(t.item())))
        ctx.close()
    inner = (slice(None),) + g.interior()
    a, b = res[0][0][inner], res[1][0][inner]
    scale = np.abs(b).reshape(5, -1).max(axis=1)
    scale = np.where(scale > 0, scale, scale.max())
    rel = np.abs(a - b).reshape(5, -1).max(axis=1) / scale
    print('rk3 steps partition vs other kernels', precision, rel.tolist(), flush=True)
    assert rel.max() <= (1e-12 if precision == 'fp64' else 1e-5)
    assert abs(res[0][1] - res[1][1]) <= 1e-12 * res[1][1]
    if precision == 'fp64':
        M = ogrid.node_metrics(g)
        Q, t = c.Q, 0.0
        for _ in range(2):
            Q, t, dt, bad = orhs.rk3_step(Q, t, 10.0, g, gas, opts, 'lad', M)
            assert bad == 0
        assert abs(res[0][1] - t) <= 1e-13 * t
        U.compare(res[0][0], Q, g, U.STAGE_RTOL, label='c6 face part rk3')
