"""The implicit filter (Sec. 2.1; FILTER_CALLS of Alg. 1) along xi by the partition method
(bounded lines of 128 to 2048 unknowns: segment solves per lane joined through their end
unknowns) against the oracle's banded solves, beside the line-tile / PCR kernels it
replaces there (line-tile mask bit 13).  States at 1e-12 of each variable's max norm (FP64:
the same tridiagonal systems, different elimination orders).

Cases: reflective / transmissive walls with 300 and 1030 unknowns per line (several segment
lengths, lines of 2 and 1 unknowns more than a multiple of 64), a FIXED inflow face, the 3D
ramp generator (curvilinear, FIXED inflow, no-slip wall, periodic span), alpha_f 0.49 and
0.3; the whole RK3 step of the per-cell hybrid (the filter keeps the nodes of the dilated
troubled set) and of the global hybrid.
"""
import numpy as np
import pytest

import gpu_util as U
from oracle import grid as ogrid, rhs as orhs, implicit_filter as oflt
from paper_2511_18042_amd import cases

pytestmark = pytest.mark.gpu

T, RF, FX = cases.TRANSMISSIVE, cases.REFLECTIVE, cases.FIXED
NO_PART = 0xFFF | 0x2000


def case_walls(nx, ny=12):
    c = cases.Case(2, (nx, ny, 1), [(RF, T), (T, RF)], h=(1.0 / nx, 0.3 / ny, 1))
    return cases.random_rough_state(c, seed=nx)


def case_fixed(nx=1030, ny=8):
    c = cases.Case(2, (nx, ny, 1), [(FX, T), (T, T)], h=(1.0 / nx, 0.2 / ny, 1))
    return cases.random_rough_state(c, seed=41)


def case_ramp():
    return cases.ramp3d(160, 24, 8)


CASES = {'walls300': lambda: case_walls(300), 'walls1030': lambda: case_walls(1030, 6), 'fixed1030': case_fixed,
         'ramp160': case_ramp}


def _gas(name, c):
    if name == 'ramp160':
        e = c.extra
        return orhs.Gas(gamma=1.4, Re=e['Re'], Pr=e['Pr'], Mref=e['Mref'], suth=e['suth'], viscous=True)
    return orhs.Gas(gamma=c.gamma)


@pytest.mark.parametrize('name', list(CASES))
@pytest.mark.parametrize('alpha', [0.49, 0.3])
@pytest.mark.parametrize('mask', [-1, NO_PART])
def test_filter_parity(name, alpha, mask):
    print('filter', name, alpha, mask, flush=True)
    c = CASES[name]()
    gas = _gas(name, c)
    g = U.oracle_grid(c)
    ref = oflt.filter_state(c.Q, g, alpha, gas=gas)
    ctx, _ = U.gpu_context(c, gas, orhs.Opts(filter_alpha=alpha))
    ctx.set_line_tiles(mask)
    Qd = U.dev(c.Q)
    ctx.lad_filter(Qd)
    out = Qd.cpu().numpy()
    ctx.close()
    U.compare(out, ref, g, U.STAGE_RTOL, label='filter %s %g %d' % (name, alpha, mask))
    # FIXED ghosts are the caller's (rows of interior y; corner ghosts take the y images)
    if name == 'fixed1030':
        assert np.array_equal(out[:, :, 5:-5, :5], c.Q[:, :, 5:-5, :5])


@pytest.mark.parametrize('mode', ['percell', 'global'])
@pytest.mark.parametrize('mask', [-1, NO_PART])
def test_hybrid_rk3_step_with_filter(mode, mask):
    """One RK3 step of the hybrid on rough data with troubled nodes (rho < 0.8): under the
    per-cell switch the third stage's dilated troubled set keeps its unfiltered values;
    under the global switch the step is not filtered at all (its stages ran C-GBR)."""
    torch = U.torch_mod()
    c = case_walls(300)
    gas = orhs.Gas()
    opts = orhs.Opts(grad='E6', hybrid_mode=mode, rho_thr=0.8, p_thr=0.5)
    g = U.oracle_grid(c)
    M = ogrid.node_metrics(g)
    Qn, t1, _, _ = orhs.rk3_step(c.Q, 0.0, 1.0, g, gas, opts, 'hybrid', M)
    ctx, _ = U.gpu_context(c, gas, opts)
    ctx.set_line_tiles(mask)
    Qd = U.dev(c.Q)
    td = torch.zeros(1, dtype=torch.float64, device='cuda')
    ctx.rk3_step('hybrid', Qd, 1.0, td)
    torch.cuda.synchronize()
    ctx.close()
    U.compare(Qd.cpu().numpy(), Qn, g, U.STAGE_RTOL, label='hybrid rk3 %s %d' % (mode, mask))


def test_lad_e4_rk3_step_is_filtered():
    """LAD-E4 steps end with the filter (Alg. 1): the GPU step equals the oracle's stages
    followed by the filter, and differs from the unfiltered stages."""
    torch = U.torch_mod()
    c = case_walls(300)
    gas = orhs.Gas()
    opts = orhs.Opts(grad='E6')
    g = U.oracle_grid(c)
    M = ogrid.node_metrics(g)
    Qn, _, _, _ = orhs.rk3_step(c.Q, 0.0, 1.0, g, gas, opts, 'lad', M)
    Qu, _, _, _ = orhs.rk3_step(c.Q, 0.0, 1.0, g, gas, orhs.Opts(grad='E6', filter_alpha=0.5), 'lad', M)
    ctx, _ = U.gpu_context(c, gas, opts)
    Qd = U.dev(c.Q)
    td = torch.zeros(1, dtype=torch.float64, device='cuda')
    ctx.rk3_step('lad', Qd, 1.0, td)
    torch.cuda.synchronize()
    ctx.close()
    U.compare(Qd.cpu().numpy(), Qn, g, U.STAGE_RTOL, label='lad-e4 filtered step')
    inner = (slice(None),) + g.interior()
    assert np.max(np.abs(Qn[inner] - Qu[inner])) > 1e-6


def case_strong_contact():
    """Problem 1 of the 64-problem batch at 64 x 64: a density ratio of 17 between quadrants;
    the filter after the first (LAD) step rings below zero density there."""
    return cases.batch64(scale=16)[1]


@pytest.mark.parametrize('mode', ['global', 'percell'])
def test_hybrid_filter_positivity_guard(mode):
    """The hybrid's filter keeps the unfiltered state where it would leave a non-physical
    node (R37): the GPU step equals the oracle's guarded step, and no node is non-physical."""
    torch = U.torch_mod()
    c = case_strong_contact()
    gas = orhs.Gas()
    opts = orhs.Opts(grad='E6', hybrid_mode=mode, rho_thr=c.extra['rho_thr'], p_thr=c.extra['p_thr'])
    g = U.oracle_grid(c)
    M = ogrid.node_metrics(g)
    Qn, _, _, bad = orhs.rk3_step(c.Q, 0.0, 1.0, g, gas, opts, 'hybrid', M)
    assert bad == 0
    ctx, _ = U.gpu_context(c, gas, opts)
    Qd = U.dev(c.Q)
    td = torch.zeros(1, dtype=torch.float64, device='cuda')
    ctx.rk3_step('hybrid', Qd, 1.0, td)
    torch.cuda.synchronize()
    assert ctx.poll_status() == 0
    ctx.close()
    out = Qd.cpu().numpy()
    U.compare(out, Qn, g, U.STAGE_RTOL, label='hybrid guard %s' % mode)
    inner = (slice(None),) + g.interior()
    W = orhs.primitives(out[inner], 1.4)
    assert W[0].min() > 0 and W[4].min() > 0


# --- strided directions: register segments joined through their end unknowns (k_filter_seg)
P_ = cases.PERIODIC
SEG_ON = 0xFFF & ~((1 << 7) | (1 << 8))      # no line tiles for the filter along eta / zeta
SEG_OFF = SEG_ON | 0x4000                    # ... and no segment kernel: one lane per line


def _strided(n, bc, seed):
    c = cases.Case(3 if n[2] > 1 else 2, n, bc, h=tuple(1.0 / max(m, 1) for m in n))
    return cases.random_rough_state(c, seed=seed)


STRIDED = {
    'eta300_walls': lambda: _strided((24, 300, 1), [(RF, T), (T, RF)], 5),          # 5 segments of 60
    'eta130_fixed': lambda: _strided((16, 130, 1), [(T, T), (FX, T)], 6),           # 3 segments of 43-44
    'eta70_zeta128': lambda: _strided((20, 70, 128), [(T, T), (RF, T), (P_, P_)], 7),   # 2 x 35; cyclic 2 x 64
    'eta24_zeta40': lambda: _strided((20, 24, 40), [(T, T), (T, T), (P_, P_)], 8),     # one segment each
    'eta384_zeta16': lambda: _strided((12, 384, 16), [(T, T), (T, RF), (P_, P_)], 9),  # 6 x 64; cyclic 1 x 16
}


@pytest.mark.parametrize('name', list(STRIDED))
@pytest.mark.parametrize('alpha', [0.49, 0.3])
@pytest.mark.parametrize('mask', [-1, SEG_ON, SEG_OFF])
def test_filter_strided_segments_parity(name, alpha, mask):
    """The filter along eta and zeta by register segments (k_filter_seg: bounded and
    periodic lines of 16 to 512 unknowns, one to six segments, FIXED ghosts read and never
    written) against the oracle, beside the line tiles (default where lines are few) and the
    one-lane-per-line solves it replaces."""
    print('filter strided', name, alpha, mask, flush=True)
    c = STRIDED[name]()
    gas = orhs.Gas(gamma=c.gamma)
    g = U.oracle_grid(c)
    ref = oflt.filter_state(c.Q, g, alpha, gas=gas)
    ctx, _ = U.gpu_context(c, gas, orhs.Opts(filter_alpha=alpha))
    ctx.set_line_tiles(mask)
    Qd = U.dev(c.Q)
    ctx.lad_filter(Qd)
    out = Qd.cpu().numpy()
    ctx.close()
    U.compare(out, ref, g, U.STAGE_RTOL, label='filter %s %g %d' % (name, alpha, mask))
    if name == 'eta130_fixed':
        assert np.array_equal(out[:, :, :5, 5:-5], c.Q[:, :, :5, 5:-5])
