"""The hybrid's filter positivity guard (R37) in the oracle: after a LAD phase the implicit
filter (Sec. 2.1, FILTER_CALLS of Alg. 1) rings at a strong contact that the first LAD step
has not smoothed; the nodes it would leave non-physical keep their unfiltered state and no
other node does."""
import numpy as np

from oracle import grid as ogrid, rhs as orhs
from oracle.implicit_filter import filter_state
from paper_2511_18042_amd import cases


def _first_step_parts(mode):
    c = cases.batch64(scale=16)[1]        # density ratio 17 between quadrants, 64 x 64
    g = ogrid.Grid(c.ndim, c.n, c.bc, c.h, c.coords)
    M = ogrid.node_metrics(g)
    gas = orhs.Gas()
    opts = orhs.Opts(grad='E6', hybrid_mode=mode, rho_thr=c.extra['rho_thr'], p_thr=c.extra['p_thr'])
    dt = orhs.cfl_dt(c.Q, g, gas, opts.cfl, M)
    U = c.Q
    for s in range(3):
        info = {}
        U = orhs.rk3_stage(c.Q, U, dt, s, g, gas, opts, 'hybrid', M, info=info)
    assert not info['flags'].any()         # every stage ran LAD
    Qn, _, _, bad = orhs.rk3_step(c.Q, 0.0, 1e30, g, gas, opts, 'hybrid', M)
    return g, U, filter_state(U, g, opts.filter_alpha, gas=gas), Qn, bad


def test_unguarded_filter_is_not_physical_here():
    g, U, Uf, _, _ = _first_step_parts('global')
    inner = (slice(None),) + g.interior()
    assert orhs.nonphysical_count(U, g, 1.4) == 0
    assert orhs.primitives(Uf[inner], 1.4)[0].min() < 0.0


def test_guard_restores_exactly_the_non_physical_nodes():
    for mode in ('global', 'percell'):
        g, U, Uf, Qn, bad = _first_step_parts(mode)
        inner = (slice(None),) + g.interior()
        assert bad == 0
        Wf = orhs.primitives(Uf[inner], 1.4)
        badf = ~(Wf[0] > 0) | ~(Wf[4] > 0)
        assert 0 < badf.sum() < 0.01 * badf.size
        got = Qn[inner]
        assert np.array_equal(got[:, badf], U[inner][:, badf])
        assert np.array_equal(got[:, ~badf], Uf[inner][:, ~badf])
