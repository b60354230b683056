"""The hybrid's switching record (lg_switch_stats; Sec. 5 reports the share of a run spent
on each scheme): stages counted per hybrid stage, troubled ones where a node is below the
thresholds at the stage's start, checked against the oracle's troubled flags."""
import numpy as np
import pytest

import gpu_util as U
from oracle import rhs as orhs
from paper_2511_18042_amd import cases, lgbr

pytestmark = pytest.mark.gpu


def _case():
    c = cases.triple_point(224, 96)
    return c


def _opts(mode, rho_thr):
    return orhs.Opts(grad='E6', hybrid_mode=mode, rho_thr=rho_thr, p_thr=-1.0)


@pytest.mark.parametrize('mode', ['global', 'percell'])
@pytest.mark.parametrize('rho_thr,troubled', [(2.0, True), (-1.0, False)])
def test_switch_stats_count_every_stage(mode, rho_thr, troubled):
    torch = U.torch_mod()
    c = _case()
    gas = orhs.Gas(gamma=c.gamma)
    ctx, _ = U.gpu_context(c, gas, _opts(mode, rho_thr))
    assert ctx.switch_stats() == (0, 0)
    Qd = U.dev(c.Q)
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    for _ in range(3):
        ctx.rk3_step('hybrid', Qd, 10.0, t)
    assert ctx.switch_stats(reset=True) == (9, 9 if troubled else 0)
    assert ctx.switch_stats() == (0, 0)
    ctx.rk3_step('cgbr', Qd, 10.0, t)            # other schemes do not count
    ctx.rk3_step('lad', Qd, 10.0, t)
    assert ctx.switch_stats() == (0, 0)
    ctx.close()


def test_switch_stats_follow_the_oracle_flags():
    """A threshold between the two densities of the state: troubled nodes exist (the
    oracle's flags say so) and the one hybrid RHS call counts one troubled stage; a
    threshold below both counts none."""
    c = _case()
    gas = orhs.Gas(gamma=c.gamma)
    g = U.oracle_grid(c)
    for rho_thr, expect in ((0.5, 1), (0.1, 0)):
        opts = _opts('global', rho_thr)
        info = {}
        orhs.rhs(c.Q, g, gas, opts, 'hybrid', info=info)
        assert int(np.any(info['flags'][g.interior()])) == expect
        ctx, _ = U.gpu_context(c, gas, opts)
        U.gpu_rhs(ctx, c, 'hybrid')
        assert ctx.switch_stats() == (1, expect)
        ctx.close()


def test_switch_stats_in_a_batch():
    torch = U.torch_mod()
    ctxs, Qs, ts = [], [], []
    for rho_thr in (2.0, -1.0):
        c = _case()
        ctx, _ = U.gpu_context(c, orhs.Gas(gamma=c.gamma), _opts('global', rho_thr))
        ctxs.append(ctx)
        Qs.append(U.dev(c.Q))
        ts.append(torch.zeros(1, dtype=torch.float64, device='cuda'))
    b = lgbr.Batch(ctxs, Qs, ts, [10.0, 10.0], 4, 'hybrid')
    b.run()
    b.run()
    torch.cuda.synchronize()
    assert ctxs[0].switch_stats() == (24, 24)
    assert ctxs[1].switch_stats() == (24, 0)
    b.close()
    for ctx in ctxs:
        ctx.close()
