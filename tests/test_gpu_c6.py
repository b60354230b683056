"""LAD-C6 on the GPU (through the C ABI) against the FP64 oracle: compact sixth-order
gradients and interface fluxes (lad_rhs, RK stages) and the tenth-order implicit filter
(lad_filter, the end of every rk3_step).

The cases cover every line-solve kernel: LDS line tiles (all five variables of a few
lines), lines too long for a tile by PCR per (line, variable) or one lane per line, short
periodic lines one lane per line; FIXED, reflective, no-slip and transmissive faces;
curvilinear grids with full and planar metric storage.
Tolerances: RHS 1e-10 and states 1e-12 of each variable's max norm (FP64; the two sides
solve the same tridiagonal systems with different elimination orders).
"""
import numpy as np
import pytest

import gpu_util as U
from oracle import grid as ogrid, rhs as orhs, implicit_filter as oflt
from paper_2511_18042_amd import cases, lgbr

pytestmark = pytest.mark.gpu

T, P, RF, NS, FX = cases.TRANSMISSIVE, cases.PERIODIC, cases.REFLECTIVE, cases.NOSLIP, cases.FIXED


def case_1d_fixed():
    c = cases.shu_osher(96)
    return c


def case_1d_periodic():
    c = cases.periodic_case(1, (40,))
    return cases.random_rough_state(c, seed=21)


def case_2d_walls():
    c = cases.Case(2, (67, 45, 1), [(RF, T), (T, RF)], h=(1.0 / 67, 0.7 / 45, 1))
    return cases.random_rough_state(c, seed=13)


def case_2d_periodic_wide():
    """Periodic x lines long enough for the PCR kernels of every system (filter: 512)."""
    c = cases.periodic_case(2, (520, 9), curvilinear=True, amp=0.04)
    return cases.random_smooth_state(c, seed=22)


def case_2d_curv():
    c = cases.periodic_case(2, (70, 37), curvilinear=True, amp=0.06)
    return cases.random_rough_state(c, seed=12)


def case_3d_curv():
    c = cases.periodic_case(3, (21, 14, 12), curvilinear=True, amp=0.05)
    c.bc = [(P, P), (NS, T), (P, P)]
    return cases.random_rough_state(c, seed=14)


def case_ramp():
    return cases.ramp3d(40, 32, 16)


def case_2d_long_x():
    """x lines longer than an LDS line tile holds (PCR per line and variable)."""
    c = cases.Case(2, (1300, 6, 1), [(RF, T), (T, RF)], h=(1.0 / 1300, 0.05 / 6, 1))
    return cases.random_rough_state(c, seed=23)


def case_2d_long_y():
    """y lines longer than a tile: PCR gradients, one lane per line for fluxes and filter."""
    c = cases.Case(2, (6, 1300, 1), [(T, T), (NS, FX)], h=(0.05 / 6, 1.0 / 1300, 1))
    return cases.random_rough_state(c, seed=24)


CASES = {'1d_fixed': case_1d_fixed, '1d_periodic': case_1d_periodic, '2d_walls': case_2d_walls,
         '2d_periodic_wide': case_2d_periodic_wide, '2d_curv': case_2d_curv, '3d_curv': case_3d_curv,
         'ramp': case_ramp, '2d_long_x': case_2d_long_x, '2d_long_y': case_2d_long_y}


def _gas(name, c):
    if name == '3d_curv':
        return orhs.Gas(gamma=1.4, viscous=True, Re=300.0, Mref=0.8, Pr=0.72)
    if name == 'ramp':
        e = c.extra
        return orhs.Gas(gamma=1.4, Re=e['Re'], Pr=e['Pr'], Mref=e['Mref'], suth=e['suth'], viscous=True)
    return orhs.Gas(gamma=c.gamma)


def _opts(alpha=0.49, every=False):
    return orhs.Opts(lad='C6', filter_alpha=alpha, C_mu=0.002, filter_every_stage=every)


# line-solve kernels: LDS line tiles everywhere (also on strided directions whatever their
# line count: bit 12), or the PCR / lane-per-line kernels only
TILES = {'default': -1, 'tiles': 0xFFF, 'strided_tiles': 0x1FFF, 'no_tiles': 0}


@pytest.mark.parametrize('name', list(CASES))
@pytest.mark.parametrize('tiles', list(TILES))
def test_lad_c6_rhs_parity_fp64(name, tiles):
    print('case', name, tiles, flush=True)
    c = CASES[name]()
    gas, opts = _gas(name, c), _opts()
    g = U.oracle_grid(c)
    ref = orhs.rhs(c.Q, g, gas, opts, 'lad')
    ctx, _ = U.gpu_context(c, gas, opts)
    ctx.set_line_tiles(TILES[tiles])
    assert ctx.get_line_tiles() == (TILES[tiles] if TILES[tiles] >= 0 else 0xFFF)
    with pytest.raises(lgbr.LgError):
        ctx.set_line_tiles(0x8000)
    assert ctx.get_line_tiles() == (TILES[tiles] if TILES[tiles] >= 0 else 0xFFF)
    out = U.gpu_rhs(ctx, c, 'lad')
    U.compare(out, ref, g, U.RHS_RTOL, label='lad-c6 %s %s' % (name, tiles))
    ctx.close()


@pytest.mark.parametrize('name', ['1d_fixed', '1d_periodic', '2d_walls', '2d_periodic_wide', '3d_curv', 'ramp',
                                  '2d_long_x', '2d_long_y'])
@pytest.mark.parametrize('alpha', [0.49, 0.3])
@pytest.mark.parametrize('tiles', list(TILES))
def test_filter_parity_fp64(name, alpha, tiles):
    print('filter', name, alpha, tiles, flush=True)
    torch = U.torch_mod()
    c = CASES[name]()
    gas, opts = _gas(name, c), _opts(alpha)
    g = U.oracle_grid(c)
    ref = oflt.filter_state(c.Q, g, alpha)
    ctx, _ = U.gpu_context(c, gas, opts)
    ctx.set_line_tiles(TILES[tiles])
    Qd = U.dev(c.Q)
    ctx.lad_filter(Qd)
    torch.cuda.synchronize()
    got = Qd.cpu().numpy()
    U.compare(got, ref, g, U.STAGE_RTOL, label='filter ' + name)
    # FIXED ghosts are the caller's and stay untouched
    if name == '1d_fixed':
        assert np.array_equal(got[:, :, :, :5], c.Q[:, :, :, :5])
    ctx.close()


# measured conditioning of the two-step result (see the test's docstring)
RK3_RTOL = {'2d_periodic_wide': 1e-9}


@pytest.mark.parametrize('name,every', [(n, False) for n in ('2d_walls', '1d_fixed', '3d_curv', '2d_periodic_wide')] +
                         [(n, True) for n in ('2d_walls', '3d_curv', '2d_periodic_wide')])
def test_lad_c6_rk3_step_parity_fp64(name, every):
    """Three stages and the filter (after the last stage, or after every stage); two steps in
    a row.  Left out, because LAD alone loses positivity on them within two steps in the
    oracle as on the GPU: the 40x32x16 ramp crop (E4 or C6), and the 96-cell Shu-Osher
    tube with the filter after every stage.

    Tolerance: 1e-12 where the step is well conditioned.  On the 520 x 9 periodic case a
    1e-15 relative perturbation of the input moves the oracle's own two-step result by up
    to 5.3e-11 in rho u (the LAD switch f_sw at nodes where theta and omega both nearly
    vanish), every other case by about 1e-14; there the bound is 1e-9."""
    print('rk3', name, every, flush=True)
    torch = U.torch_mod()
    c = CASES[name]()
    gas, opts = _gas(name, c), _opts(every=every)
    g = U.oracle_grid(c)
    M = ogrid.node_metrics(g)
    ctx, _ = U.gpu_context(c, gas, opts)
    Qd = U.dev(c.Q)
    td = torch.zeros(1, dtype=torch.float64, device='cuda')
    Q, t = c.Q, 0.0
    for step in range(2):
        ctx.rk3_step('lad', Qd, 10.0, td)
        Q, t, dt, bad = orhs.rk3_step(Q, t, 10.0, g, gas, opts, 'lad', M)
        torch.cuda.synchronize()
        assert bad == 0
        assert abs(td.item() - t) <= 1e-13 * t
        U.compare(Qd.cpu().numpy(), Q, g, RK3_RTOL.get(name, U.STAGE_RTOL), label='lad-c6 rk3 %s step %d' % (name, step))
    assert ctx.poll_status() == 0
    ctx.close()


def test_lad_c6_stages_leave_the_filter_to_the_step():
    """lg_rk3_stage runs no filter; rk3_step = three stages + lad_filter."""
    torch = U.torch_mod()
    c = case_2d_walls()
    gas, opts = orhs.Gas(), _opts()
    g = U.oracle_grid(c)
    M = ogrid.node_metrics(g)
    dt = orhs.cfl_dt(c.Q, g, gas, 0.2, M)
    ctx, _ = U.gpu_context(c, gas, opts)
    Un, Us = c.Q, c.Q
    for s in range(3):
        ref = orhs.rk3_stage(Un, Us, dt, s, g, gas, opts, 'lad', M)
        Und, Usd = U.dev(Un), U.dev(Us)
        ctx.rk3_stage('lad', s, Und, Usd, dt)
        torch.cuda.synchronize()
        U.compare(Usd.cpu().numpy(), ref, g, U.STAGE_RTOL, label='c6 stage %d' % s)
        Us = ref
    ctx.lad_filter(Usd)
    Qd = U.dev(c.Q)
    td = torch.zeros(1, dtype=torch.float64, device='cuda')
    ctx.rk3_step('lad', Qd, 10.0, td)
    torch.cuda.synchronize()
    inner = (slice(None),) + g.interior()
    a, b = Usd.cpu().numpy()[inner], Qd.cpu().numpy()[inner]
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))
    ctx.close()


def test_lad_c6_mixed_precision_on_smooth_data():
    """FP32 bulk (node fluxes, coefficients, gradients stored in FP32; solves and state in
    FP64): RHS within 1e-4 of the largest oracle value per variable, the bound used for the
    other schemes (FP32 rounding 6e-8 of the node fluxes amplified by the flux-difference
    cancellation, |F| / |dF| of order 10^3 on this grid)."""
    c = case_2d_periodic_wide()
    gas, opts = orhs.Gas(), _opts()
    g = U.oracle_grid(c)
    ref = orhs.rhs(c.Q, g, gas, opts, 'lad')
    ctx, _ = U.gpu_context(c, gas, opts, precision='mixed')
    out = U.gpu_rhs(ctx, c, 'lad')
    U.compare(out, ref, g, 1e-4, label='lad-c6 mixed')
    ctx.close()


@pytest.mark.parametrize('every', [False, True])
def test_lad_c6_batch_graph_matches_the_oracle(every):
    """Two problems of different sizes, two steps per captured graph, replayed twice."""
    torch = U.torch_mod()
    cs = [case_2d_walls(), cases.random_rough_state(cases.Case(2, (40, 52, 1), [(T, T), (RF, RF)],
                                                              h=(1.0 / 40, 1.0 / 52, 1)), seed=31)]
    gas, opts = orhs.Gas(), _opts(every=every)
    ctxs, Qs, ts = [], [], []
    for c in cs:
        ctx, _ = U.gpu_context(c, gas, opts)
        ctxs.append(ctx)
        Qs.append(U.dev(c.Q))
        ts.append(torch.zeros(1, dtype=torch.float64, device='cuda'))
    b = lgbr.Batch(ctxs, Qs, ts, [10.0, 10.0], 2, 'lad')
    for _ in range(2):
        b.run()
        torch.cuda.synchronize()
    for c, Qd, td in zip(cs, Qs, ts):
        g = U.oracle_grid(c)
        M = ogrid.node_metrics(g)
        Q, t = c.Q, 0.0
        for _ in range(4):
            Q, t, _, _ = orhs.rk3_step(Q, t, 10.0, g, gas, opts, 'lad', M)
        assert abs(td.item() - t) <= 1e-13 * t
        U.compare(Qd.cpu().numpy(), Q, g, U.STAGE_RTOL * 10, label='c6 batch')
    b.close()
    for ctx in ctxs:
        ctx.close()


def test_lad_c6_context_refuses_the_hybrid_and_filter_needs_alpha_below_half():
    """The hybrid's LAD is LAD-E4 (Sec. 5), so LAD-C6 contexts refuse it; the filter runs on
    any context with alpha_f < 1/2 (every LAD phase ends with it, Alg. 1) and is refused at
    alpha_f = 1/2 (no filter)."""
    torch = U.torch_mod()
    c = case_2d_walls()
    ctx, _ = U.gpu_context(c, orhs.Gas(), _opts())
    Qd = U.dev(c.Q)
    dQ = torch.zeros_like(Qd)
    with pytest.raises(lgbr.LgError) as e:
        ctx.hybrid_rhs(Qd, dQ)
    assert e.value.code == lgbr.LG_EUNSUPPORTED
    ctx.close()
    for opts in (orhs.Opts(filter_alpha=0.5), _opts(alpha=0.5)):     # alpha_f = 1/2: no filter
        ctx, _ = U.gpu_context(c, orhs.Gas(), opts)
        with pytest.raises(lgbr.LgError) as e:
            ctx.lad_filter(Qd)
        assert e.value.code == lgbr.LG_EUNSUPPORTED
        ctx.close()


@pytest.mark.parametrize('name,every', [(n, False) for n in ('2d_walls', '1d_fixed', '3d_curv', '2d_curv')] +
                         [('2d_walls', True), ('3d_curv', True)])
@pytest.mark.parametrize('lad', ['C6', 'E4'])
def test_lad_rk4_step_parity_fp64(name, every, lad):
    """The classic RK4 (R38): four stages, the filter after the fourth (or after every stage);
    two steps in a row against the oracle, at 1e-12 of each variable's max norm.  (Cases on
    which LAD alone stays physical for two steps in the oracle.)"""
    print('rk4', name, every, lad, flush=True)
    torch = U.torch_mod()
    c = CASES[name]()
    gas = _gas(name, c)
    opts = orhs.Opts(lad=lad, filter_alpha=0.49, C_mu=0.002, filter_every_stage=every, time_scheme='rk4')
    g = U.oracle_grid(c)
    M = ogrid.node_metrics(g)
    ctx, _ = U.gpu_context(c, gas, opts)
    Qd = U.dev(c.Q)
    td = torch.zeros(1, dtype=torch.float64, device='cuda')
    Q, t = c.Q, 0.0
    for step in range(2):
        ctx.rk3_step('lad', Qd, 10.0, td)
        Q, t, dt, bad = orhs.rk4_step(Q, t, 10.0, g, gas, opts, 'lad', M)
        torch.cuda.synchronize()
        assert bad == 0
        assert abs(td.item() - t) <= 1e-13 * t
        U.compare(Qd.cpu().numpy(), Q, g, U.STAGE_RTOL, label='lad rk4 %s %s step %d' % (name, lad, step))
    assert ctx.poll_status() == 0
    for scheme in ('cgbr', 'hybrid'):   # RK4 marches the LAD scheme only
        with pytest.raises(lgbr.LgError):
            ctx.rk3_step(scheme, Qd, 10.0, td)
    ctx.close()


def test_lad_c6_rk4_batch_graph_matches_single_steps():
    """Graph-captured batches of RK4 steps equal the same steps one call at a time, bitwise."""
    torch = U.torch_mod()
    c = case_2d_walls()
    gas = _gas('2d_walls', c)
    opts = orhs.Opts(lad='C6', filter_alpha=0.49, time_scheme='rk4')
    ctx, _ = U.gpu_context(c, gas, opts)
    Q1, t1 = U.dev(c.Q), torch.zeros(1, dtype=torch.float64, device='cuda')
    for _ in range(3):
        ctx.rk3_step('lad', Q1, 10.0, t1)
    Q2, t2 = U.dev(c.Q), torch.zeros(1, dtype=torch.float64, device='cuda')
    b = lgbr.Batch([ctx], [Q2], [t2], [10.0], 3, 'lad')
    b.run()
    torch.cuda.synchronize()
    b.close()
    assert torch.equal(Q1, Q2) and torch.equal(t1, t2)
    ctx.close()
