"""GPU parity of the HIP library (through the C ABI) against the FP64 oracle.

Every case uses the same seeded input on both sides; sizes span several waves / line
segments with ragged tails.  Tolerances and the excusal rule are stated in gpu_util.
"""
import numpy as np
import pytest

import gpu_util as U
from oracle import grid as ogrid, rhs as orhs
from paper_2511_18042_amd import cases, lgbr

pytestmark = pytest.mark.gpu

T, P, RF, NS, FX = cases.TRANSMISSIVE, cases.PERIODIC, cases.REFLECTIVE, cases.NOSLIP, cases.FIXED


def case_1d():
    c = cases.Case(1, (150, 1, 1), [(T, T)], h=(1.0 / 150, 1, 1))
    return cases.random_rough_state(c, seed=11)


def case_2d_curv():
    c = cases.periodic_case(2, (70, 37), curvilinear=True, amp=0.06)
    return cases.random_rough_state(c, seed=12)


def case_2d_walls():
    c = cases.Case(2, (67, 45, 1), [(RF, T), (T, RF)], h=(1.0 / 67, 0.7 / 45, 1))
    return cases.random_rough_state(c, seed=13)


def case_3d_curv():
    c = cases.periodic_case(3, (21, 14, 12), curvilinear=True, amp=0.05)
    c.bc = [(P, P), (NS, T), (P, P)]
    return cases.random_rough_state(c, seed=14)


CASES = {'1d': case_1d, '2d_curv': case_2d_curv, '2d_walls': case_2d_walls, '3d_curv': case_3d_curv}
SCHEMES = [('cgbr', 'E6', 'percell'), ('cgbr', 'C4', 'percell'), ('lad', 'E6', 'percell'),
           ('hybrid', 'E6', 'percell'), ('hybrid', 'C4', 'global')]


def _gas(name):
    if name == '3d_curv':
        return orhs.Gas(gamma=1.4, viscous=True, Re=300.0, Mref=0.8, Pr=0.72)
    return orhs.Gas(gamma=1.4)


def _opts(grad, mode):
    return orhs.Opts(grad=grad, hybrid_mode=mode, rho_thr=0.8, p_thr=0.5, C_mu=0.002)


@pytest.mark.parametrize('name', list(CASES))
@pytest.mark.parametrize('scheme,grad,mode', SCHEMES)
def test_rhs_parity_fp64(name, scheme, grad, mode):
    print('case', name, scheme, grad, mode, flush=True)
    c = CASES[name]()
    gas, opts = _gas(name), _opts(grad, mode)
    g = U.oracle_grid(c)
    info = {}
    ref = orhs.rhs(c.Q, g, gas, opts, scheme, info=info)
    ctx, _ = U.gpu_context(c, gas, opts)
    out = U.gpu_rhs(ctx, c, scheme)
    U.compare(out, ref, g, U.RHS_RTOL, U.excused_mask(info, g), label='%s/%s/%s' % (name, scheme, grad))
    ctx.close()


@pytest.mark.parametrize('name', list(CASES))
@pytest.mark.parametrize('mask', [0, 0xFFF])
def test_mig4_line_kernels_parity_fp64(name, mask):
    """MIG4 gradients solved in LDS line tiles (mask 0xFFF; small problems use them in every
    direction) or by the PCR / lane-per-line kernels only (mask 0): both against the oracle."""
    print('mig4 lines', name, mask, flush=True)
    c = CASES[name]()
    gas, opts = _gas(name), _opts('C4', 'global')
    g = U.oracle_grid(c)
    info = {}
    ref = orhs.rhs(c.Q, g, gas, opts, 'cgbr', info=info)
    ctx, _ = U.gpu_context(c, gas, opts)
    ctx.set_line_tiles(mask)
    out = U.gpu_rhs(ctx, c, 'cgbr')
    U.compare(out, ref, g, U.RHS_RTOL, U.excused_mask(info, g), label='mig4 %s mask %x' % (name, mask))
    ctx.close()


@pytest.mark.parametrize('scheme,grad', [('cgbr', 'E6'), ('cgbr', 'C4'), ('lad', 'E6'), ('hybrid', 'E6')])
def test_stage_parity_fp64(scheme, grad):
    """Each stage starts from the oracle's own stage input; the stage output must agree to
    1e-12 of the state's max norm."""
    torch = U.torch_mod()
    c = case_2d_walls()
    gas, opts = orhs.Gas(), _opts(grad, 'percell')
    g = U.oracle_grid(c)
    M = ogrid.node_metrics(g)
    dt = orhs.cfl_dt(c.Q, g, gas, 0.2, M)
    ctx, _ = U.gpu_context(c, gas, opts)
    Un = c.Q
    Us = c.Q
    for s in range(3):
        print('stage', s, scheme, grad, flush=True)
        info = {}
        ref = orhs.rk3_stage(Un, Us, dt, s, g, gas, opts, scheme, M, info=info)
        Und, Usd = U.dev(Un), U.dev(Us)
        ctx.rk3_stage(scheme, s, Und, Usd, dt)
        torch.cuda.synchronize()
        U.compare(Usd.cpu().numpy(), ref, g, U.STAGE_RTOL, U.excused_mask(info, g), label='stage %d' % s)
        Us = ref
    ctx.close()


def test_rk3_step_and_dt():
    torch = U.torch_mod()
    c = case_2d_curv()
    gas, opts = orhs.Gas(), _opts('E6', 'percell')
    g = U.oracle_grid(c)
    M = ogrid.node_metrics(g)
    ctx, _ = U.gpu_context(c, gas, opts)
    Qd = U.dev(c.Q)
    dtd = torch.zeros(1, dtype=torch.float64, device='cuda')
    ctx.compute_dt(Qd, dtd)
    dt_ref = orhs.cfl_dt(c.Q, g, gas, 0.2, M)
    assert abs(dtd.item() - dt_ref) <= 1e-14 * dt_ref
    td = torch.zeros(1, dtype=torch.float64, device='cuda')
    ctx.rk3_step('hybrid', Qd, 1.0, td)
    Qn, t1, dt1, bad = orhs.rk3_step(c.Q, 0.0, 1.0, g, gas, opts, 'hybrid', M)
    torch.cuda.synchronize()
    assert abs(td.item() - t1) <= 1e-14 * t1
    U.compare(Qd.cpu().numpy(), Qn, g, U.STAGE_RTOL, label='rk3 step')
    # clipping to t_end
    t_end = 0.25 * dt_ref
    td.zero_()
    Qd = U.dev(c.Q)
    ctx.rk3_step('cgbr', Qd, t_end, td)
    torch.cuda.synchronize()
    assert td.item() == pytest.approx(t_end, rel=1e-15)
    assert ctx.poll_status() == 0
    ctx.close()


@pytest.mark.parametrize('ndim', [2, 3])
def test_metrics_from_coords(ndim):
    n = (40, 22) if ndim == 2 else (18, 14, 11)
    c = cases.periodic_case(ndim, n, curvilinear=True, amp=0.08)
    cases.uniform_state(c)
    g = U.oracle_grid(c)
    ref = ogrid.node_metrics(g)
    _, met = U.gpu_context(c, orhs.Gas(), orhs.Opts())
    got = met.cpu().numpy()
    sl = (slice(None),) + g.band(-3, 3)
    assert np.allclose(got[sl], ref[sl], rtol=1e-13, atol=1e-15)


def test_forced_flags_and_flags_out():
    torch = U.torch_mod()
    c = case_2d_walls()
    gas, opts = orhs.Gas(), _opts('E6', 'percell')
    g = U.oracle_grid(c)
    flags = np.random.default_rng(5).random(g.shape) < 0.02
    ref = orhs.rhs(c.Q, g, gas, opts, 'hybrid', force_flags=flags)
    ctx, _ = U.gpu_context(c, gas, opts)
    Qd = U.dev(c.Q)
    dQ = torch.zeros_like(Qd)
    fout = torch.zeros(g.shape, dtype=torch.uint8, device='cuda')
    ctx.hybrid_rhs(Qd, dQ, U.dev(flags.astype(np.uint8)), fout)
    torch.cuda.synchronize()
    U.compare(dQ.cpu().numpy(), ref, g, U.RHS_RTOL, label='forced flags')
    assert np.array_equal(fout.cpu().numpy().astype(bool), flags)
    # criterion flags reported back
    info = {}
    orhs.rhs(c.Q, g, gas, opts, 'hybrid', info=info)
    ctx.hybrid_rhs(Qd, dQ, None, fout)
    torch.cuda.synchronize()
    assert np.array_equal(fout.cpu().numpy().astype(bool), info['flags'])
    ctx.close()


def test_nonphysical_state_is_reported():
    """A negative density planted in the input (host side) is counted after the stage."""
    torch = U.torch_mod()
    c = case_2d_walls()
    Q = c.Q.copy()
    Q[0, 0, 20, 30] = -0.5
    ctx, _ = U.gpu_context(c, orhs.Gas(), _opts('E6', 'percell'))
    Qd = U.dev(Q)
    Us = Qd.clone()
    ctx.rk3_stage('cgbr', 0, Qd, Us, 1e-4)
    assert ctx.poll_status() > 0
    assert ctx.poll_status() == 0   # reset after the poll
    ctx.close()


@pytest.mark.parametrize('precision_case', ['2d_smooth', '3d_smooth'])
def test_mixed_precision_on_smooth_data(precision_case):
    """FP32 bulk / FP64 state: RHS within 1e-4 of the largest oracle value per variable on
    smooth data (FP32 rounding 6e-8 amplified by the flux-difference cancellation)."""
    if precision_case == '2d_smooth':
        c = cases.random_smooth_state(cases.periodic_case(2, (64, 40), curvilinear=True, amp=0.05), seed=21)
        gas = orhs.Gas()
    else:
        c = cases.random_smooth_state(cases.periodic_case(3, (20, 16, 12), curvilinear=True, amp=0.05), seed=22)
        gas = orhs.Gas(viscous=True, Re=200.0, Mref=0.5)
    g = U.oracle_grid(c)
    for scheme, grad in (('cgbr', 'E6'), ('cgbr', 'C4'), ('lad', 'E6'), ('hybrid', 'E6')):
        opts = _opts(grad, 'percell')
        opts.rho_thr = 1.0
        ref = orhs.rhs(c.Q, g, gas, opts, scheme)
        ctx, _ = U.gpu_context(c, gas, opts, precision='mixed')
        out = U.gpu_rhs(ctx, c, scheme)
        inner = (slice(None),) + g.interior()
        for q in range(5 if g.ndim == 3 else 5):
            scale = max(np.max(np.abs(ref[inner][q])), 1e-30)
            if q == 3 and g.ndim < 3:
                continue
            err = np.max(np.abs(out[inner][q] - ref[inner][q])) / scale
            assert err < 1e-4, (scheme, grad, q, err)
        ctx.close()


def test_batch_matches_single_problems():
    """Three problems of different sizes advanced together (one graph launch of two RK3
    steps) give the same bits as each advanced alone, and agree with the oracle."""
    torch = U.torch_mod()
    probs = cases.batch64(count=3, scale=16)
    gas = orhs.Gas()
    ctxs, Qs, ts, singles = [], [], [], []
    for c in probs:
        opts = orhs.Opts(rho_thr=c.extra['rho_thr'], p_thr=c.extra['p_thr'])
        ctx, _ = U.gpu_context(c, gas, opts)
        ctxs.append(ctx)
        Qs.append(U.dev(c.Q))
        ts.append(torch.zeros(1, dtype=torch.float64, device='cuda'))
        # single-problem reference run
        ctx1, _ = U.gpu_context(c, gas, opts)
        Q1 = U.dev(c.Q)
        t1 = torch.zeros(1, dtype=torch.float64, device='cuda')
        for _ in range(2):
            ctx1.rk3_step('hybrid', Q1, 10.0, t1)
        torch.cuda.synchronize()
        singles.append(Q1.cpu().numpy())
        ctx1.close()
    from paper_2511_18042_amd import lgbr
    b = lgbr.Batch(ctxs, Qs, ts, [10.0] * 3, 2, 'hybrid')
    b.run()
    torch.cuda.synchronize()
    for c, Qd, ref1 in zip(probs, Qs, singles):
        got = Qd.cpu().numpy()
        assert np.array_equal(got, ref1)
        g = U.oracle_grid(c)
        opts = orhs.Opts(rho_thr=c.extra['rho_thr'], p_thr=c.extra['p_thr'])
        Q, t = c.Q, 0.0
        for _ in range(2):
            Q, t, _, _ = orhs.rk3_step(Q, t, 10.0, g, gas, opts, 'hybrid')
        U.compare(got, Q, g, U.STAGE_RTOL * 10, label='batch vs oracle')
    b.close()
    for ctx in ctxs:
        ctx.close()


@pytest.mark.parametrize('scheme', ['hybrid', 'cgbr'])
def test_full_size_triple_point_rhs(scheme):
    """The 1792 x 768 triple-point state at t = 0, element by element (oracle ~20 s)."""
    c = cases.triple_point()
    gas = orhs.Gas()
    opts = orhs.Opts(rho_thr=0.5)          # flags the rho = 0.125 region: both schemes active
    g = U.oracle_grid(c)
    info = {}
    ref = orhs.rhs(c.Q, g, gas, opts, scheme, info=info)
    ctx, _ = U.gpu_context(c, gas, opts)
    out = U.gpu_rhs(ctx, c, scheme)
    U.compare(out, ref, g, U.RHS_RTOL, U.excused_mask(info, g), label='triple point ' + scheme)
    ctx.close()


def _ramp_case(nx=40, ny=32, nz=16):
    c = cases.ramp3d(nx, ny, nz)
    e = c.extra
    gas = orhs.Gas(gamma=1.4, Re=e['Re'], Pr=e['Pr'], Mref=e['Mref'], suth=e['suth'], viscous=True)
    return c, gas


@pytest.mark.parametrize('scheme,grad', [('cgbr', 'C4'), ('cgbr', 'E6'), ('lad', 'E6'), ('hybrid', 'C4')])
def test_ramp_crop_rhs_parity_fp64(scheme, grad):
    """The compression-ramp workload (same generator, 40x32x16 crop): curvilinear metrics from
    the GPU, fixed inflow ghosts, no-slip wall, periodic span, Sutherland viscosity; the
    hybrid runs with 10 % random troubled cells so that both schemes and their seams are hit."""
    print('ramp', scheme, grad, flush=True)
    c, gas = _ramp_case()
    g = U.oracle_grid(c)
    opts = orhs.Opts(grad=grad, p_thr=c.extra['p_thr'])
    flags = (np.random.default_rng(9).random(g.shape) < 0.1) if scheme == 'hybrid' else None
    info = {}
    ref = orhs.rhs(c.Q, g, gas, opts, scheme, info=info, force_flags=flags)
    ctx, _ = U.gpu_context(c, gas, opts)
    out = U.gpu_rhs(ctx, c, scheme, flags=flags)
    U.compare(out, ref, g, U.RHS_RTOL, U.excused_mask(info, g), label='ramp %s %s' % (scheme, grad))
    ctx.close()


def test_ramp_crop_rk3_step_and_mixed_error():
    """One full hybrid MIG4 RK3 step on the ramp crop (FP64 gate), and the mixed path's
    state error after the step relative to the FP64 oracle (bound 1e-4 of each variable's
    max norm: FP32 rounding amplified by the near-wall viscous cancellation)."""
    torch = U.torch_mod()
    c, gas = _ramp_case()
    g = U.oracle_grid(c)
    opts = orhs.Opts(grad='C4', p_thr=c.extra['p_thr'])
    Qn, t1, dt1, bad = orhs.rk3_step(c.Q, 0.0, 1.0, g, gas, opts, 'hybrid')
    assert bad == 0
    for precision, tol in (('fp64', U.STAGE_RTOL), ('mixed', 1e-4)):
        ctx, _ = U.gpu_context(c, gas, opts, precision=precision)
        Qd = U.dev(c.Q)
        td = torch.zeros(1, dtype=torch.float64, device='cuda')
        ctx.rk3_step('hybrid', Qd, 1.0, td)
        torch.cuda.synchronize()
        assert abs(td.item() - t1) <= 1e-13 * t1
        U.compare(Qd.cpu().numpy(), Qn, g, tol, label='ramp rk3 ' + precision)
        assert ctx.poll_status() == 0
        ctx.close()


def test_launch_tuning_leaves_results_bitwise_unchanged(tmp_path, monkeypatch):
    """Segment length of the strided sweeps, the persistent PCR grid size, the z-marching
    tile shape, its chunk length and the lines per LDS line tile only change the launch
    shape: the RHS is bitwise identical for every setting, invalid shapes are refused, and
    the autotuner picks one of its candidates and caches it."""
    torch = U.torch_mod()
    from paper_2511_18042_amd import autotune
    c, gas = _ramp_case()
    g = U.oracle_grid(c)
    opts = orhs.Opts(grad='C4', p_thr=c.extra['p_thr'])
    flags = np.random.default_rng(10).random(g.shape) < 0.1
    ctx, _ = U.gpu_context(c, gas, opts)
    outs = []
    for seg, pcr, zc, zw, lb in ((0, 0, 0, 0, 0), (2, 256, 1, 32, 1), (7, 1000, 5, 128, 3),
                                 (64, 65536, 1024, 64, 16), (4, 0, 3, 32, 2)):
        print('tuning', seg, pcr, zc, zw, lb, flush=True)
        ctx.set_tuning(seg, pcr, zc)
        ctx.set_tile_shape(zw, lb)
        s, p, z = ctx.get_tuning()
        assert (seg == 0 or s == seg) and p == (pcr or 16384) and (zc == 0 or z == zc)
        assert ctx.get_tile_shape() == (zw or 64, lb)
        for scheme, fl in (('hybrid', flags), ('lad', None)):
            outs.append(U.gpu_rhs(ctx, c, scheme, flags=fl))
    for i, o in enumerate(outs[2:]):
        assert np.array_equal(o, outs[i % 2])
    for bad in ((48, 0), (64, 17), (64, -1)):
        with pytest.raises(lgbr.LgError):
            ctx.set_tile_shape(*bad)
    monkeypatch.setenv('LGBR_TUNE_CACHE', str(tmp_path / 'tune.json'))
    Q0 = U.dev(c.Q)
    best, timings = autotune.tune(ctx, Q0, 'hybrid', steps=1)
    assert best['zc'] in autotune.CANDIDATE_ZC and best['seg'] in autotune.CANDIDATE_SEG
    assert best['pcr_blocks'] in autotune.CANDIDATE_PCR and best['zm_width'] in autotune.CANDIDATE_ZM_WIDTH
    assert best['line_batch'] in autotune.CANDIDATE_LINE_BATCH
    assert len(timings) >= len(autotune.CANDIDATE_ZC)
    assert autotune.tune(ctx, Q0, 'hybrid')[0] == best          # served from the cache
    ctx.close()
    torch.cuda.synchronize()


def test_planar_metric_storage_matches_full_storage():
    """The ramp grid is a 2D section extruded spanwise: the library keeps one plane of
    metrics and grid factors for it.  A copy whose coordinates are perturbed along zeta
    (1e-6 of the spacing, so the metrics vary with k) is stored in full.  Both right-hand
    sides meet the oracle's on their own grids, the planar context holds less workspace,
    and the two agree where the grids agree to 1e-6."""
    torch = U.torch_mod()
    c, gas = _ramp_case()
    opts = orhs.Opts(grad='C4', p_thr=c.extra['p_thr'], hybrid_mode='global')
    c2 = cases.ramp3d(40, 32, 16)
    kk = np.arange(c2.coords.shape[1])[:, None, None]
    c2.coords = c2.coords.copy()
    c2.coords[0] += 1e-6 * c2.h[0] * np.sin(0.7 * kk) * np.ones_like(c2.coords[0])
    outs, sizes = [], []
    for cc in (c, c2):
        g = U.oracle_grid(cc)
        ref = orhs.rhs(cc.Q, g, gas, opts, 'hybrid')
        ctx, _ = U.gpu_context(cc, gas, opts)
        sizes.append(ctx.workspace_bytes())
        assert ctx.metrics_planar() == (cc is c)
        out = U.gpu_rhs(ctx, cc, 'hybrid')
        U.compare(out, ref, g, U.RHS_RTOL, label='planar' if cc is c else 'full')
        outs.append(out)
        ctx.close()
    assert sizes[0] < sizes[1]
    g = U.oracle_grid(c)
    U.compare(outs[1], outs[0], g, 1e-4, label='planar vs perturbed')


@pytest.mark.parametrize('scheme,grad', [('hybrid', 'C4'), ('cgbr', 'C4'), ('lad', 'C4')])
def test_ramp_large_crop_rhs_parity(scheme, grad):
    """The ramp generator on a 256x192x64 crop: large enough that the library picks, without
    any forcing switch, the paths of the full 1024x384x128 grid -- one lane per line for the
    compact solves along zeta (more than 32768 lines), LDS line tiles along xi and eta, the
    z-chunked stencil kernels -- with the hybrid at 10 % random troubled cells (compacted
    per-cell path), MIG4 C-GBR and LAD-E4.  FP64 at the RHS gate; the mixed path's error is
    printed (RHS-REPORT) and bounded by 1e-4 of each variable's max norm."""
    print('ramp large crop', scheme, grad, flush=True)
    c, gas = _ramp_case(256, 192, 64)
    g = U.oracle_grid(c)
    opts = orhs.Opts(grad=grad, p_thr=c.extra['p_thr'], hybrid_mode='percell')
    flags = (np.random.default_rng(11).random(g.shape) < 0.1) if scheme == 'hybrid' else None
    info = {}
    ref = orhs.rhs(c.Q, g, gas, opts, scheme, info=info, force_flags=flags)
    inner = (slice(None),) + g.interior()
    for precision in ('fp64', 'mixed'):
        ctx, _ = U.gpu_context(c, gas, opts, precision=precision)
        out = U.gpu_rhs(ctx, c, scheme, flags=flags)
        ctx.close()
        if precision == 'fp64':
            U.compare(out, ref, g, U.RHS_RTOL, U.excused_mask(info, g), label='ramp 256 %s %s' % (scheme, grad))
        else:
            rel = [float(np.max(np.abs(out[q][inner[1:]] - ref[q][inner[1:]])) / max(np.max(np.abs(ref[q][inner[1:]])),
                                                                                 1e-300)) for q in range(5)]
            print('RHS-REPORT ramp 256x192x64 %s mixed max rel err per variable %s' % (scheme, rel), flush=True)
            assert max(rel) <= 1e-4


def test_launch_timing_per_class_and_per_launch():
    """lg_prof_stop_launches: the per-launch durations add up to the per-class sums, every
    class of an LAD-E4 RK3 step appears, and timing stopped twice is refused."""
    torch = U.torch_mod()
    c = case_2d_walls()
    gas, opts = orhs.Gas(), _opts('E6', 'global')
    ctx, _ = U.gpu_context(c, gas, opts)
    Qd = U.dev(c.Q)
    td = torch.zeros(1, dtype=torch.float64, device='cuda')
    ctx.prof_start(-1, 1000)
    ctx.rk3_step('lad', Qd, 10.0, td)
    per, each = ctx.prof_stop_launches()
    assert {'prim', 'lad_raw', 'lad_flux', 'lad_sweep', 'filter', 'dt'} <= set(per)
    for k, (ms, n) in per.items():
        d = [x for kk, x in each if kk == k]
        assert len(d) == n and abs(sum(d) - ms) <= 1e-3 * max(ms, 1e-6) + 1e-6
    with pytest.raises(lgbr.LgError):
        ctx.prof_stop_launches()
    ctx.close()
