#!/usr/bin/env python3
"""Throughput of the hybrid LAD-GBR right-hand side on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload all|ramp3d|triple_point|batch64] [--no-cpu-baseline]
                    [--variants all|none] [--copy-probe-mib M]

A step is one SSP-RK3 step of the whole hot path (ghost images, primitives, troubled
flags, gradients, sensor, LAD coefficients, interface fluxes, stage combination and the
CFL reduction) on synthetic inputs resident in HBM before timing starts.

Headline workload (``value``): the M2.9 24-degree compression-ramp stand-in, 1024 x 384 x
128 cells on a curvilinear grid (tanh wall clustering, spanwise periodic), viscous
(Sutherland, Re 2e4, Pr 0.72), per-cell hybrid of LAD-E4 and C-GBR with compact MIG4
gradients, troubled where p < 0.5 p_inf, the paper's global switch (any troubled node
puts the whole field on C-GBR), FP32 bulk arithmetic with FP64 state; K steps after W
warm-up steps.  Also measured on the same grid: FP64, the per-cell switch, the C-GBR and
LAD forms, and the per-cell hybrid right-hand side with forced troubled-tile fractions of
0, 5, 17.6, 50 and 100 %.  Further workloads: the 2D triple point (1792 x 768) in a window at t = 0 and one
from a t = 3 state (reached on the GPU first), and 64 independent four-quadrant Riemann
problems (128^2 .. 1024^2) advanced 100 hybrid RK3 steps per graph launch, FP32 and FP64,
default and autotuned launch shapes.

Each workload reports its dominant kernel's roofline: the kernel class's algorithmic bytes
per launch over its average launch time from HIP events recorded on the library's stream
around that class in a timed pass.  The FP64 CPU oracle is timed on a bounded sample on
this host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TILE = 8                      # edge of the tiles of the forced-flag sweep
FORCED_FRACTIONS = (0.0, 0.05, 0.176, 0.5, 1.0)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=100)
    ap.add_argument('--warmup', type=int, default=10)
    ap.add_argument('--workload', default='all', choices=['all', 'ramp3d', 'triple_point', 'batch64'])
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--variants', default='all', choices=['all', 'none'])
    ap.add_argument('--only-variant', default=None,
                    help='with --workload ramp3d: of the config-4 variants run only this one (profiling)')
    ap.add_argument('--copy-probe-mib', type=int, default=0,
                    help='run one plain device copy of this many MiB first (calibrates HBM counters)')
    return ap.parse_args()


def log(msg):
    print('[bench] ' + msg, file=sys.stderr, flush=True)


def algorithmic_bytes(kclass, nodes, rs, ndim, gbr_frac, viscous, curv, planar=False):
    """Minimum bytes one launch of a kernel class moves (every input read once, every
    output written once) for ``nodes`` interior nodes; rs = bytes of the bulk real type,
    curv: node metrics (9 components + J) are fields rather than constants; planar: they
    (and the LAD grid factors) are stored for one plane only, so they add nothing per node."""
    vis = 5 * rs if viscous else 0
    per_node_geom = curv and not planar
    met = 10 * rs if per_node_geom else 0
    if kclass == 'sweep_x':
        per = (1 - gbr_frac) * 5 * rs + gbr_frac * (11 * rs + vis) + 1 + 40
    elif kclass in ('sweep_y', 'sweep_z'):
        per = (1 - gbr_frac) * 5 * rs + gbr_frac * (11 * rs + vis) + 1 + 80
    elif kclass == 'lad_node':
        per = 5 * rs + met + 2 * rs                          # W, metrics -> |S|, theta
    elif kclass == 'lad_raw':
        per = 5 * rs + 2 * rs + met + (3 * ndim * rs if per_node_geom else 0) + 3 * rs   # + Delta x_l -> raw
    elif kclass == 'gauss':
        per = 6 * rs                                         # one launch: 3 fields in, 3 out
    elif kclass == 'lad_flux':
        per = 5 * rs + 3 * rs + met + 5 * ndim * rs          # W, coefficients, metrics -> F_l
    elif kclass == 'lad_sweep':
        per = 5 * ndim * rs + (8 if per_node_geom else 0) + 120   # F_l, J, U^n, U^s -> stage result
    elif kclass == 'grad_e6':
        per = 10 * rs
    elif kclass == 'grad_c4':
        per = 40 + 5 * rs
    elif kclass == 'sensor':
        per = (2 + 3 * ndim) * rs
    elif kclass == 'visc':
        per = 5 * rs + 5 * ndim * rs + 5 * rs * ndim
    elif kclass == 'prim':
        per = 40 + 5 * rs + 1
    elif kclass == 'combine':
        per = 160
    elif kclass == 'dt':
        per = 40 + (72 if per_node_geom else 0)
    else:
        per = 0.0
    return per * nodes


def interface_fraction(flags, mode='percell'):
    """Share of interior nodes whose interfaces take C-GBR: per cell, the flags dilated by
    the hybrid radius (3 nodes); with the global switch, all or nothing."""
    import numpy as np
    from scipy.ndimage import maximum_filter
    inner = tuple(slice(5, -5) if s > 1 else slice(None) for s in flags.shape)
    if mode == 'global':
        return 1.0 if flags[inner].any() else 0.0
    ft = maximum_filter(flags.astype(np.uint8), size=7, mode='constant') > 0
    return float(ft[inner].mean())


def mcell(cells, ms):
    return round(cells / (ms * 1e-3) / 1e6, 2)


class Runner:
    """Timing helpers (HIP events on torch's current stream, which the contexts use)."""

    def __init__(self, K, W):
        self.K, self.W = K, W

    def steps(self, ctx, scheme, Q0, K=None, W=None, prof_class=None, t_end=1e30):
        import torch
        K = self.K if K is None else K
        W = self.W if W is None else W
        Q = Q0.clone()
        t = torch.zeros(1, dtype=torch.float64, device='cuda')
        for _ in range(W):
            ctx.rk3_step(scheme, Q, t_end, t)
        torch.cuda.synchronize()
        if prof_class is not None:
            ctx.prof_start(prof_class, 400 * K + 400)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K):
            ctx.rk3_step(scheme, Q, t_end, t)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        kern = ctx.prof_stop() if prof_class is not None else None
        bad = ctx.poll_status()
        return ms, kern, bad, Q, float(t.item())

    def roofline(self, ctx, scheme, Q0, cells, ndim, gbr_frac, viscous, curv, K=20, traffic_file=None):
        """Per-class breakdown, then the dominant class timed alone."""
        planar = ctx.metrics_planar()
        _, breakdown, _, _, _ = self.steps(ctx, scheme, Q0, K=K, W=2, prof_class=-1)
        dominant = max(breakdown, key=lambda k: breakdown[k][0])
        _, kern, _, _, _ = self.steps(ctx, scheme, Q0, K=K, W=2, prof_class=dominant)
        dom_ms, dom_n = kern[dominant]
        dom_avg = dom_ms / max(dom_n, 1)
        algo = algorithmic_bytes(dominant, cells, 4, ndim, gbr_frac, viscous, curv, planar)
        achieved = algo / (dom_avg * 1e-3) / 1e9
        roof = {'bound': 'hbm', 'kernel': dominant, 'achieved': round(achieved, 1), 'peak': HBM_PEAK_GBS,
                'unit': 'GB/s', 'frac': round(achieved / HBM_PEAK_GBS, 4), 'avg_launch_ms': round(dom_avg, 5),
                'launches': dom_n, 'algorithmic_bytes_per_launch': int(algo), 'traffic': None}
        if traffic_file:
            tr, why = profiled_traffic(traffic_file, dominant)
            roof['traffic'] = tr
            roof['traffic_source'] = os.path.relpath(traffic_file, ROOT) + ('' if tr else ' (%s)' % why)
            if tr:
                roof['traffic_over_algorithmic'] = round(tr / algo, 3)
        brk = {k: round(v[0] / K, 4) for k, v in sorted(breakdown.items(), key=lambda kv: -kv[1][0])}
        return roof, brk


def profiled_traffic(path, kclass):
    """HBM bytes per launch of kernel class kclass from a committed rocprofv3 counter summary
    (its TRAFFIC line: FETCH_SIZE and WRITE_SIZE in KiB per dispatch and their scales from a
    copy of known size), or None with the reason: no such line, or the kernel sources no
    longer hash to what was profiled."""
    import hashlib
    if not os.path.exists(path):
        return None, 'no profile'
    for line in open(path):
        f = line.split()
        if len(f) < 3 or f[0] != 'TRAFFIC' or f[1] != kclass:
            continue
        kv = dict(x.split('=', 1) for x in f[2:])
        h = hashlib.sha256()
        for src in kv['sources'].split(','):
            h.update(open(os.path.join(ROOT, src), 'rb').read())
        if h.hexdigest() != kv['sha256']:
            return None, 'kernel sources changed since the counters were taken'
        kib = float(kv['fetch_kib']) * float(kv['fetch_scale']) + float(kv['write_kib']) * float(kv['write_scale'])
        return int(kib * 1024), ''
    return None, 'no counters for this kernel'


def profiled_step(path):
    """Whole-step HBM bytes and VALU-busy % of the workload from a committed counter summary
    (its STEP line: every kernel of a step, FETCH_SIZE and WRITE_SIZE scaled by the copy of
    known size), or (None, reason) once any library source no longer hashes to what was
    profiled."""
    import hashlib
    if not os.path.exists(path):
        return None, 'no profile'
    for line in open(path):
        f = line.split()
        if len(f) < 2 or f[0] != 'STEP':
            continue
        kv = dict(x.split('=', 1) for x in f[1:])
        h = hashlib.sha256()
        for src in kv['sources'].split(','):
            h.update(open(os.path.join(ROOT, src), 'rb').read())
        if h.hexdigest() != kv['sha256']:
            return None, 'library sources changed since the counters were taken'
        return {'bytes_per_step': int(float(kv['bytes_per_step'])), 'valu_busy_pct': float(kv['valu_busy_pct'])}, ''
    return None, 'no STEP line'


def flags_of(ctx, Q):
    import torch
    fl = torch.zeros(tuple(Q.shape[1:]), dtype=torch.uint8, device='cuda')
    dQ = torch.empty_like(Q)
    ctx.hybrid_rhs(Q, dQ, None, fl)
    torch.cuda.synchronize()
    return fl.cpu().numpy().astype(bool)


# ------------------------------------------------------------------ M2.9 ramp (headline)
def ramp3d(args, variants, cpu):
    import torch
    from paper_2511_18042_amd import cases, lgbr
    R = Runner(args.steps, args.warmup)
    log('ramp3d: generating the 1024x384x128 state')
    c = cases.ramp3d()
    e = c.extra
    gas = lgbr.make_gas(gamma=1.4, Re=e['Re'], Pr=e['Pr'], Mref=e['Mref'], suth=e['suth'], viscous=True)
    coords = torch.from_numpy(c.coords).cuda()
    grid = lgbr.make_grid(3, c.n, c.bc, c.h, curvilinear=True)
    metrics = torch.zeros((10,) + tuple(c.shape), dtype=torch.float64, device='cuda')
    lgbr.metrics_from_coords(grid, coords, metrics)
    Q0 = torch.from_numpy(c.Q).cuda()
    cells = c.cells
    c.Q = c.coords = None

    def context(precision, grad='C4', mode='global', lad='E4'):
        return lgbr.Context(grid, gas, lgbr.make_opts(precision=precision, cfl=0.2, grad=grad, hybrid_mode=mode,
                                                      p_thr=e['p_thr'], lad=lad), metrics, coords)

    desc = ('M2.9 24-deg ramp stand-in 1024x384x128 curvilinear, viscous, hybrid LAD-E4/MIG4 (global switch), '
            'p_thr 0.5 p_inf, CFL 0.2')
    res = {'workload': desc, 'cells': cells}
    head = context('mixed')
    log('ramp3d: headline %d steps' % args.steps)
    ms, _, bad, Q, t_end = R.steps(head, 'hybrid', Q0)
    gbr_frac = interface_fraction(flags_of(head, Q), 'global')
    del Q
    roof, brk = R.roofline(head, 'hybrid', Q0, cells, 3, gbr_frac, True, True,
                           traffic_file=os.path.join(ROOT, 'profiles', 'ramp3d_hybrid_mig4_mixed_hbm_traffic.txt'))
    prof = os.path.join(ROOT, 'profiles', 'ramp3d_hybrid_mig4_mixed_hbm_traffic.txt')
    st, why = profiled_step(prof)
    if st:   # whole-step figure: every kernel's HBM bytes over the measured step time
        gbs = st['bytes_per_step'] / (ms * 1e-3) / 1e9
        res['hbm_step'] = {'bytes_per_step': st['bytes_per_step'], 'achieved': round(gbs, 1), 'unit': 'GB/s',
                           'frac_of_peak': round(gbs / HBM_PEAK_GBS, 4), 'valu_busy_pct': st['valu_busy_pct'],
                           'source': os.path.relpath(prof, ROOT)}
    else:
        res['hbm_step'] = {'source': os.path.relpath(prof, ROOT) + ' (%s)' % why}
    res.update({'value': mcell(cells, ms), 'ms_per_step': round(ms, 4), 'nonphysical_nodes': bad,
                'sim_time_end': round(t_end, 6), 'troubled_interface_fraction': round(gbr_frac, 5),
                'roofline': roof, 'kernel_breakdown_ms_per_step': brk})
    head.close()
    if variants and not args.only_variant:
        log('ramp3d: forced-flag sweep')
        pc = context('mixed', mode='percell')
        res['forced_flag_sweep'] = forced_sweep(pc, Q0, tuple(c.shape))
        pc.close()
    torch.cuda.empty_cache()
    if variants:
        var = {}
        for vname, prec, scheme, grad, mode, *vv in (
                ('hybrid_fp64', 'fp64', 'hybrid', 'C4', 'global'),
                ('hybrid_percell_mixed', 'mixed', 'hybrid', 'C4', 'percell'),
                ('hybrid_percell_fp64', 'fp64', 'hybrid', 'C4', 'percell'),
                ('cgbr_mig4_fp64', 'fp64', 'cgbr', 'C4', 'global'),
                ('cgbr_mig4_mixed', 'mixed', 'cgbr', 'C4', 'global'),
                ('cgbr_meg6_fp64', 'fp64', 'cgbr', 'E6', 'global'),
                ('cgbr_meg6_mixed', 'mixed', 'cgbr', 'E6', 'global'),
                ('lad_e4_fp64', 'fp64', 'lad', 'C4', 'global'),
                ('lad_e4_mixed', 'mixed', 'lad', 'C4', 'global'),
                ('lad_c6_fp64', 'fp64', 'lad', 'C4', 'global', 'C6'),
                ('lad_c6_mixed', 'mixed', 'lad', 'C4', 'global', 'C6')):
            if args.only_variant and vname != args.only_variant:
                continue
            log('ramp3d: variant ' + vname)
            ctx = context(prec, grad, mode, *vv)
            vms, _, vbad, _, _ = R.steps(ctx, scheme, Q0, K=min(args.steps, 20), W=3)
            var[vname] = {'ms_per_step': round(vms, 4), 'mcell_per_s': mcell(cells, vms), 'nonphysical_nodes': vbad}
            if vname.startswith('lad_c6'):
                _, kern, _, _, _ = R.steps(ctx, scheme, Q0, K=5, W=1, prof_class=-1)
                var[vname]['kernel_breakdown_ms_per_step'] = {
                    k: round(v[0] / 5, 4) for k, v in sorted(kern.items(), key=lambda kv: -kv[1][0])}
            ctx.close()
            torch.cuda.empty_cache()
        # the paper's per-stage speed-up study: LAD-C6 against MEG6 / MIG4 C-GBR (FP64 there)
        res['variants'] = var
        if args.only_variant:
            return res
        res['lad_c6_speedup'] = {
            p: {'over_meg6': round(var['cgbr_meg6_' + p]['ms_per_step'] / var['lad_c6_' + p]['ms_per_step'], 3),
                'over_mig4': round(var['cgbr_mig4_' + p]['ms_per_step'] / var['lad_c6_' + p]['ms_per_step'], 3),
                'lad_e4_over_meg6': round(var['cgbr_meg6_' + p]['ms_per_step'] / var['lad_e4_' + p]['ms_per_step'], 3),
                'lad_e4_over_mig4': round(var['cgbr_mig4_' + p]['ms_per_step'] / var['lad_e4_' + p]['ms_per_step'], 3)}
            for p in ('fp64', 'mixed')}
    if cpu:
        res['cpu_baseline'] = cpu_baseline_ramp()
    return res


def forced_sweep(ctx, Q0, shape):
    """Right-hand side time of the mixed hybrid with forced troubled tiles (8^3 nodes,
    seeded choice), beside the LAD and C-GBR right-hand sides of the same context."""
    import numpy as np
    import torch
    rng = np.random.default_rng(2511)
    nt = [max(1, s // TILE) for s in shape]
    ntiles = int(np.prod(nt))
    order = rng.permutation(ntiles)
    Q = Q0.clone()
    dQ = torch.empty_like(Q)

    def time_rhs(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {'tile': TILE, 'rhs_ms': {}}
    out['rhs_ms']['lad'] = round(time_rhs(lambda: ctx.lad_rhs(Q, dQ)), 4)
    out['rhs_ms']['cgbr'] = round(time_rhs(lambda: ctx.cgbr_rhs(Q, dQ)), 4)
    for f in FORCED_FRACTIONS:
        m = np.zeros(ntiles, bool)
        m[order[:int(round(f * ntiles))]] = True
        tiles = m.reshape(nt)
        flags = np.repeat(np.repeat(np.repeat(tiles, TILE, 0), TILE, 1), TILE, 2)
        full = np.zeros(shape, bool)
        full[:flags.shape[0], :flags.shape[1], :flags.shape[2]] = flags[:shape[0], :shape[1], :shape[2]]
        fl = torch.from_numpy(full.astype(np.uint8)).cuda()
        ms = time_rhs(lambda: ctx.hybrid_rhs(Q, dQ, fl, None))
        out['rhs_ms']['hybrid_%g%%' % (100 * f)] = {'ms': round(ms, 4),
                                                    'interface_fraction': round(interface_fraction(full), 4)}
        del fl
    return out


def cpu_baseline_ramp():
    """The FP64 oracle as it stands, one SSP-RK3 step on a 256x192x64 crop of the ramp
    generator, one host thread."""
    from oracle import grid as ogrid, rhs as orhs
    from paper_2511_18042_amd import cases
    c = cases.ramp3d(256, 192, 64)
    e = c.extra
    gas = orhs.Gas(gamma=1.4, Re=e['Re'], Pr=e['Pr'], Mref=e['Mref'], suth=e['suth'], viscous=True)
    opts = orhs.Opts(grad='C4', p_thr=e['p_thr'])
    g = ogrid.Grid(c.ndim, c.n, c.bc, c.h, c.coords)
    M = ogrid.node_metrics(g)
    log('ramp3d: oracle step on the 256x192x64 crop')
    t0 = time.perf_counter()
    orhs.rk3_step(c.Q, 0.0, 1e30, g, gas, opts, 'hybrid', M)
    s = time.perf_counter() - t0
    return {'value': round(c.cells / s / 1e6, 4), 'unit': 'Mcell-updates/s', 'cores': 1, 'kind': 'oracle',
            'sample': ('one SSP-RK3 step of the per-cell hybrid MIG4 RHS on a 256x192x64 crop from the same '
                       'generator (rate per cell-update, scales linearly with cells); %.1f s' % s)}


# ------------------------------------------------------------------ 2D triple point
def triple_point(args, variants, cpu):
    import torch
    from paper_2511_18042_amd import cases, lgbr
    R = Runner(args.steps, args.warmup)
    c = cases.triple_point()
    gas = lgbr.make_gas(gamma=1.4)
    grid = lgbr.make_grid(2, c.n, c.bc, c.h)
    cells = c.cells
    Q0 = torch.from_numpy(c.Q).cuda()

    def context(precision, grad='E6', mode='global', lad='E4'):
        return lgbr.Context(grid, gas, lgbr.make_opts(precision=precision, cfl=0.2, grad=grad, hybrid_mode=mode,
                                                      rho_thr=c.extra['rho_thr'], lad=lad))

    desc = 'triple point 1792x768, hybrid LAD-E4/MEG6 (global switch), rho_thr 0.0625, CFL 0.2'
    res = {'workload': desc, 'cells': cells}
    head = context('mixed')
    log('triple_point: t=0 window')
    ms, _, bad, Q, _ = R.steps(head, 'hybrid', Q0)
    frac0 = interface_fraction(flags_of(head, Q), 'global')
    del Q
    roof, brk = R.roofline(head, 'hybrid', Q0, cells, 2, frac0, False, False)
    res.update({'value': mcell(cells, ms), 'ms_per_step': round(ms, 4), 'nonphysical_nodes': bad,
                'troubled_interface_fraction': round(frac0, 5), 'roofline': roof,
                'kernel_breakdown_ms_per_step': brk})
    if variants:
        # the t = 3 state comes from FP64 MEG6 C-GBR, the form that stays positive to t = 5
        # on this grid (the hybrid's LAD-E4 phases, without the paper's implicit filter, and
        # the FP32 forms lose positivity earlier)
        log('triple_point: advancing to t=3 with FP64 MEG6 C-GBR')
        adv = context('fp64')
        Q3 = Q0.clone()
        t = torch.zeros(1, dtype=torch.float64, device='cuda')
        b = lgbr.Batch([adv], [Q3], [t], [3.0], 500, 'cgbr')
        t0 = time.perf_counter()
        while t.item() < 3.0 and time.perf_counter() - t0 < 120:
            b.run()
            torch.cuda.synchronize()
        b.close()
        w3 = {'t': round(float(t.item()), 6), 'advanced_with': 'cgbr_meg6_fp64',
              'nonphysical_nodes_to_t3': adv.poll_status()}
        adv.close()
        fl3 = flags_of(head, Q3)
        w3['troubled_interface_fraction'] = {'global': interface_fraction(fl3, 'global'),
                                             'percell': round(interface_fraction(fl3), 5)}
        for vname, prec, scheme, grad, mode, *vv in (
                ('hybrid_mixed', 'mixed', 'hybrid', 'E6', 'global'),
                ('hybrid_fp64', 'fp64', 'hybrid', 'E6', 'global'),
                ('hybrid_percell_mixed', 'mixed', 'hybrid', 'E6', 'percell'),
                ('cgbr_meg6_mixed', 'mixed', 'cgbr', 'E6', 'global'),
                ('cgbr_meg6_fp64', 'fp64', 'cgbr', 'E6', 'global'),
                ('cgbr_mig4_mixed', 'mixed', 'cgbr', 'C4', 'global'),
                ('lad_e4_mixed', 'mixed', 'lad', 'E6', 'global'),
                ('lad_c6_mixed', 'mixed', 'lad', 'E6', 'global', 'C6')):
            ctx = context(prec, grad, mode, *vv)
            vms, _, vbad, _, _ = R.steps(ctx, scheme, Q3, K=min(args.steps, 50), W=3)
            ctx.close()
            w3[vname] = {'ms_per_step': round(vms, 4), 'mcell_per_s': mcell(cells, vms), 'nonphysical_nodes': vbad}
        res['window_t3'] = w3
        var = {}
        for vname, prec, scheme, grad, mode, *vv in (
                ('hybrid_fp64', 'fp64', 'hybrid', 'E6', 'global'),
                ('hybrid_percell_mixed', 'mixed', 'hybrid', 'E6', 'percell'),
                ('hybrid_percell_fp64', 'fp64', 'hybrid', 'E6', 'percell'),
                ('cgbr_meg6_fp64', 'fp64', 'cgbr', 'E6', 'global'),
                ('cgbr_meg6_mixed', 'mixed', 'cgbr', 'E6', 'global'),
                ('cgbr_mig4_fp64', 'fp64', 'cgbr', 'C4', 'global'),
                ('cgbr_mig4_mixed', 'mixed', 'cgbr', 'C4', 'global'),
                ('lad_e4_fp64', 'fp64', 'lad', 'E6', 'global'),
                ('lad_e4_mixed', 'mixed', 'lad', 'E6', 'global'),
                ('lad_c6_fp64', 'fp64', 'lad', 'E6', 'global', 'C6'),
                ('lad_c6_mixed', 'mixed', 'lad', 'E6', 'global', 'C6')):
            ctx = context(prec, grad, mode, *vv)
            vms, _, vbad, _, _ = R.steps(ctx, scheme, Q0, K=min(args.steps, 50), W=3)
            ctx.close()
            var[vname] = {'ms_per_step': round(vms, 4), 'mcell_per_s': mcell(cells, vms), 'nonphysical_nodes': vbad}
        res['variants'] = var
    head.close()
    if cpu:
        res['cpu_baseline'] = cpu_baseline_triple()
    return res


def cpu_baseline_triple():
    """The oracle, six SSP-RK3 steps of the full triple point from t = 0, one host thread."""
    from oracle import grid as ogrid, rhs as orhs
    from paper_2511_18042_amd import cases
    c = cases.triple_point()
    gas = orhs.Gas()
    opts = orhs.Opts(rho_thr=c.extra['rho_thr'])
    g = ogrid.Grid(c.ndim, c.n, c.bc, c.h, c.coords)
    M = ogrid.node_metrics(g)
    log('triple_point: oracle steps')
    Q, t, n = c.Q, 0.0, 0
    t0 = time.perf_counter()
    while n < 6:
        Q, t, _, _ = orhs.rk3_step(Q, t, 1e30, g, gas, opts, 'hybrid', M)
        n += 1
    s = time.perf_counter() - t0
    return {'value': round(n * c.cells / s / 1e6, 4), 'unit': 'Mcell-updates/s', 'cores': 1, 'kind': 'oracle',
            'sample': '%d SSP-RK3 steps of the per-cell hybrid RHS on the full 1792x768 triple point from t=0; '
                      '%.1f s' % (n, s)}


# ------------------------------------------------------------------ 64 problems, one graph
def batch64(args, variants, cpu):
    import numpy as np
    import torch
    from paper_2511_18042_amd import autotune, cases, lgbr
    log('batch64: generating 64 problems')
    probs = cases.batch64()
    cells = int(sum(c.cells for c in probs))
    nsteps = 100
    res = {'workload': '64 four-quadrant Riemann problems, sizes from {128,256,512,1024}^2 (seed 18042), '
                       'hybrid LAD-E4/MEG6 (global switch per problem), %d RK3 steps per graph launch' % nsteps,
           'cells': cells, 'problems': len(probs), 'steps_per_launch': nsteps}
    Q0s = [torch.from_numpy(c.Q).cuda() for c in probs]
    big = int(np.argmax([c.cells for c in probs]))

    def contexts(precision, mode='global'):
        out = []
        for c in probs:
            grid = lgbr.make_grid(2, c.n, c.bc, c.h)
            out.append(lgbr.Context(grid, lgbr.make_gas(gamma=1.4),
                                    lgbr.make_opts(precision=precision, cfl=0.2, grad='E6', hybrid_mode=mode,
                                                   rho_thr=c.extra['rho_thr'], p_thr=c.extra['p_thr'])))
        return out

    def run(ctxs, scheme='hybrid'):
        Qs = [q.clone() for q in Q0s]
        ts = [torch.zeros(1, dtype=torch.float64, device='cuda') for _ in probs]
        b = lgbr.Batch(ctxs, Qs, ts, [1e30] * len(probs), nsteps, scheme)
        b.run()                                   # warm-up launch (the first nsteps steps)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        b.close()
        bad = sum(cx.poll_status() for cx in ctxs)
        return ms / nsteps, bad

    for precision in (('mixed', 'fp64') if variants else ('mixed',)):
        log('batch64: %s, default launch shapes' % precision)
        ctxs = contexts(precision)
        ms, bad = run(ctxs)
        entry = {'ms_per_step': round(ms, 4), 'mcell_per_s': mcell(cells, ms), 'nonphysical_nodes': bad}
        if variants:
            log('batch64: %s, autotuning on the largest problem' % precision)
            (zc, seg, pcr), _ = autotune.tune(ctxs[big], Q0s[big], 'hybrid', steps=3, use_cache=False)
            for cx in ctxs:
                cx.set_tuning(seg, pcr, zc)
            tms, tbad = run(ctxs)
            entry['autotuned'] = {'zc': zc, 'seg': seg, 'ms_per_step': round(tms, 4),
                                  'mcell_per_s': mcell(cells, tms), 'nonphysical_nodes': tbad}
        for cx in ctxs:
            cx.close()
        torch.cuda.empty_cache()
        res[precision] = entry
    if variants:
        for vname, prec, mode, scheme in (('percell_mixed', 'mixed', 'percell', 'hybrid'),
                                          ('cgbr_meg6_mixed', 'mixed', 'global', 'cgbr'),
                                          ('cgbr_meg6_fp64', 'fp64', 'global', 'cgbr')):
            log('batch64: ' + vname)
            ctxs = contexts(prec, mode)
            ms, bad = run(ctxs, scheme)
            res[vname] = {'ms_per_step': round(ms, 4), 'mcell_per_s': mcell(cells, ms), 'nonphysical_nodes': bad}
            for cx in ctxs:
                cx.close()
            torch.cuda.empty_cache()
    res['value'] = res['mixed']['mcell_per_s']
    res['ms_per_step'] = res['mixed']['ms_per_step']
    if cpu:
        res['cpu_baseline'] = cpu_baseline_batch(probs)
    return res


def cpu_baseline_batch(probs):
    """The oracle on a bounded sample of the 64 problems: whole problems in draw order until
    at least 6 M cells, one SSP-RK3 step each, one host thread."""
    from oracle import grid as ogrid, rhs as orhs
    gas = orhs.Gas()
    cells, n, s = 0, 0, 0.0
    log('batch64: oracle steps')
    for c in probs:
        if cells >= 6_000_000:
            break
        g = ogrid.Grid(c.ndim, c.n, c.bc, c.h, c.coords)
        M = ogrid.node_metrics(g)
        opts = orhs.Opts(rho_thr=c.extra['rho_thr'], p_thr=c.extra['p_thr'])
        t0 = time.perf_counter()
        orhs.rk3_step(c.Q, 0.0, 1e30, g, gas, opts, 'hybrid', M)
        s += time.perf_counter() - t0
        cells += c.cells
        n += 1
    return {'value': round(cells / s / 1e6, 4), 'unit': 'Mcell-updates/s', 'cores': 1, 'kind': 'oracle',
            'sample': 'one SSP-RK3 step of the first %d problems in draw order (%d cells); %.1f s' % (n, cells, s)}


WORKLOADS = {'ramp3d': ramp3d, 'triple_point': triple_point, 'batch64': batch64}


def main():
    args = parse()
    if args.gpus != 1:
        print('bench.py: this build measures one GPU only (one process, one MI355X); '
              '--gpus %d is not supported' % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        a = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device='cuda')
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
    names = list(WORKLOADS) if args.workload == 'all' else [args.workload]
    results = {}
    for nm in names:
        results[nm] = WORKLOADS[nm](args, args.variants == 'all', not args.no_cpu_baseline)
        torch.cuda.empty_cache()
    head = results[names[0]]
    out = {
        'metric': 'Mcell-updates/s per RK3 step (hybrid vs C-GBR, FP32 vs FP64) and % HBM peak',
        'value': head['value'],
        'unit': 'Mcell-updates/s',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': head['ms_per_step'],
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'f32 (f64 state, RK combination, compact solves and flux differences)',
        'data': 'synthetic: seeded generator states',
        'config': {'workload': head['workload'], 'cells': head['cells'], 'parallelism': 'single GPU'},
        'roofline': head.get('roofline'),
        'hbm_step': head.get('hbm_step'),
        'cpu_baseline': head.get('cpu_baseline'),
        'nonphysical_nodes': head.get('nonphysical_nodes'),
        'workloads': results,
    }
    print(json.dumps(out))


if __name__ == '__main__':
    main()
