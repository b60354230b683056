#!/usr/bin/env python3
"""Throughput of the hybrid LAD-GBR right-hand side on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ramp3d|triple_point|all]
                    [--no-cpu-baseline] [--variants all|none]

A step is one SSP-RK3 step of the whole hot path (ghost images, primitives, troubled
flags, gradients, sensor, LAD coefficients, interface sweeps, stage combination and the
CFL reduction) on synthetic inputs resident in HBM before timing starts.

Headline workload (``value``): the M2.9 24-degree compression-ramp stand-in, 1024 x 384 x
128 cells on a curvilinear grid (tanh wall clustering, spanwise periodic), viscous
(Sutherland, Re 2e4, Pr 0.72), per-cell hybrid of LAD-E4 and C-GBR with compact MIG4
gradients, troubled where p < 0.5 p_inf, FP32 bulk arithmetic with FP64 state.  Also
measured: FP64 and the C-GBR / LAD forms on the same grid, and the 2D triple point
(1792 x 768).  Each workload reports the dominant kernel's roofline: its algorithmic bytes
per launch over its average launch time from HIP events bracketing that kernel class in
the timed region.  The FP64 CPU oracle is timed on a bounded sample on this host.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--warmup', type=int, default=3)
    ap.add_argument('--workload', default='all', choices=['all', 'ramp3d', 'triple_point'])
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--variants', default='all', choices=['all', 'none'])
    ap.add_argument('--copy-probe-mib', type=int, default=0,
                    help='run one plain device copy of this many MiB first (calibrates HBM counters)')
    return ap.parse_args()


def algorithmic_bytes(kclass, nodes, rs, ndim, gbr_frac, viscous, curv):
    """Minimum bytes one launch of a kernel class moves (every input read once, every
    output written once) for ``nodes`` interior nodes; rs = bytes of the bulk real type,
    curv: node metrics (9 components + J) are fields rather than constants."""
    vis = 5 * rs if viscous else 0
    met = 10 * rs if curv else 0
    if kclass == 'sweep_x':
        per = (1 - gbr_frac) * 5 * rs + gbr_frac * (11 * rs + vis) + 1 + 40
    elif kclass in ('sweep_y', 'sweep_z'):
        per = (1 - gbr_frac) * 5 * rs + gbr_frac * (11 * rs + vis) + 1 + 80
    elif kclass == 'lad_node':
        per = 5 * rs + met + 2 * rs                          # W, metrics -> |S|, theta
    elif kclass == 'lad_raw':
        per = 5 * rs + 2 * rs + met + (3 * ndim * rs if curv else 0) + 3 * rs   # + Delta x_l -> raw
    elif kclass == 'gauss':
        per = 6 * rs                                         # one launch: 3 fields in, 3 out
    elif kclass == 'lad_flux':
        per = 5 * rs + 3 * rs + met + 5 * ndim * rs          # W, coefficients, metrics -> F_l
    elif kclass == 'lad_sweep':
        per = 5 * ndim * rs + (8 if curv else 0) + 120       # F_l, J, U^n, U^s -> stage result
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
    else:
        per = 0.0
    return per * nodes


def setup_workload(name):
    from paper_2511_18042_amd import cases, lgbr
    import torch
    if name == 'triple_point':
        c = cases.triple_point()
        gas = lgbr.make_gas(gamma=1.4)
        okw = dict(grad='E6', rho_thr=0.5 * 0.125)
        coords = metrics = None
        desc = 'triple point 1792x768, hybrid LAD-E4/MEG6 per-cell, rho_thr 0.0625, CFL 0.2'
        grad_label = 'meg6'
    else:
        c = cases.ramp3d()
        e = c.extra
        gas = lgbr.make_gas(gamma=1.4, Re=e['Re'], Pr=e['Pr'], Mref=e['Mref'], suth=e['suth'], viscous=True)
        okw = dict(grad='C4', p_thr=e['p_thr'])
        coords = torch.from_numpy(c.coords).cuda()
        g = lgbr.make_grid(3, c.n, c.bc, c.h, curvilinear=True)
        metrics = torch.zeros((10,) + tuple(c.shape), dtype=torch.float64, device='cuda')
        lgbr.metrics_from_coords(g, coords, metrics)
        c.coords = None   # release the host copy
        desc = ('M2.9 24-deg ramp stand-in 1024x384x128 curvilinear, viscous, hybrid LAD-E4/MIG4 per-cell, '
                'p_thr 0.5 p_inf, CFL 0.2')
        grad_label = 'mig4'
    Q0 = torch.from_numpy(c.Q).cuda()
    c.Q = None
    return c, gas, okw, coords, metrics, Q0, desc, grad_label


def run_workload(name, K, W, variants, cpu):
    import numpy as np
    import torch
    from paper_2511_18042_amd import lgbr

    c, gas, okw, coords, metrics, Q0, desc, grad_label = setup_workload(name)
    cells = c.cells
    curv = metrics is not None
    grid = lgbr.make_grid(c.ndim, c.n, c.bc, c.h, curvilinear=curv)
    viscous = bool(gas.viscous)

    def context(precision, grad=None, mode='percell'):
        kw = dict(okw)
        if grad is not None:
            kw['grad'] = grad
        return lgbr.Context(grid, gas, lgbr.make_opts(precision=precision, cfl=0.2, hybrid_mode=mode, **kw),
                            metrics, coords)

    def timed(ctx, scheme, prof_class=None, want_flags=False):
        Q = Q0.clone()
        t = torch.zeros(1, dtype=torch.float64, device='cuda')
        for _ in range(W):
            ctx.rk3_step(scheme, Q, 1e30, t)
        torch.cuda.synchronize()
        if prof_class is not None:
            ctx.prof_start(prof_class, 400 * K + 400)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K):
            ctx.rk3_step(scheme, Q, 1e30, t)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        kern = ctx.prof_stop() if prof_class is not None else None
        bad = ctx.poll_status()
        flags = None
        if want_flags:
            fl = torch.zeros(tuple(c.shape), dtype=torch.uint8, device='cuda')
            dQ = torch.empty_like(Q)
            ctx.hybrid_rhs(Q, dQ, None, fl)
            torch.cuda.synchronize()
            flags = fl.cpu().numpy().astype(bool)
            del dQ
        del Q
        return ms, kern, bad, float(t.item()), flags

    res = {'workload': desc, 'cells': cells}
    head = context('mixed')
    _, breakdown, _, _, _ = timed(head, 'hybrid', prof_class=-1)
    dominant = max(breakdown, key=lambda k: breakdown[k][0])
    ms, kern, bad, t_end, flags = timed(head, 'hybrid', prof_class=dominant, want_flags=True)
    head.close()
    from scipy.ndimage import maximum_filter
    ft = maximum_filter(flags.astype(np.uint8), size=7, mode='constant') > 0
    inner = tuple(slice(5, -5) if s > 1 else slice(None) for s in flags.shape)
    gbr_frac = float(ft[inner].mean())
    dom_ms, dom_n = kern[dominant]
    dom_avg = dom_ms / max(dom_n, 1)
    algo = algorithmic_bytes(dominant, cells, 4, c.ndim, gbr_frac, viscous, curv)
    achieved = algo / (dom_avg * 1e-3) / 1e9
    res.update({
        'value': round(cells / (ms * 1e-3) / 1e6, 2), 'ms_per_step': round(ms, 4), 'nonphysical_nodes': bad,
        'sim_time_end': round(t_end, 6), 'troubled_interface_fraction': round(gbr_frac, 5),
        'roofline': {'bound': 'hbm', 'kernel': dominant, 'achieved': round(achieved, 1), 'peak': HBM_PEAK_GBS,
                     'unit': 'GB/s', 'frac': round(achieved / HBM_PEAK_GBS, 4), 'avg_launch_ms': round(dom_avg, 5),
                     'launches': dom_n, 'algorithmic_bytes_per_launch': int(algo), 'traffic': None},
        'kernel_breakdown_ms_per_step': {k: round(v[0] / K, 4) for k, v in
                                         sorted(breakdown.items(), key=lambda kv: -kv[1][0])},
    })
    if variants:
        other = 'C4' if okw['grad'] == 'E6' else 'E6'
        other_label = 'mig4' if other == 'C4' else 'meg6'
        var = {}
        for vname, prec, scheme, grad, mode in (
                ('hybrid_fp64', 'fp64', 'hybrid', None, 'percell'),
                ('hybrid_global_fp64', 'fp64', 'hybrid', None, 'global'),
                ('cgbr_%s_fp64' % grad_label, 'fp64', 'cgbr', None, 'percell'),
                ('cgbr_%s_mixed' % grad_label, 'mixed', 'cgbr', None, 'percell'),
                ('cgbr_%s_fp64' % other_label, 'fp64', 'cgbr', other, 'percell'),
                ('cgbr_%s_mixed' % other_label, 'mixed', 'cgbr', other, 'percell'),
                ('lad_e4_fp64', 'fp64', 'lad', None, 'percell'),
                ('lad_e4_mixed', 'mixed', 'lad', None, 'percell')):
            ctx = context(prec, grad, mode)
            vms, _, vbad, _, _ = timed(ctx, scheme)
            ctx.close()
            torch.cuda.empty_cache()
            var[vname] = {'ms_per_step': round(vms, 4), 'mcell_per_s': round(cells / (vms * 1e-3) / 1e6, 1),
                          'nonphysical_nodes': vbad}
        res['variants'] = var
    if cpu:
        res['cpu_baseline'] = cpu_baseline(name)
    return res


def cpu_baseline(name):
    """The FP64 oracle as it stands, one SSP-RK3 step on a bounded sample, one host thread."""
    from oracle import grid as ogrid, rhs as orhs
    from paper_2511_18042_amd import cases
    if name == 'triple_point':
        c = cases.triple_point()
        gas = orhs.Gas()
        opts = orhs.Opts(rho_thr=0.5 * 0.125)
        sample = 'one SSP-RK3 step of the per-cell hybrid RHS on the full 1792x768 triple-point initial state'
    else:
        c = cases.ramp3d(128, 96, 32)
        e = c.extra
        gas = orhs.Gas(gamma=1.4, Re=e['Re'], Pr=e['Pr'], Mref=e['Mref'], suth=e['suth'], viscous=True)
        opts = orhs.Opts(grad='C4', p_thr=e['p_thr'])
        sample = ('one SSP-RK3 step of the per-cell hybrid MIG4 RHS on a 128x96x32 ramp grid from the same '
                  'generator (rate per cell-update, scales linearly with cells)')
    g = ogrid.Grid(c.ndim, c.n, c.bc, c.h, c.coords)
    M = ogrid.node_metrics(g)
    t0 = time.perf_counter()
    orhs.rk3_step(c.Q, 0.0, 1e30, g, gas, opts, 'hybrid', M)
    s = time.perf_counter() - t0
    return {'value': round(c.cells / s / 1e6, 4), 'unit': 'Mcell-updates/s', 'cores': 1, 'kind': 'oracle',
            'sample': '%s; %.1f s' % (sample, s)}


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
    names = ['ramp3d', 'triple_point'] if args.workload == 'all' else [args.workload]
    results = {}
    for nm in names:
        results[nm] = run_workload(nm, args.steps, args.warmup, args.variants == 'all', not args.no_cpu_baseline)
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
        'data': 'synthetic: seeded generator states advanced by the warm-up steps',
        'config': {'workload': head['workload'], 'cells': head['cells'], 'parallelism': 'single GPU'},
        'roofline': head['roofline'],
        'cpu_baseline': head.get('cpu_baseline'),
        'nonphysical_nodes': head['nonphysical_nodes'],
        'workloads': results,
    }
    print(json.dumps(out))


if __name__ == '__main__':
    main()
