#!/usr/bin/env python3
"""Throughput of the hybrid LAD-GBR right-hand side on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one SSP-RK3 step of the whole hot path (ghost images, primitives, troubled
flags, gradients, sensor, LAD coefficients, interface sweeps, stage combination and the
CFL reduction) on the 2D triple-point workload: 1792 x 768 cells on [0,7] x [0,3], the
three-state initial condition, reflective walls, CFL 0.2, per-cell hybrid with the
density criterion rho < 0.5 rho_C3 = 0.0625.  Inputs are resident in HBM before timing.

Prints one JSON line: the headline is the per-cell hybrid with FP32 bulk arithmetic and
FP64 state (``value``), next to the FP64 hybrid, C-GBR (MEG6 and MIG4) and LAD-E4 rates,
the per-kernel breakdown, the roofline of the dominant kernel (its algorithmic bytes per
launch over its average launch time, HIP events on the library's stream) and the FP64
CPU oracle timed on this host.
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
RHO_THR = 0.5 * 0.125


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=50)
    ap.add_argument('--warmup', type=int, default=10)
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--variants', default='all', help="'all' or 'none'")
    return ap.parse_args()


def algorithmic_bytes(kclass, nodes, rs, ndim, gbr_frac):
    """Bytes one launch of a kernel class must move at minimum, per the algorithm
    (each input read once, each output written once), for ``nodes`` interior nodes.
    rs = bytes of the bulk real type.  See the design notes for the derivation."""
    if kclass == 'sweep_x':
        # LAD interface: node fluxes F (5 rs); C-GBR interface: W (5 rs), gradient (5 rs),
        # Omega (rs); flag byte; dQ/dt written (5 x 8 B, first direction)
        per = (1 - gbr_frac) * 5 * rs + gbr_frac * 11 * rs + 1 + 40
    elif kclass in ('sweep_y', 'sweep_z'):
        per = (1 - gbr_frac) * 5 * rs + gbr_frac * 11 * rs + 1 + 80   # dQ/dt read + written
    elif kclass == 'lad_flux':
        per = 5 * rs + 3 * rs + 5 * rs * ndim                            # W, coefficients -> F_l
    elif kclass == 'lad_raw':
        per = 5 * rs + 3 * rs + 3 * rs                                   # W, |S| theta e -> raw
    elif kclass == 'lad_node':
        per = 5 * rs + 3 * rs
    elif kclass == 'gauss':
        per = 3 * rs + 3 * rs
    elif kclass == 'grad_e6':
        per = 5 * rs + 5 * rs
    elif kclass == 'grad_c4':
        per = 40 + 5 * rs
    elif kclass == 'sensor':
        per = rs + 3 * ndim * rs + rs
    elif kclass == 'prim':
        per = 40 + 5 * rs + 1
    elif kclass == 'combine':
        per = 40 * 4
    else:
        per = 0.0
    return per * nodes


def main():
    args = parse()
    if args.gpus != 1:
        print('bench.py: this build measures one GPU only (one process, one MI355X); '
              '--gpus %d is not supported' % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2511_18042_amd import cases, lgbr

    torch.cuda.set_device(0)
    c = cases.triple_point()
    cells = c.cells
    K, W = args.steps, args.warmup

    def context(precision, grad='E6', mode='percell'):
        return lgbr.Context(lgbr.make_grid(2, c.n, c.bc, c.h), lgbr.make_gas(gamma=1.4),
                            lgbr.make_opts(grad=grad, precision=precision, cfl=0.2, rho_thr=RHO_THR,
                                           hybrid_mode=mode))

    def timed(ctx, scheme, prof_class=None):
        Q = torch.from_numpy(c.Q).cuda()
        t = torch.zeros(1, dtype=torch.float64, device='cuda')
        for _ in range(W):
            ctx.rk3_step(scheme, Q, c.t_end, t)
        torch.cuda.synchronize()
        if prof_class is not None:
            ctx.prof_start(prof_class, 64 * K + 64)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(K):
            ctx.rk3_step(scheme, Q, c.t_end, t)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / K
        kern = ctx.prof_stop() if prof_class is not None else None
        bad = ctx.poll_status()
        fl = torch.zeros(c.shape, dtype=torch.uint8, device='cuda')
        dQ = torch.zeros_like(Q)
        ctx.hybrid_rhs(Q, dQ, None, fl)
        torch.cuda.synchronize()
        flags = fl.cpu().numpy().astype(bool)
        return ms, kern, bad, float(t.item()), flags

    # --- per-kernel breakdown of the headline configuration (events around every launch)
    head = context('mixed')
    _, breakdown, _, _, _ = timed(head, 'hybrid', prof_class=-1)
    dominant = max(breakdown, key=lambda k: breakdown[k][0])
    # --- headline timed region: events only around the dominant kernel's launches
    ms, kern, bad, t_end, flags = timed(head, 'hybrid', prof_class=dominant)
    head.close()
    value = cells / (ms * 1e-3) / 1e6

    # selected-interface fraction (dilated troubled flags) at the end of the timed region
    from scipy.ndimage import maximum_filter
    ft = maximum_filter(flags.astype(np.uint8), size=7, mode='constant') > 0
    gbr_frac = float(ft[0, 5:-5, 5:-5].mean())
    dom_ms, dom_n = kern[dominant]
    dom_avg = dom_ms / max(dom_n, 1)
    algo = algorithmic_bytes(dominant, cells, 4, 2, gbr_frac)
    achieved = algo / (dom_avg * 1e-3) / 1e9

    variants = {}
    if args.variants == 'all':
        for name, prec, scheme, grad, mode in (('hybrid_fp64', 'fp64', 'hybrid', 'E6', 'percell'),
                                               ('hybrid_global_fp64', 'fp64', 'hybrid', 'E6', 'global'),
                                               ('cgbr_meg6_fp64', 'fp64', 'cgbr', 'E6', 'percell'),
                                               ('cgbr_meg6_mixed', 'mixed', 'cgbr', 'E6', 'percell'),
                                               ('cgbr_mig4_fp64', 'fp64', 'cgbr', 'C4', 'percell'),
                                               ('cgbr_mig4_mixed', 'mixed', 'cgbr', 'C4', 'percell'),
                                               ('lad_e4_fp64', 'fp64', 'lad', 'E6', 'percell'),
                                               ('lad_e4_mixed', 'mixed', 'lad', 'E6', 'percell')):
            ctx = context(prec, grad, mode)
            vms, _, vbad, _, _ = timed(ctx, scheme)
            ctx.close()
            variants[name] = {'ms_per_step': round(vms, 4), 'mcell_per_s': round(cells / (vms * 1e-3) / 1e6, 1),
                              'nonphysical_nodes': vbad}

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import grid as ogrid, rhs as orhs
        g = ogrid.Grid(c.ndim, c.n, c.bc, c.h)
        M = ogrid.node_metrics(g)
        t0 = time.perf_counter()
        orhs.rk3_step(c.Q, 0.0, c.t_end, g, orhs.Gas(), orhs.Opts(rho_thr=RHO_THR), 'hybrid', M)
        cpu_s = time.perf_counter() - t0
        cpu = {'value': round(cells / cpu_s / 1e6, 4), 'unit': 'Mcell-updates/s', 'cores': 1, 'kind': 'oracle',
               'sample': 'one SSP-RK3 step of the per-cell hybrid RHS (FP64 numpy oracle) on the full '
                         '1792x768 triple-point initial state; %.1f s' % cpu_s}

    out = {
        'metric': 'Mcell-updates/s per RK3 step (hybrid vs C-GBR, FP32 vs FP64) and % HBM peak',
        'value': round(value, 2),
        'unit': 'Mcell-updates/s',
        'n_gpus': 1,
        'steps': K,
        'warmup': W,
        'ms_per_step': round(ms, 4),
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'f32 (f64 state, RK combination, compact solves and flux differences)',
        'data': 'synthetic: the configured triple-point initial state advanced %d warm-up steps' % W,
        'config': {'workload': 'triple point 1792x768, hybrid LAD-E4/MEG6 per-cell, rho_thr 0.0625, CFL 0.2',
                   'cells': cells, 'parallelism': 'single GPU'},
        'nonphysical_nodes': bad,
        'sim_time_end': round(t_end, 6),
        'gbr_interface_fraction': round(gbr_frac, 5),
        'roofline': {'bound': 'hbm', 'kernel': dominant, 'achieved': round(achieved, 1), 'peak': HBM_PEAK_GBS,
                     'unit': 'GB/s', 'frac': round(achieved / HBM_PEAK_GBS, 4),
                     'avg_launch_ms': round(dom_avg, 5), 'launches': dom_n,
                     'algorithmic_bytes_per_launch': int(algo), 'traffic': None},
        'kernel_breakdown_ms_per_step': {k: round(v[0] / K, 4) for k, v in sorted(breakdown.items(),
                                                                                   key=lambda kv: -kv[1][0])},
        'variants': variants,
        'cpu_baseline': cpu,
    }
    print(json.dumps(out))


if __name__ == '__main__':
    main()
