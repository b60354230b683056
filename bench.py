#!/usr/bin/env python3
"""Throughput of the hybrid LAD-GBR right-hand side on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload all|ramp3d|triple_point|batch64] [--no-cpu-baseline]
                    [--variants all|none] [--copy-probe-mib M]

A step is one SSP-RK3 step of the whole hot path (ghost images, primitives, troubled
flags, gradients, sensor, LAD coefficients, interface fluxes, stage combination, the
implicit filter after LAD phases and the CFL reduction) on synthetic inputs resident in HBM
before timing starts.

Headline workload (``value``): the M2.9 24-degree compression-ramp stand-in, 1024 x 384 x
128 cells on a curvilinear grid (tanh wall clustering, spanwise periodic), viscous
(Sutherland, Re 2e4, Pr 0.72), hybrid of LAD-E4 and C-GBR with compact MIG4 gradients,
troubled where p < 0.5 p_inf, the paper's global switch (any troubled node puts the whole
field on C-GBR for that stage), FP32 bulk arithmetic with FP64 state, at the paper's stage
mix: C-GBR phases (forced by a second context of the same hybrid whose threshold marks every
node troubled) take 17.6 % of the steps, as the paper reports for its M2.9 run (Sec. 5);
from this generator's state the switch itself finds no troubled node for thousands of steps.
W warm-up steps (default 10), six steps that find the dominant kernel class, then exactly K
timed steps; the natural window (no forcing) is reported beside it.  Also on the same grid: the same window
in FP64 (with the FP32-bulk error against it), the per-cell switch, the C-GBR and LAD forms
(median of five timed blocks), and the per-cell hybrid right-hand side with forced troubled
tiles against the cost-weighted ideal.  Further workloads: the 2D triple point (1792 x 768),
its FP64 run to t = 5 (LAD share beside the paper's 13.6 %) and a window from t = 3, and 64
independent four-quadrant Riemann problems advanced 100 hybrid RK3 steps per graph launch.

Each workload reports its dominant kernel's roofline from live HIP-event times of that
class's launches inside the timed steps (algorithmic bytes per launch over the average
launch time), and the whole step against the method's algorithmic floor.  The FP64 CPU
oracle is timed on this host's cores before the GPU is used.
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
    ap.add_argument('--profile-summary', default=None, metavar='OUT',
                    help='write a per-kernel summary of rocprofv3 output (--trace, --fetch, --write csv files) to '
                         'OUT and exit; no GPU is used')
    ap.add_argument('--trace', default=None, help='rocprofv3 --kernel-trace csv (with --profile-summary)')
    ap.add_argument('--fetch', default=None, help='rocprofv3 --pmc FETCH_SIZE csv (with --profile-summary)')
    ap.add_argument('--write', default=None, help='rocprofv3 --pmc WRITE_SIZE csv (with --profile-summary)')
    ap.add_argument('--title', default='', help='first line of the summary (with --profile-summary)')
    ap.add_argument('--commands', default='', help='the commands that made the csv files, ; separated')
    return ap.parse_args()


def log(msg):
    print('[bench] ' + msg, file=sys.stderr, flush=True)


def algorithmic_bytes(kclass, nodes, rs, ndim, gbr_frac, viscous, curv, planar=False, global_hybrid=False):
    """Minimum bytes one launch of a kernel class moves (every input read once, every
    output written once) for ``nodes`` interior nodes; rs = bytes of the bulk real type,
    curv: node metrics (9 components + J) are fields rather than constants; planar: they
    (and the LAD grid factors) are stored for one plane only, so they add nothing per node.
    global_hybrid: the all-LAD pass of an RK3 step of the global hybrid also writes the
    primitives and troubled flags of its result in stages 1 and 2, and the filter guard's
    FP64 copy of it in stage 3 (the mean over the three launches)."""
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
        if global_hybrid:
            per += (2 * (5 * rs + 1) + 40) / 3.0
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
    elif kclass == 'filter':
        per = 80                                             # one direction: Q (FP64) in and out
    elif kclass == 'c6_faces':
        per = 5 * rs + (8 if per_node_geom else 0) + 80      # node fluxes, J, dQ/dt in and out
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

    def steps(self, ctx, scheme, Q0, K=None, W=None, prof_class=None, t_end=1e30, Q=None, t=None):
        """W untimed steps, then exactly K timed steps (HIP events around the K steps, the
        stream synchronised on both sides).  prof_class: a kernel class whose launches are
        bracketed by HIP events during the timed steps (live per-launch times).  Returns
        (ms per step, per-class (ms, launches) or None, non-physical count, state, t, switch
        record of the timed steps (hybrid stages, troubled ones))."""
        import torch
        K = self.K if K is None else K
        W = self.W if W is None else W
        Q = Q0.clone() if Q is None else Q
        t = torch.zeros(1, dtype=torch.float64, device='cuda') if t is None else t
        for _ in range(W):
            ctx.rk3_step(scheme, Q, t_end, t)
        torch.cuda.synchronize()
        ctx.switch_stats(reset=True)
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
        kern = ctx.prof_stop_launches() if prof_class is not None else None
        sw = ctx.switch_stats(reset=True)
        bad = ctx.poll_status()
        return ms, kern, bad, Q, t, sw

    def median_ms(self, ctx, scheme, Q0, K, W, repeats=5):
        """Median over ``repeats`` timed blocks of K steps (each after W warm-up steps from Q0)."""
        import statistics
        out, bad = [], 0
        for _ in range(repeats):
            ms, _, b, Q, _, _ = self.steps(ctx, scheme, Q0, K=K, W=W)
            del Q
            out.append(ms)
            bad += b
        return statistics.median(out), bad


def dominant_class(ctx, scheme, Q, t, steps=6):
    """Kernel class with the most time over a few steps from the given state (advances it)."""
    ctx.prof_start(-1, 400 * steps + 400)
    for _ in range(steps):
        ctx.rk3_step(scheme, Q, 1e30, t)
    brk = ctx.prof_stop()
    ctx.poll_status()
    ctx.switch_stats(reset=True)
    return max(brk, key=lambda k: brk[k][0]), {k: round(v[0] / steps, 4) for k, v in
                                                sorted(brk.items(), key=lambda kv: -kv[1][0])}


EXECUTED_FRACTION = 0.25   # a launch shorter than this share of its class's longest one returned at once


def live_roofline(kern, dom, cells, ndim, gbr_frac, viscous, curv, planar, traffic_file=None, global_hybrid=False):
    """Roofline of the dominant class from its live per-launch HIP-event times in the timed
    steps: algorithmic bytes per launch over the average duration of the launches that did
    the work.  Launches the device-side hybrid switch turned into immediate returns (a few
    microseconds against milliseconds) are counted apart and left out of the average."""
    _, each = kern
    dur = [ms for k, ms in each if k == dom]
    top = max(dur)
    run = [ms for ms in dur if ms >= EXECUTED_FRACTION * top]
    dom_avg = sum(run) / len(run)
    algo = algorithmic_bytes(dom, cells, 4, ndim, gbr_frac, viscous, curv, planar, global_hybrid)
    achieved = algo / (dom_avg * 1e-3) / 1e9
    roof = {'bound': 'hbm', 'kernel': dom, 'achieved': round(achieved, 1), 'peak': HBM_PEAK_GBS, 'unit': 'GB/s',
            'frac': round(achieved / HBM_PEAK_GBS, 4), 'avg_launch_ms': round(dom_avg, 5), 'launches': len(run),
            'skipped_launches': len(dur) - len(run), 'algorithmic_bytes_per_launch': int(algo),
            'timing': 'live HIP events around each launch of the class on the library stream during the timed '
                      'steps; launches under %g of the longest are immediate returns of the hybrid switch and are '
                      'not averaged' % EXECUTED_FRACTION, 'traffic': None}
    if traffic_file:
        tr, why = profiled_traffic(traffic_file, dom)
        roof['traffic'] = tr['bytes'] if tr else None
        roof['traffic_source'] = os.path.relpath(traffic_file, ROOT) + ('' if tr else ' (%s)' % why)
        if tr:
            roof['traffic_over_algorithmic'] = round(tr['bytes'] / algo, 3)
            roof['profile_avg_launch_ms'] = tr['profile_avg_launch_ms']
    return roof


def step_floor(cells, ms, bytes_per_cell):
    """The whole RK3 step against the method's algorithmic floor (state read and written
    once per stage, U^n re-read in stages 2-3, metrics): bytes per cell over the step time."""
    gbs = bytes_per_cell * cells / (ms * 1e-3) / 1e9
    return {'bytes_per_cell': bytes_per_cell, 'achieved': round(gbs, 1), 'unit': 'GB/s',
            'frac': round(gbs / HBM_PEAK_GBS, 4)}


def precision_error(Qa, Qb, gamma=1.4):
    """L1 (mean) and Linf of the primitive variables of two interior states (FP32 bulk
    against FP64), absolute and relative to the FP64 field's largest magnitude."""
    import numpy as np
    A = Qa.double().cpu().numpy()
    B = Qb.double().cpu().numpy()
    sl = tuple(slice(5, -5) if A.shape[1 + ax] > 1 else slice(None) for ax in range(3))
    A, B = A[(slice(None),) + sl], B[(slice(None),) + sl]

    def prim(Q):
        rho = Q[0]
        u, v, w = Q[1] / rho, Q[2] / rho, Q[3] / rho
        p = (gamma - 1.0) * (Q[4] - 0.5 * rho * (u * u + v * v + w * w))
        return {'rho': rho, 'u': u, 'v': v, 'w': w, 'p': p}
    pa, pb = prim(A), prim(B)
    out = {}
    for k in ('rho', 'u', 'v', 'w', 'p'):
        scale = float(np.max(np.abs(pb[k])))
        if scale == 0.0:
            continue
        d = np.abs(pa[k] - pb[k])
        out[k] = {'L1': float(np.mean(d)), 'Linf': float(np.max(d)), 'L1_rel': float(np.mean(d) / scale),
                  'Linf_rel': float(np.max(d) / scale)}
    return out


def _profile_lines(path):
    """(KTIME, TRAFFIC) dicts by class of a committed summary written by --profile-summary,
    or (None, reason) once any library source no longer hashes to what was profiled."""
    import hashlib
    if not os.path.exists(path):
        return None, 'no profile'
    kt, tr, sha, files = {}, {}, None, None
    for line in open(path):
        f = line.split()
        if len(f) < 2:
            continue
        if f[0] == 'SOURCES':
            kv = dict(x.split('=', 1) for x in f[1:])
            sha, files = kv['sha256'], kv['files'].split(',')
        elif f[0] in ('KTIME', 'TRAFFIC'):
            kv = dict(x.split('=', 1) for x in f[2:])
            (kt if f[0] == 'KTIME' else tr)[f[1]] = kv
    if sha is None:
        return None, 'no SOURCES line'
    h = hashlib.sha256()
    for src in files:
        h.update(open(os.path.join(ROOT, src), 'rb').read())
    if h.hexdigest() != sha:
        return None, 'library sources changed since the profile was taken'
    return (kt, tr), ''


def profiled_traffic(path, kclass):
    """Counted HBM bytes per executed launch of kernel class kclass (FETCH_SIZE and
    WRITE_SIZE scaled by a copy of known size) and the profile's own average launch time,
    from a committed summary; (None, reason) otherwise."""
    got, why = _profile_lines(path)
    if got is None:
        return None, why
    kt, tr = got
    if kclass in ('sweep_y', 'sweep_z') and kclass not in tr:
        kclass = 'sweep_yz'   # one kernel serves both directions
    if kclass not in tr:
        return None, 'no counters for this kernel class'
    return {'bytes': int(float(tr[kclass]['bytes'])),
            'profile_avg_launch_ms': float(kt[kclass]['avg_ms']) if kclass in kt else None}, ''


def profiled_step(path, launches_per_step):
    """Whole-step counted HBM bytes: each class's counted bytes per executed launch times its
    executed launches per step (measured live); (None, reason) when a class has no counters."""
    got, why = _profile_lines(path)
    if got is None:
        return None, why
    _, tr = got

    def key(k):   # the profile names the strided sweeps of eta and zeta (one kernel) together
        return 'sweep_yz' if k in ('sweep_y', 'sweep_z') and k not in tr else k
    missing = [k for k in launches_per_step if key(k) not in tr and launches_per_step[k] > 0]
    total = sum(float(tr[key(k)]['bytes']) * n for k, n in launches_per_step.items() if key(k) in tr)
    return {'bytes_per_step': int(total), 'classes_without_counters': missing}, ''


def flags_of(ctx, Q):
    import torch
    fl = torch.zeros(tuple(Q.shape[1:]), dtype=torch.uint8, device='cuda')
    dQ = torch.empty_like(Q)
    ctx.hybrid_rhs(Q, dQ, None, fl)
    torch.cuda.synchronize()
    return fl.cpu().numpy().astype(bool)


# ------------------------------------------------------------------ M2.9 ramp (headline)
RAMP_FLOOR_B_PER_CELL = 320   # state 3 x (40 + 40) + U^n 2 x 40; metrics: one plane (extruded grid)
PAPER_GBR_STEP_SHARE = 0.176  # Sec. 5: on the M2.9 ramp the hybrid runs LAD 82.4 % of the time


def mix_window(ctx_lad, ctx_gbr, Q, t, W, K, share=PAPER_GBR_STEP_SHARE, prof=True):
    """W warm-up steps, six steps that find the dominant class (prof), then exactly K timed
    steps of the global hybrid on Q, step i (counted from the first warm-up step) taken by
    ctx_gbr (every node troubled: a C-GBR phase) when floor((i + 1) share) > floor(i share),
    by ctx_lad (the switch as it finds the state) otherwise.  HIP events around the K steps,
    the stream synchronised on both sides.  Returns (ms per step, (per-class, per-launch)
    times of the dominant class in the timed steps, non-physical count, (hybrid stages,
    troubled stages) of the timed steps, dominant class, per-class ms per step of the six
    steps, forced steps in the window)."""
    import torch

    def ctx_of(i):
        return ctx_gbr if int((i + 1) * share) > int(i * share) else ctx_lad
    i = 0
    for _ in range(W):
        ctx_of(i).rk3_step('hybrid', Q, 1e30, t)
        i += 1
    dom, brk = None, None
    if prof:
        for cx in (ctx_lad, ctx_gbr):
            cx.prof_start(-1, 2400)
        for _ in range(6):
            ctx_of(i).rk3_step('hybrid', Q, 1e30, t)
            i += 1
        tot, each = {}, []
        for cx in (ctx_lad, ctx_gbr):
            p, e = cx.prof_stop_launches()
            for k, v in p.items():
                tot[k] = tot.get(k, 0.0) + v[0]
            each += e
            cx.poll_status()
        dom = max(tot, key=tot.get)
        brk = {k: round(v / 6, 4) for k, v in sorted(tot.items(), key=lambda kv: -kv[1])}
        lps = {}   # executed launches per step of each class
        for k in tot:
            d = [ms for kk, ms in each if kk == k]
            lps[k] = sum(1 for ms in d if ms >= EXECUTED_FRACTION * max(d)) / 6.0
        brk = {'ms_per_step': brk, 'executed_launches_per_step': lps}
    else:
        for _ in range(6):
            ctx_of(i).rk3_step('hybrid', Q, 1e30, t)
            i += 1
    torch.cuda.synchronize()
    for cx in (ctx_lad, ctx_gbr):
        cx.switch_stats(reset=True)
        if prof:
            cx.prof_start(dom, 400 * K + 400)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    n_gbr = 0
    e0.record()
    for _ in range(K):
        cx = ctx_of(i)
        n_gbr += cx is ctx_gbr
        cx.rk3_step('hybrid', Q, 1e30, t)
        i += 1
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / K
    kern = None
    if prof:
        per, each = {}, []
        for cx in (ctx_lad, ctx_gbr):
            p, e = cx.prof_stop_launches()
            for k, v in p.items():
                a = per.get(k, (0.0, 0))
                per[k] = (a[0] + v[0], a[1] + v[1])
            each += e
        kern = (per, each)
    sw = [0, 0]
    bad = 0
    for cx in (ctx_lad, ctx_gbr):
        a = cx.switch_stats(reset=True)
        sw[0] += a[0]
        sw[1] += a[1]
        bad += cx.poll_status()
    return ms, kern, bad, sw, dom, brk, n_gbr


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

    def context(precision, grad='C4', mode='global', lad='E4', p_thr=e['p_thr']):
        return lgbr.Context(grid, gas, lgbr.make_opts(precision=precision, cfl=0.2, grad=grad, hybrid_mode=mode,
                                                      p_thr=p_thr, lad=lad), metrics, coords)

    desc = ('M2.9 24-deg ramp stand-in 1024x384x128 curvilinear, viscous, hybrid LAD-E4/MIG4 (global switch, '
            'LAD phases filtered) at the paper stage mix (C-GBR steps forced at 17.6 %), p_thr 0.5 p_inf, CFL 0.2')
    res = {'workload': desc, 'cells': cells}
    traffic = os.path.join(ROOT, 'profiles', 'ramp3d_hybrid_paper_mix_mixed.txt')
    # headline: the hybrid at the paper's stage mix (Sec. 5: LAD 82.4 % of the M2.9 run).  From
    # this generator's state the switch finds no troubled node for thousands of steps (the
    # corner interaction that produces them in the paper develops over a flow-through), so
    # the C-GBR phases are forced: a second context of the same hybrid whose pressure
    # threshold marks every node troubled takes a 17.6 % share of the steps, spread evenly
    # (step i is C-GBR when floor((i + 1) s) > floor(i s), s = 0.176).  W warm-up steps, the
    # dominant kernel class over six more, then exactly K timed steps with that class's
    # launches timed live on both contexts.  The natural window (the same steps, no forcing)
    # is reported beside it.
    if args.only_variant:   # one variant alone (profiling): no headline window
        return ramp3d_variants(args, R, res, context, Q0, cells, variants=True)
    head = context('mixed')
    forced = context('mixed', p_thr=1e30)
    log('ramp3d: headline at the paper stage mix, %d warm-up + %d timed steps' % (args.warmup, args.steps))
    Q = Q0.clone()
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    ms, kern, bad, sw, dom, brk, n_gbr = mix_window(head, forced, Q, t, args.warmup, args.steps)
    planar = head.metrics_planar()
    roof = live_roofline(kern, dom, cells, 3, 1.0, True, True, planar, traffic_file=traffic, global_hybrid=True)
    res.update({'value': mcell(cells, ms), 'ms_per_step': round(ms, 4), 'nonphysical_nodes': bad,
                'steps_before_window': args.warmup + 6, 'sim_time_end': round(float(t.item()), 6),
                'stage_mix': {'forced_cgbr_steps': n_gbr, 'steps': args.steps, 'hybrid_stages': sw[0],
                              'cgbr_stages': sw[1], 'lad_share': round(1 - sw[1] / max(sw[0], 1), 4),
                              'paper_lad_share': 0.824,
                              'how': 'C-GBR steps forced by a second context of the same global hybrid whose '
                                     'pressure threshold marks every node troubled, at a share of %.3f of the '
                                     'steps spread evenly' % PAPER_GBR_STEP_SHARE},
                'roofline': roof, 'roofline_step_floor': step_floor(cells, ms, RAMP_FLOOR_B_PER_CELL),
                'kernel_breakdown': brk})
    forced.close()
    # the natural window: the same number of steps from the same input, troubled stages as
    # the switch finds them
    Qn = Q0.clone()
    tn = torch.zeros(1, dtype=torch.float64, device='cuda')
    msn, _, badn, Qn, tn, swn = R.steps(head, 'hybrid', None, W=args.warmup + 6, Q=Qn, t=tn)
    res['natural_window'] = {'ms_per_step': round(msn, 4), 'mcell_per_s': mcell(cells, msn), 'nonphysical_nodes': badn,
                             'hybrid_stages': swn[0], 'cgbr_stages': swn[1],
                             'lad_share': round(1 - swn[1] / max(swn[0], 1), 4)}
    del Qn
    st, why = profiled_step(traffic, brk['executed_launches_per_step'])
    if st:   # whole-step figure: every kernel's counted HBM bytes over the measured step time
        gbs = st['bytes_per_step'] / (ms * 1e-3) / 1e9
        res['hbm_step'] = {'bytes_per_step': st['bytes_per_step'], 'achieved': round(gbs, 1), 'unit': 'GB/s',
                           'frac_of_peak': round(gbs / HBM_PEAK_GBS, 4),
                           'classes_without_counters': st['classes_without_counters'],
                           'how': 'each class: counted bytes per executed launch (profile) x executed launches per '
                                  'step (six live-profiled steps of the same mix)',
                           'source': os.path.relpath(traffic, ROOT)}
    else:
        res['hbm_step'] = {'source': os.path.relpath(traffic, ROOT) + ' (%s)' % why}
    Q32 = Q
    head.close()
    torch.cuda.empty_cache()
    if variants and not args.only_variant:
        # the same window in FP64: throughput and the FP32-bulk error after the same steps
        log('ramp3d: FP64 over the same steps')
        h64 = context('fp64')
        f64 = context('fp64', p_thr=1e30)
        Q64 = Q0.clone()
        t64 = torch.zeros(1, dtype=torch.float64, device='cuda')
        ms64, _, bad64, sw64, _, _, _ = mix_window(h64, f64, Q64, t64, args.warmup, args.steps, prof=False)
        res['fp64_same_window'] = {'ms_per_step': round(ms64, 4), 'mcell_per_s': mcell(cells, ms64),
                                   'nonphysical_nodes': bad64, 'stages': list(sw64),
                                   'fp32_speedup': round(ms64 / ms, 3)}
        res['fp32_vs_fp64_after_window'] = {'steps': args.warmup + 6 + args.steps,
                                            'error': precision_error(Q32, Q64)}
        h64.close()
        f64.close()
        del Q64
        torch.cuda.empty_cache()
        log('ramp3d: forced-flag sweep')
        pc = context('mixed', mode='percell')
        res['forced_flag_sweep'] = forced_sweep(pc, Q0, tuple(metrics.shape[1:]))
        pc.close()
    del Q32
    torch.cuda.empty_cache()
    res = ramp3d_variants(args, R, res, context, Q0, cells, variants)
    if cpu:
        res['cpu_baseline'] = cpu['ramp3d']
    return res


def ramp3d_variants(args, R, res, context, Q0, cells, variants):
    """The config-4 variants (median of five timed blocks from the initial state) and the
    paper's per-stage LAD / C-GBR speed-up study; with --only-variant, that one alone with
    its per-class breakdown."""
    import torch
    if variants:
        var = {}
        for vname, prec, scheme, grad, mode, *vv in (
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
            vms, vbad = R.median_ms(ctx, scheme, Q0, K=min(args.steps, 10), W=2)
            var[vname] = {'ms_per_step': round(vms, 4), 'mcell_per_s': mcell(cells, vms), 'nonphysical_nodes': vbad,
                          'timing': 'median of 5 blocks of %d steps from the initial state' % min(args.steps, 10)}
            if vname.startswith('lad_c6') or args.only_variant:
                _, kern, _, _, _, _ = R.steps(ctx, scheme, Q0, K=5, W=1, prof_class=-1)
                var[vname]['kernel_breakdown_ms_per_step'] = {
                    k: round(v[0] / 5, 4) for k, v in sorted(kern[0].items(), key=lambda kv: -kv[1][0])}
            ctx.close()
            torch.cuda.empty_cache()
        res['variants'] = var
        if args.only_variant:
            return res
        # the paper's per-stage speed-up study: LAD-C6 / LAD-E4 against MEG6 / MIG4 C-GBR (FP64 there)
        res['lad_speedup'] = {
            p: {'lad_c6_over_meg6': round(var['cgbr_meg6_' + p]['ms_per_step'] / var['lad_c6_' + p]['ms_per_step'], 3),
                'lad_c6_over_mig4': round(var['cgbr_mig4_' + p]['ms_per_step'] / var['lad_c6_' + p]['ms_per_step'], 3),
                'lad_e4_over_meg6': round(var['cgbr_meg6_' + p]['ms_per_step'] / var['lad_e4_' + p]['ms_per_step'], 3),
                'lad_e4_over_mig4': round(var['cgbr_mig4_' + p]['ms_per_step'] / var['lad_e4_' + p]['ms_per_step'], 3)}
            for p in ('fp64', 'mixed')}
        res['lad_speedup']['paper_a100_fp64'] = {'lad_c6_over_meg6': '1.17-1.22', 'lad_c6_over_mig4': '1.38-1.43',
                                                 'lad_e4_over_meg6': '1.9-2.0', 'lad_e4_over_mig4': '2.2-2.3'}
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
        frac = interface_fraction(full)
        ideal = (1 - frac) * out['rhs_ms']['lad'] + frac * out['rhs_ms']['cgbr']
        out['rhs_ms']['hybrid_%g%%' % (100 * f)] = {'ms': round(ms, 4), 'interface_fraction': round(frac, 4),
                                                    'cost_weighted_ideal_ms': round(ideal, 4),
                                                    'over_ideal': round(ms / ideal, 3)}
        del fl
    return out


# ------------------------------------------------------------------ oracle on the host cores
def host_info():
    model = ''
    try:
        for line in open('/proc/cpuinfo'):
            if line.startswith('model name'):
                model = line.split(':', 1)[1].strip()
                break
    except OSError:
        pass
    return {'os_cpu_count': os.cpu_count(), 'cpu_model': model}


def _oracle_ramp_step(args):
    """One SSP-RK3 step of the oracle's global hybrid (MIG4, LAD-E4 filtered) on a crop of the
    ramp generator; returns (cells, seconds)."""
    nx, ny, nz = args
    from oracle import grid as ogrid, rhs as orhs
    from paper_2511_18042_amd import cases
    c = cases.ramp3d(nx, ny, nz)
    e = c.extra
    gas = orhs.Gas(gamma=1.4, Re=e['Re'], Pr=e['Pr'], Mref=e['Mref'], suth=e['suth'], viscous=True)
    opts = orhs.Opts(grad='C4', p_thr=e['p_thr'], hybrid_mode='global')
    g = ogrid.Grid(c.ndim, c.n, c.bc, c.h, c.coords)
    M = ogrid.node_metrics(g)
    t0 = time.perf_counter()
    orhs.rk3_step(c.Q, 0.0, 1e30, g, gas, opts, 'hybrid', M)
    return c.cells, time.perf_counter() - t0


def _oracle_tp_steps(args):
    """``n`` SSP-RK3 steps of the oracle's global hybrid on the triple point at (nx, ny)."""
    nx, ny, n = args
    from oracle import grid as ogrid, rhs as orhs
    from paper_2511_18042_amd import cases
    c = cases.triple_point(nx, ny)
    g = ogrid.Grid(c.ndim, c.n, c.bc, c.h, c.coords)
    M = ogrid.node_metrics(g)
    opts = orhs.Opts(rho_thr=c.extra['rho_thr'], p_thr=c.extra['p_thr'], hybrid_mode='global')
    Q, t = c.Q, 0.0
    t0 = time.perf_counter()
    for _ in range(n):
        Q, t, _, _ = orhs.rk3_step(Q, t, 1e30, g, orhs.Gas(), opts, 'hybrid', M)
    return n * c.cells, time.perf_counter() - t0


def _oracle_batch_problem(c):
    """One SSP-RK3 step of the oracle's global hybrid on one batch problem."""
    from oracle import grid as ogrid, rhs as orhs
    g = ogrid.Grid(c.ndim, c.n, c.bc, c.h, c.coords)
    M = ogrid.node_metrics(g)
    opts = orhs.Opts(rho_thr=c.extra['rho_thr'], p_thr=c.extra['p_thr'], hybrid_mode='global')
    t0 = time.perf_counter()
    orhs.rk3_step(c.Q, 0.0, 1e30, g, orhs.Gas(), opts, 'hybrid', M)
    return c.cells, time.perf_counter() - t0


def _pool_rate(fn, tasks, workers):
    """Oracle throughput with ``workers`` host processes on independent tasks: total cells
    over the wall time of the pool (forked before the GPU is touched)."""
    import multiprocessing as mp
    t0 = time.perf_counter()
    with mp.get_context('fork').Pool(workers) as pool:
        out = pool.map(fn, tasks)
    wall = time.perf_counter() - t0
    cells = sum(o[0] for o in out)
    return cells / wall / 1e6, wall, cells


def cpu_baselines(names):
    """The FP64 oracle as it stands, timed on this host before any GPU work: one thread on a
    bounded sample, and all host cores (up to 16 worker processes) on independent samples
    of the same workload.  Rates in cell-updates per second of one RK3 step."""
    info = host_info()
    workers = max(1, min(16, os.cpu_count() or 1))
    out = {}
    if 'ramp3d' in names:
        log('cpu baseline: ramp crops')
        cells, sec = _oracle_ramp_step((128, 96, 32))
        rate_all, wall, tot = _pool_rate(_oracle_ramp_step, [(128, 96, 32)] * workers, workers)
        out['ramp3d'] = dict(info, **{
            'value': round(rate_all, 4), 'unit': 'Mcell-updates/s', 'cores': workers, 'kind': 'oracle',
            'one_thread': round(cells / sec / 1e6, 4),
            'sample': ('one SSP-RK3 step of the global hybrid (MIG4 / LAD-E4 filtered) on a 128x96x32 crop of the '
                       'ramp generator: %.1f s on one thread; %d crops on %d worker processes in %.1f s wall'
                       % (sec, workers, workers, wall))})
    if 'triple_point' in names:
        log('cpu baseline: triple point')
        cells, sec = _oracle_tp_steps((448, 192, 3))
        rate_all, wall, _ = _pool_rate(_oracle_tp_steps, [(448, 192, 3)] * workers, workers)
        out['triple_point'] = dict(info, **{
            'value': round(rate_all, 4), 'unit': 'Mcell-updates/s', 'cores': workers, 'kind': 'oracle',
            'one_thread': round(cells / sec / 1e6, 4),
            'sample': ('three SSP-RK3 steps of the global hybrid on the triple point at 448x192 from t = 0: %.1f s on '
                       'one thread; %d copies on %d worker processes in %.1f s wall' % (sec, workers, workers, wall))})
    if 'batch64' in names:
        log('cpu baseline: batch problems')
        from paper_2511_18042_amd import cases
        probs = cases.batch64()
        small = [c for c in probs if c.cells <= 256 * 256]
        cells, sec = _oracle_batch_problem(small[0])
        rate_all, wall, tot = _pool_rate(_oracle_batch_problem, small, workers)
        out['batch64'] = dict(info, **{
            'value': round(rate_all, 4), 'unit': 'Mcell-updates/s', 'cores': workers, 'kind': 'oracle',
            'one_thread': round(cells / sec / 1e6, 4),
            'sample': ('one SSP-RK3 step of the global hybrid on each of the %d batch problems of at most 256^2 cells '
                       '(%d cells) on %d worker processes in %.1f s wall; one thread: the first of them alone, %.1f s'
                       % (len(small), tot, workers, wall, sec))})
    return out


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
                                                      rho_thr=c.extra['rho_thr'], p_thr=c.extra['p_thr'], lad=lad))

    desc = ('triple point 1792x768, hybrid LAD-E4/MEG6 (global switch, LAD phases filtered), rho_thr 0.0625, '
            'p_thr 0.025, CFL 0.2')
    res = {'workload': desc, 'cells': cells}
    head = context('mixed')
    log('triple_point: %d warm-up + %d timed steps' % (args.warmup, args.steps))
    Q = Q0.clone()
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    for _ in range(args.warmup):
        head.rk3_step('hybrid', Q, 1e30, t)
    dom, brk = dominant_class(head, 'hybrid', Q, t)
    ms, kern, bad, Q, t, sw = R.steps(head, 'hybrid', None, W=0, prof_class=dom, Q=Q, t=t)
    share = sw[1] / max(sw[0], 1)
    roof = live_roofline(kern, dom, cells, 2, 1.0, False, False, False, global_hybrid=True)
    res.update({'value': mcell(cells, ms), 'ms_per_step': round(ms, 4), 'nonphysical_nodes': bad,
                'sim_time_end': round(float(t.item()), 6),
                'stages': {'hybrid': sw[0], 'troubled_cgbr': sw[1], 'lad_share': round(1 - share, 4)},
                'roofline': roof, 'roofline_step_floor': step_floor(cells, ms, 320),
                'kernel_breakdown_ms_per_step': brk})
    Q32 = Q
    head.close()
    if variants:
        log('triple_point: FP64 over the same steps')
        h64 = context('fp64')
        Q64 = Q0.clone()
        t64 = torch.zeros(1, dtype=torch.float64, device='cuda')
        for _ in range(args.warmup + 6):
            h64.rk3_step('hybrid', Q64, 1e30, t64)
        ms64, _, bad64, Q64, t64, sw64 = R.steps(h64, 'hybrid', None, W=0, Q=Q64, t=t64)
        res['fp64_same_window'] = {'ms_per_step': round(ms64, 4), 'mcell_per_s': mcell(cells, ms64),
                                   'nonphysical_nodes': bad64, 'stages': list(sw64), 'fp32_speedup': round(ms64 / ms, 3)}
        res['fp32_vs_fp64_after_window'] = {'steps': args.warmup + 6 + args.steps, 'error': precision_error(Q32, Q64)}
        # the whole run to t = 5 with the paper's global switch (FP64): its LAD share (Sec. 5
        # reports 13.6 %) and whether it stays physical, with the configured reflective walls
        # and with the paper's extrapolated walls
        def run_to_t5(ctx):
            tt = torch.zeros(1, dtype=torch.float64, device='cuda')
            Qr = Q0.clone()
            b = lgbr.Batch([ctx], [Qr], [tt], [5.0], 500, 'hybrid')
            ctx.switch_stats(reset=True)
            t0 = time.perf_counter()
            while tt.item() < 5.0 and time.perf_counter() - t0 < 60:
                b.run()
                torch.cuda.synchronize()
            b.close()
            swr = ctx.switch_stats(reset=True)
            return {'t': round(float(tt.item()), 6), 'nonphysical_nodes': ctx.poll_status(), 'stages': swr[0],
                    'lad_share': round(1 - swr[1] / max(swr[0], 1), 4), 'paper_lad_share': 0.136,
                    'seconds': round(time.perf_counter() - t0, 2)}
        log('triple_point: FP64 hybrid runs to t = 5')
        res['run_to_t5_fp64'] = run_to_t5(h64)
        gx = lgbr.make_grid(2, c.n, [(cases.TRANSMISSIVE, cases.TRANSMISSIVE)] * 2, c.h)
        hx = lgbr.Context(gx, gas, lgbr.make_opts(precision='fp64', cfl=0.2, grad='E6', hybrid_mode='global',
                                                  rho_thr=c.extra['rho_thr'], p_thr=c.extra['p_thr']))
        res['run_to_t5_fp64_extrapolated_walls'] = run_to_t5(hx)
        hx.close()
        Q3 = Q0.clone()
        t3 = torch.zeros(1, dtype=torch.float64, device='cuda')
        b = lgbr.Batch([h64], [Q3], [t3], [3.0], 500, 'hybrid')
        while t3.item() < 3.0:
            b.run()
            torch.cuda.synchronize()
        b.close()
        h64.close()
        del Q64
        w3 = {'t': round(float(t3.item()), 6), 'advanced_with': 'hybrid_fp64'}
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
            vms, vbad = R.median_ms(ctx, scheme, Q3, K=min(args.steps, 20), W=2)
            ctx.close()
            w3[vname] = {'ms_per_step': round(vms, 4), 'mcell_per_s': mcell(cells, vms), 'nonphysical_nodes': vbad}
        res['window_t3'] = w3
        var = {}
        for vname, prec, scheme, grad, mode, *vv in (
                ('hybrid_percell_mixed', 'mixed', 'hybrid', 'E6', 'percell'),
                ('cgbr_meg6_fp64', 'fp64', 'cgbr', 'E6', 'global'),
                ('cgbr_meg6_mixed', 'mixed', 'cgbr', 'E6', 'global'),
                ('cgbr_mig4_fp64', 'fp64', 'cgbr', 'C4', 'global'),
                ('cgbr_mig4_mixed', 'mixed', 'cgbr', 'C4', 'global'),
                ('lad_e4_fp64', 'fp64', 'lad', 'E6', 'global'),
                ('lad_e4_mixed', 'mixed', 'lad', 'E6', 'global'),
                ('lad_c6_fp64', 'fp64', 'lad', 'E6', 'global', 'C6'),
                ('lad_c6_mixed', 'mixed', 'lad', 'E6', 'global', 'C6')):
            ctx = context(prec, grad, mode, *vv)
            vms, vbad = R.median_ms(ctx, scheme, Q0, K=min(args.steps, 20), W=2)
            ctx.close()
            var[vname] = {'ms_per_step': round(vms, 4), 'mcell_per_s': mcell(cells, vms), 'nonphysical_nodes': vbad}
        res['variants'] = var
    if cpu:
        res['cpu_baseline'] = cpu['triple_point']
    return res


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
                       'hybrid LAD-E4/MEG6 (global switch per problem, LAD phases filtered), %d RK3 steps per graph '
                       'launch' % nsteps,
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
        """One warm-up launch (nsteps steps), then one timed launch; per-problem
        non-physical counts over both (a problem counted bad invalidates the row)."""
        Qs = [q.clone() for q in Q0s]
        ts = [torch.zeros(1, dtype=torch.float64, device='cuda') for _ in probs]
        b = lgbr.Batch(ctxs, Qs, ts, [1e30] * len(probs), nsteps, scheme)
        b.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        b.close()
        bad = [cx.poll_status() for cx in ctxs]
        return ms / nsteps, bad, Qs

    def entry(ms, bad):
        nbad = sum(1 for v in bad if v)
        return {'ms_per_step': round(ms, 4), 'mcell_per_s': mcell(cells, ms), 'nonphysical_nodes': int(sum(bad)),
                'problems_nonphysical': nbad, 'valid': nbad == 0}

    finals = {}
    for precision in (('mixed', 'fp64') if variants else ('mixed',)):
        log('batch64: %s, default launch shapes' % precision)
        ctxs = contexts(precision)
        ms, bad, Qs = run(ctxs)
        e = entry(ms, bad)
        finals[precision] = Qs
        if variants:
            log('batch64: %s, autotuning on the largest problem' % precision)
            best, _ = autotune.tune(ctxs[big], Q0s[big], 'hybrid', steps=3, use_cache=False)
            for cx in ctxs:
                autotune.apply(cx, best)
            tms, tbad, _ = run(ctxs)
            e['autotuned'] = dict(entry(tms, tbad), **best)
        for cx in ctxs:
            cx.close()
        torch.cuda.empty_cache()
        res[precision] = e
    if 'fp64' in finals:   # FP32 bulk against FP64 after the same 2 x nsteps steps, over all problems
        errs = [precision_error(a, b) for a, b in zip(finals['mixed'], finals['fp64'])]
        w = np.array([c.cells for c in probs], float)
        res['fp32_vs_fp64_after_%d_steps' % (2 * nsteps)] = {
            k: {'L1_cell_weighted': float(np.sum(w * [e[k]['L1'] for e in errs]) / w.sum()),
                'Linf': float(max(e[k]['Linf'] for e in errs))} for k in ('rho', 'u', 'v', 'p')}
    del finals
    if variants:
        for vname, prec, mode, scheme in (('percell_mixed', 'mixed', 'percell', 'hybrid'),
                                          ('cgbr_meg6_mixed', 'mixed', 'global', 'cgbr'),
                                          ('cgbr_meg6_fp64', 'fp64', 'global', 'cgbr')):
            log('batch64: ' + vname)
            ctxs = contexts(prec, mode)
            ms, bad, _ = run(ctxs, scheme)
            res[vname] = entry(ms, bad)
            for cx in ctxs:
                cx.close()
            torch.cuda.empty_cache()
    # the batch's throughput is reported only from a row in which every problem stayed physical
    res['value'] = res['mixed']['mcell_per_s'] if res['mixed']['valid'] else None
    res['ms_per_step'] = res['mixed']['ms_per_step']
    if cpu:
        res['cpu_baseline'] = cpu['batch64']
    return res


WORKLOADS = {'ramp3d': ramp3d, 'triple_point': triple_point, 'batch64': batch64}


# ------------------------------------------------------------------ rocprofv3 summaries
LIB_SOURCES = ['paper_2511_18042_amd/csrc/' + f for f in ('k_basic.hip', 'k_compact.hip', 'k_grad.hip', 'k_inflow.hip',
                                                          'k_lad.hip', 'k_sweep.hip', 'lgbr.cpp', 'lgbr_dev.h',
                                                          'lgbr_kernels.h')] + ['include/lgbr.h']


def kernel_class(name):
    """The library's kernel class (lg_prof_* classes; k_sweep_s serves eta and zeta) of a
    kernel name as rocprofv3 prints it, or None for kernels outside the library."""
    import re
    base = name.split('(')[0].replace('void ', '').strip()
    if not base.startswith('lg::'):
        return None
    k = base[4:]
    m = re.match(r'k_line_tiles<\w+, (\d)', k)
    if m:
        return {0: 'grad_c4', 1: 'c6_faces', 2: 'filter', 3: 'grad_c4'}[int(m.group(1))]
    table = [('k_bc_cons', 'bc'), ('k_fixed_ghosts', 'combine'), ('k_stage_ghosts', 'combine'), ('k_prim', 'prim'),
             ('k_zero_any', 'flags'), ('k_any_flag', 'flags'), ('k_all_flag', 'flags'), ('k_switch_count', 'flags'),
             ('k_dilate', 'flags'), ('k_line_list', 'flags'), ('k_hyb_queue', 'flags'),
             ('k_grad_explicit', 'grad_e6'), ('k_grad_c4', 'grad_c4'), ('k_grad_c6', 'grad_c4'),
             ('k_grad_part', 'grad_c4'), ('k_c6_seg_check', 'combine'), ('k_rk4_combine', 'combine'),
             ('k_gbr_queue', 'flags'),
             ('k_sensor', 'sensor'), ('k_gbr_viscflux', 'visc'), ('k_lad_shear', 'lad_node'),
             ('k_lad_raw', 'lad_raw'), ('k_gauss', 'gauss'), ('k_lad_nodeflux', 'lad_flux'),
             ('k_sweep_x', 'sweep_x'), ('k_sweep_s', 'sweep_yz'), ('k_dt_', 'dt'), ('k_lad_sweep', 'lad_sweep'),
             ('k_c6_faces', 'c6_faces'), ('k_filter_save', 'filter_guard'), ('k_filter_guard', 'filter_guard'),
             ('k_filter', 'filter'), ('k_gbr_items', 'gbr_items'), ('k_hyb_assemble', 'hyb_assemble'),
             ('k_bc_scalar', 'bc_scalar')]
    for pre, cls in table:
        if k.startswith(pre):
            return cls
    return None


def _dispatches(path, counter=False):
    """(kernel name, duration ns, counter value or None) per dispatch of a rocprofv3 csv."""
    import csv
    out = []
    for r in csv.DictReader(open(path)):
        dur = int(r['End_Timestamp']) - int(r['Start_Timestamp'])
        out.append((r['Kernel_Name'], dur, float(r['Counter_Value']) if counter else None))
    return out


def _executed(disp):
    """Per kernel name: the dispatches that did work (at least EXECUTED_FRACTION of that
    kernel's longest), the others being immediate returns of the hybrid switch."""
    by = {}
    for name, dur, val in disp:
        by.setdefault(name, []).append((dur, val))
    out = {}
    for name, v in by.items():
        top = max(d for d, _ in v)
        out[name] = ([x for x in v if x[0] >= EXECUTED_FRACTION * top], len(v))
    return out


def profile_summary(a):
    """Per-kernel and per-class summary of a kernel trace (and optionally FETCH_SIZE /
    WRITE_SIZE counter runs of the same workload), with machine-readable KTIME / TRAFFIC
    lines that bench.py reads while the library sources hash to what was profiled."""
    import hashlib
    h = hashlib.sha256()
    for src in LIB_SOURCES:
        h.update(open(os.path.join(ROOT, src), 'rb').read())
    sha = h.hexdigest()
    lines = ['# ' + a.title, '# commands:'] + ['#   ' + c.strip() for c in a.commands.split(';') if c.strip()]
    lines.append('# a dispatch shorter than %g of its kernel\'s longest is an immediate return of the device-side '
                 'hybrid switch ("skipped"); averages are over the executed dispatches' % EXECUTED_FRACTION)
    ex = _executed(_dispatches(a.trace))
    rows = []
    for name, (run, n) in ex.items():
        cls = kernel_class(name)
        if cls is None:
            continue
        tot = sum(d for d, _ in run)
        rows.append((tot, name.split('(')[0].replace('void ', ''), cls, n, len(run), tot / max(len(run), 1)))
    rows.sort(reverse=True)
    lines.append('%-44s %-12s %8s %8s %12s %12s' % ('kernel', 'class', 'calls', 'executed', 'avg exec us',
                                                    'total ms'))
    for tot, nm, cls, n, ne, avg in rows:
        lines.append('%-44s %-12s %8d %8d %12.1f %12.3f' % (nm[:44], cls, n, ne, avg / 1e3, tot / 1e6))
    cls_t = {}
    for tot, nm, cls, n, ne, avg in rows:
        a0 = cls_t.get(cls, (0, 0))
        cls_t[cls] = (a0[0] + tot, a0[1] + ne)
    lines.append('# per class (executed dispatches)')
    for cls, (tot, ne) in sorted(cls_t.items(), key=lambda kv: -kv[1][0]):
        lines.append('KTIME %s avg_ms=%.5f launches=%d' % (cls, tot / ne / 1e6, ne))
    if a.fetch and a.write:
        cal = {}
        per = {}
        for kind, path in (('fetch', a.fetch), ('write', a.write)):
            disp = _dispatches(path, counter=True)
            for name, dur, val in disp:   # the probe copy is the run's first large copy
                if name.startswith('__amd_rocclr_copyBuffer') and val > 1e5 and kind not in cal:
                    cal[kind] = val
            for name, (run, n) in _executed(disp).items():
                cls = kernel_class(name)
                if cls is None:
                    continue
                p = per.setdefault(cls, {'fetch': [0.0, 0], 'write': [0.0, 0]})
                p[kind][0] += sum(v for _, v in run)
                p[kind][1] += len(run)
        copy_kib = float(a.copy_kib)
        fs = copy_kib / cal['fetch'] if 'fetch' in cal else 1.0
        ws = copy_kib / cal['write'] if 'write' in cal else 1.0
        lines.append('# HBM counters: FETCH_SIZE and WRITE_SIZE in KiB per executed dispatch; a plain copy of %d KiB '
                     'reads FETCH_SIZE %.0f and WRITE_SIZE %.0f: scales %.4f (fetch), %.4f (write)'
                     % (copy_kib, cal.get('fetch', 0), cal.get('write', 0), fs, ws))
        for cls, p in sorted(per.items()):
            fk = p['fetch'][0] / max(p['fetch'][1], 1)
            wk = p['write'][0] / max(p['write'][1], 1)
            lines.append('TRAFFIC %s fetch_kib=%.0f write_kib=%.0f fetch_scale=%.4f write_scale=%.4f bytes=%.0f '
                         'sha256=%s' % (cls, fk, wk, fs, ws, (fk * fs + wk * ws) * 1024, sha))
    lines.append('SOURCES sha256=%s files=%s' % (sha, ','.join(LIB_SOURCES)))
    with open(a.profile_summary, 'w') as f:
        f.write('\n'.join(lines) + '\n')
    print('\n'.join(lines))


def main():
    args = parse()
    if args.profile_summary:
        args.copy_kib = args.copy_probe_mib * 1024 if args.copy_probe_mib else 1048576
        profile_summary(args)
        return
    if args.gpus != 1:
        print('bench.py: the benchmark runs on one GPU only (one process, one MI355X); '
              '--gpus %d is not supported' % args.gpus, file=sys.stderr)
        sys.exit(2)
    names = list(WORKLOADS) if args.workload == 'all' else [args.workload]
    # the oracle runs on the host cores first, before this process touches the GPU
    cpu = cpu_baselines(names) if not args.no_cpu_baseline else None
    import torch
    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        a = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device='cuda')
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
    results = {}
    for nm in names:
        results[nm] = WORKLOADS[nm](args, args.variants == 'all', cpu)
        torch.cuda.empty_cache()
    head = results[names[0]]
    out = {
        'metric': 'Mcell-updates/s per RK3 step (hybrid vs C-GBR, FP32 vs FP64) and % HBM peak',
        'value': head.get('value'),
        'unit': 'Mcell-updates/s',
        'n_gpus': 1,
        'steps': args.steps,
        'warmup': args.warmup,
        'ms_per_step': head.get('ms_per_step'),
        'higher_is_better': True,
        'scaling': 'weak',
        'vs_baseline': None,
        'dtype': 'f32 (f64 state, RK combination, compact solves and flux differences)',
        'data': 'synthetic: seeded generator states',
        'config': {'workload': head['workload'], 'cells': head['cells'], 'parallelism': 'single GPU'},
        'roofline': head.get('roofline'),
        'roofline_step_floor': head.get('roofline_step_floor'),
        'hbm_step': head.get('hbm_step'),
        'cpu_baseline': head.get('cpu_baseline'),
        'nonphysical_nodes': head.get('nonphysical_nodes'),
        'workloads': results,
    }
    print(json.dumps(out))


if __name__ == '__main__':
    main()
