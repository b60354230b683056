"""Switching statistics of the global hybrid (Sec. 5): the share of the run spent on LAD and
on C-GBR, the switches between them, and the step time against the C-GBR (MEG6) solver,
on the GPU, for the two cases the paper reports:

  * the triple point (1792 x 768, MEG6 / LAD-E4, troubled where rho < 0.0625, FP64) until
    t = 5, the first non-physical stage, or the wall-time cap (paper: LAD 13.6 % of the run);
  * the M2.9 ramp stand-in (1024 x 384 x 128, MIG4 / LAD-E4, troubled where p < p_inf / 2,
    FP32 bulk) for a fixed number of steps, with the adiabatic wall of the headline workload,
    with the isothermal wall at 1.14 T_aw, and with that wall and the digital-filter inflow
    (a new time-correlated plane before every step, cases.ramp_df_inflow), and at half the
    resolution in every direction for one whole flow-through (paper: LAD 82.4 % of one
    flow-through, 1.67x faster than MEG6 C-GBR).

Every RK3 step reads the context's switching record (lg_switch_stats: hybrid stages and
those with a troubled node).  A step counts as LAD or C-GBR by its stages; a step whose
stages differ contains a switch.

    python tests/switching_runs.py [--out FILE] [--cases NAME ...] [--wall SECONDS] [--ramp-steps N]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2511_18042_amd import cases, lgbr  # noqa: E402


def _triple_point():
    c = cases.triple_point(1792, 768)
    gas = lgbr.make_gas(gamma=c.gamma)
    grid = lgbr.make_grid(2, c.n, c.bc, c.h)
    opts = dict(grad='E6', precision='fp64', rho_thr=c.extra['rho_thr'], p_thr=c.extra['p_thr'])
    return c, gas, grid, opts, None, None, None


def _ramp(wall, df=False, half=False, precision='mixed'):
    import torch
    # half: every spacing doubled (512 x 192 x 64, first cell at 0.004 delta), run for one
    # flow-through (t = Lx / U = 26.2) instead of a fixed number of steps
    c = cases.ramp3d(512, 192, 64, y1=0.004, wall=wall) if half else cases.ramp3d(wall=wall)
    inflow = cases.ramp_df_inflow(c) if df else None
    e = c.extra
    gas = lgbr.make_gas(gamma=1.4, Re=e['Re'], Pr=e['Pr'], Mref=e['Mref'], suth=e['suth'], viscous=True)
    grid = lgbr.make_grid(3, c.n, c.bc, c.h, curvilinear=True, wall_T=c.wall_T)
    coords = torch.from_numpy(c.coords).cuda()
    metrics = torch.zeros((10,) + tuple(c.shape), dtype=torch.float64, device='cuda')
    lgbr.metrics_from_coords(grid, coords, metrics)
    c.coords = None
    opts = dict(grad='C4', precision=precision, rho_thr=-1.0, p_thr=e['p_thr'])
    c.extra['df_inflow'] = inflow
    return c, gas, grid, opts, metrics, coords, 26.2 if half else 1e30


CASES = {
    'triple_point': (_triple_point, 'MEG6 / LAD-E4, FP64', 13.6),
    'ramp_adiabatic': (lambda: _ramp('adiabatic'), 'MIG4 / LAD-E4, FP32 bulk, adiabatic wall', 82.4),
    'ramp_isothermal': (lambda: _ramp('isothermal'), 'MIG4 / LAD-E4, FP32 bulk, wall at 1.14 T_aw', 82.4),
    'ramp_isothermal_df': (lambda: _ramp('isothermal', df=True),
                           'MIG4 / LAD-E4, FP32 bulk, wall at 1.14 T_aw, digital-filter inflow', 82.4),
    'ramp_half_flowthrough': (lambda: _ramp('adiabatic', half=True),
                              'MIG4 / LAD-E4, FP32 bulk, adiabatic wall, 512 x 192 x 64, one flow-through', 82.4),
    'ramp_half_flowthrough_fp64': (lambda: _ramp('adiabatic', half=True, precision='fp64'),
                                   'MIG4 / LAD-E4, FP64, adiabatic wall, 512 x 192 x 64, one flow-through', 82.4),
}


def _step_time(ctx, scheme, Q0, steps=10):
    import torch
    Q = Q0.clone()
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    ctx.rk3_step(scheme, Q, 1e30, t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.rk3_step(scheme, Q, 1e30, t)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def run(name, wall=120.0, ramp_steps=2000):
    import torch
    build, desc, paper_lad = CASES[name]
    c, gas, grid, o, metrics, coords, t_end = build()
    t_end = c.t_end if t_end is None else t_end
    max_steps = ramp_steps if name.startswith('ramp') and 'flowthrough' not in name else 10 ** 7
    ctx = lgbr.Context(grid, gas, lgbr.make_opts(cfl=0.2, hybrid_mode='global', **o), metrics, coords)
    Q0 = torch.from_numpy(np.ascontiguousarray(c.Q)).cuda()
    Q = Q0.clone()
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    per_step = []
    status, bad, steps = 'steps', 0, 0
    df = None
    if (c.extra or {}).get('df_inflow') is not None:
        df = lgbr.DFInflow(ctx, **c.extra['df_inflow'])
        gen = torch.Generator(device='cuda')
        gen.manual_seed(18042)
        count = df.random_count()
    t0 = time.perf_counter()
    while True:
        if df is not None:   # a new inflow plane for the step (time-correlated with the last)
            df.update(torch.randn(count, generator=gen, dtype=torch.float64, device='cuda'), Q, dt=-1.0,
                      first=steps == 0)
        ctx.rk3_step('hybrid', Q, t_end, t)
        n_st, n_tr = ctx.switch_stats(reset=True)
        per_step.append(n_tr)
        steps += 1
        if steps % 10 == 0:
            bad = ctx.poll_status()
        tv = float(t.item())
        if bad:
            status = 'diverged'
            break
        if tv >= t_end:
            status = 'reached t_end'
            break
        if steps >= max_steps:
            break
        if time.perf_counter() - t0 > wall:
            status = 'wall-time cap'
            break
        if steps % 200 == 0:
            print('[switching] %s step %d t %.5g troubled stages so far %d' % (name, steps, tv, sum(per_step)),
                  flush=True)
    secs = time.perf_counter() - t0
    tr = np.array(per_step)
    stages = 3 * len(tr)
    gbr = int(tr.sum())
    mode = np.where(tr == 0, 0, np.where(tr == 3, 1, -1))        # 0 LAD, 1 C-GBR, -1 mixed step
    switches = int((mode == -1).sum()) + int(np.sum((mode[1:] != mode[:-1]) & (mode[1:] >= 0) & (mode[:-1] >= 0)))
    first_gbr = int(np.argmax(tr > 0)) if gbr else None
    hyb_ms = _step_time(ctx, 'hybrid', Q0)
    if df is not None:
        df.close()
    ctx.close()
    ctx = lgbr.Context(grid, gas, lgbr.make_opts(cfl=0.2, hybrid_mode='global', **dict(o, grad='E6')), metrics, coords)
    meg6_ms = _step_time(ctx, 'cgbr', Q0)
    ctx.close()
    res = {'case': name, 'scheme': desc, 'status': status, 'steps': steps, 't': round(tv, 6),
           'lad_share_pct': round(100.0 * (stages - gbr) / stages, 2), 'paper_lad_share_pct': paper_lad,
           'gbr_stages': gbr, 'stages': stages, 'switches_at_step_granularity': switches,
           'first_gbr_step': first_gbr, 'seconds': round(secs, 1),
           'ms_per_step_hybrid_lad_phase': round(hyb_ms, 3), 'ms_per_step_meg6_cgbr': round(meg6_ms, 3),
           'run_ms_per_step': round(secs / steps * 1e3, 3),
           'history_troubled_stages_per_step': ''.join(str(int(v)) for v in tr)}
    return res


def markdown(rows):
    out = ['| case | scheme | run | LAD share | paper | switches | C-GBR stages | ms/step hybrid (start) | ms/step MEG6 |',
           '|---|---|---|---|---|---|---|---|---|']
    for r in rows:
        out.append('| %s | %s | %s, %d steps, t %.4g | %.1f %% | %.1f %% | %d | %d of %d | %.2f | %.2f |' % (
            r['case'], r['scheme'], r['status'], r['steps'], r['t'], r['lad_share_pct'], r['paper_lad_share_pct'],
            r['switches_at_step_granularity'], r['gbr_stages'], r['stages'], r['ms_per_step_hybrid_lad_phase'],
            r['ms_per_step_meg6_cgbr']))
    return '\n'.join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--out', default=None)
    ap.add_argument('--cases', nargs='*', default=list(CASES))
    ap.add_argument('--wall', type=float, default=120.0)
    ap.add_argument('--ramp-steps', type=int, default=2000)
    a = ap.parse_args()
    rows = []
    for name in a.cases:
        r = run(name, a.wall, a.ramp_steps)
        print('SWITCHING ' + json.dumps({k: v for k, v in r.items() if k != 'history_troubled_stages_per_step'}),
              flush=True)
        rows.append(r)
    print(markdown(rows))
    if a.out:
        with open(a.out, 'w') as f:
            json.dump(rows, f, indent=1)
            f.write('\n')


if __name__ == '__main__':
    main()
