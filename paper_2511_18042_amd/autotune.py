"""Launch-shape autotuner for liblgbr (results never depend on the tuning).

Times whole RK3 steps of a context for each candidate (seg, pcr_blocks) pair through the C
ABI, keeps the fastest and caches it in a JSON file keyed by device, grid, precision,
gradient kind and scheme.  Tuning runs on a scratch copy of the state.
"""
import json
import os

CANDIDATE_SEG = (0, 4, 8, 16, 32)
CANDIDATE_PCR = (0, 4096, 32768)


def cache_path():
    return os.environ.get('LGBR_TUNE_CACHE', os.path.join(os.path.expanduser('~'), '.cache', 'lgbr_tune.json'))


def _key(ctx, scheme):
    import torch
    g = ctx.grid
    return '|'.join(str(v) for v in (torch.cuda.get_device_name(0), g.ndim, tuple(g.n), ctx.opts.precision,
                                      ctx.opts.grad, ctx.opts.hybrid_mode, scheme))


def load_cache():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + '.tmp'
    with open(tmp, 'w') as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def tune(ctx, Q0, scheme, steps=3, use_cache=True):
    """Pick (seg, pcr_blocks) for ``ctx`` by timing ``steps`` RK3 steps per candidate on a
    copy of the device state Q0; applies and returns the winner and the timings (ms/step)."""
    import torch
    key = _key(ctx, scheme)
    cache = load_cache() if use_cache else {}
    if key in cache:
        seg, pcr = cache[key]['seg'], cache[key]['pcr_blocks']
        ctx.set_tuning(seg, pcr)
        return (seg, pcr), cache[key].get('timings', {})
    grads = ctx.opts.grad == 1
    timings = {}
    for seg in CANDIDATE_SEG:
        for pcr in (CANDIDATE_PCR if grads else (0,)):
            ctx.set_tuning(seg, pcr)
            Q = Q0.clone()
            t = torch.zeros(1, dtype=torch.float64, device='cuda')
            ctx.rk3_step(scheme, Q, 1e30, t)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                ctx.rk3_step(scheme, Q, 1e30, t)
            e1.record()
            torch.cuda.synchronize()
            timings['%d,%d' % (seg, pcr)] = e0.elapsed_time(e1) / steps
            del Q
    best = min(timings, key=timings.get)
    seg, pcr = (int(v) for v in best.split(','))
    ctx.set_tuning(seg, pcr)
    ctx.poll_status()
    if use_cache:
        cache[key] = {'seg': seg, 'pcr_blocks': pcr, 'timings': timings}
        save_cache(cache)
    return (seg, pcr), timings
