"""Launch-shape autotuner for liblgbr (results never depend on the tuning).

Times whole RK3 steps of a context through the C ABI over the launch-shape knobs -- planes
per chunk of the z-marching stencil kernels, nodes per lane of the strided sweeps and the
persistent PCR grid (compact gradients only) -- one knob at a time with the others at their
best so far, keeps the fastest setting and caches it in a JSON file keyed by device, grid,
precision, gradient kind and scheme.  Tuning runs on a scratch copy of the state.
"""
import json
import os

CANDIDATE_ZC = (0, 8, 16, 32)
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
    """Pick (zc, seg, pcr_blocks) for ``ctx`` by timing ``steps`` RK3 steps per candidate on a
    copy of the device state Q0; applies and returns the winner and the timings (ms/step)."""
    import torch
    key = _key(ctx, scheme)
    cache = load_cache() if use_cache else {}
    if key in cache:
        e = cache[key]
        best = (e['zc'], e['seg'], e['pcr_blocks'])
        ctx.set_tuning(best[1], best[2], best[0])
        return best, e.get('timings', {})
    timings = {}

    def measure(zc, seg, pcr):
        name = '%d,%d,%d' % (zc, seg, pcr)
        if name in timings:
            return timings[name]
        ctx.set_tuning(seg, pcr, zc)
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
        del Q
        timings[name] = e0.elapsed_time(e1) / steps
        return timings[name]

    best = [0, 0, 0]
    for slot, cands in ((0, CANDIDATE_ZC), (1, CANDIDATE_SEG), (2, CANDIDATE_PCR if ctx.opts.grad == 1 else (0,))):
        scores = {}
        for v in cands:
            trial = list(best)
            trial[slot] = v
            scores[v] = measure(*trial)
        best[slot] = min(scores, key=scores.get)
    zc, seg, pcr = best
    ctx.set_tuning(seg, pcr, zc)
    ctx.poll_status()
    if use_cache:
        cache[key] = {'zc': zc, 'seg': seg, 'pcr_blocks': pcr, 'timings': timings}
        save_cache(cache)
    return (zc, seg, pcr), timings
