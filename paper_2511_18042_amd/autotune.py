"""Launch-shape autotuner for liblgbr (results never depend on the tuning).

Times whole RK3 steps of a context through the C ABI over its launch-shape knobs -- the tile
shape of the z-marching stencil kernels (32 x 8, 64 x 4 or 128 x 2 columns), the planes per
chunk they walk, the nodes per lane of the strided sweeps, the lines per LDS line tile of the
compact solves and the persistent PCR grid (compact gradients only) -- one knob at a time
with the others at their best so far, keeps the fastest setting and caches it in a JSON file
keyed by the GPU architecture, grid, precision, gradient kind and scheme.  Tuning runs on a
scratch copy of the state.
"""
import json
import os

CANDIDATE_ZM_WIDTH = (64, 32, 128)
CANDIDATE_ZC = (0, 8, 16, 32)
CANDIDATE_SEG = (0, 4, 8, 16, 32)
CANDIDATE_LINE_BATCH = (0, 8, 4, 2)
CANDIDATE_PCR = (0, 4096, 32768)
KNOBS = ('zm_width', 'zc', 'seg', 'line_batch', 'pcr_blocks')


def cache_path():
    return os.environ.get('LGBR_TUNE_CACHE', os.path.join(os.path.expanduser('~'), '.cache', 'lgbr_tune.json'))


def _arch():
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, 'gcnArchName', None) or p.name


def _key(ctx, scheme):
    g = ctx.grid
    return '|'.join(str(v) for v in (_arch(), g.ndim, tuple(g.n), ctx.opts.precision, ctx.opts.grad,
                                      ctx.opts.hybrid_mode, ctx.opts.lad_scheme, scheme))


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


def apply(ctx, s):
    """Set the knobs of the dict ``s`` (keys KNOBS) on a context."""
    ctx.set_tuning(s['seg'], s['pcr_blocks'], s['zc'])
    ctx.set_tile_shape(s['zm_width'], s['line_batch'])


def tune(ctx, Q0, scheme, steps=3, use_cache=True):
    """Pick the launch shape of ``ctx`` by timing ``steps`` RK3 steps per candidate on a copy
    of the device state Q0; applies and returns the winner (dict over KNOBS) and the timings
    (ms per step, keyed by the candidate)."""
    import torch
    key = _key(ctx, scheme)
    cache = load_cache() if use_cache else {}
    if key in cache:
        best = {k: cache[key][k] for k in KNOBS}
        apply(ctx, best)
        return best, cache[key].get('timings', {})
    timings = {}

    def measure(s):
        name = ','.join('%s=%d' % (k, s[k]) for k in KNOBS)
        if name in timings:
            return timings[name]
        apply(ctx, s)
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

    best = {'zm_width': 64, 'zc': 0, 'seg': 0, 'line_batch': 0, 'pcr_blocks': 0}
    compact = ctx.opts.grad == 1 or ctx.opts.lad_scheme == 1 or ctx.opts.filter_alpha < 0.5
    for knob, cands in (('zm_width', CANDIDATE_ZM_WIDTH), ('zc', CANDIDATE_ZC), ('seg', CANDIDATE_SEG),
                        ('line_batch', CANDIDATE_LINE_BATCH if compact else (0,)),
                        ('pcr_blocks', CANDIDATE_PCR if ctx.opts.grad == 1 else (0,))):
        scores = {}
        for v in cands:
            trial = dict(best, **{knob: v})
            scores[v] = measure(trial)
        best[knob] = min(scores, key=scores.get)
    apply(ctx, best)
    ctx.poll_status()
    if use_cache:
        cache[key] = dict(best, timings=timings)
        save_cache(cache)
    return best, timings
