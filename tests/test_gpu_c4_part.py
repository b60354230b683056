"""MIG4 gradients along xi by the partition method (k_grad_c4_part: bounded lines of 130 to
2050 nodes, the two decoupled end rows moved to the right-hand side of the [1/4, 1, 1/4]
system of the others; segments per lane joined through their end unknowns), and along eta /
zeta in register segments (k_grad_c4_seg: bounded lines of 16 to 512 unknowns between the
end rows, periodic lines of 16 to 512 interior nodes with their ghost images), against the
oracle's banded and cyclic solves, through C-GBR right-hand sides (FP64, the RHS tolerance of
the other parity tests), beside the kernels they replace (LDS line tiles: mask bit 13;
PCR / one lane per line: mask bit 14).

Cases: the shortest line it takes (120 interior nodes: 128 unknowns, two per segment), 300
nodes with reflective and transmissive walls, 1030 nodes with a FIXED inflow face (segments
of 16 and 17 unknowns), 2040 nodes in 1D (the longest register arrays, segments of 32), and a
periodic line of 200 nodes, which stays on the cyclic solvers; along eta / zeta, lines of
one to eight segments, a FIXED face, and periodic zeta lines of 16 and 128 nodes."""
import numpy as np
import pytest

import gpu_util as U
from oracle import rhs as orhs
from paper_2511_18042_amd import cases

pytestmark = pytest.mark.gpu

T, P, RF, FX = cases.TRANSMISSIVE, cases.PERIODIC, cases.REFLECTIVE, cases.FIXED
NO_PART = 0xFFF | 0x2000


def _case(ndim, n, bc, seed):
    h = tuple(1.0 / m if m > 1 else 1.0 for m in n)
    c = cases.Case(ndim, n, bc, h=h)
    return cases.random_rough_state(c, seed=seed)


CASES = {
    'x120': lambda: _case(2, (120, 10, 1), [(T, T), (RF, T)], 21),
    'x300_walls': lambda: _case(2, (300, 12, 1), [(RF, T), (T, RF)], 22),
    'x1030_fixed': lambda: _case(2, (1030, 6, 1), [(FX, T), (T, T)], 23),
    'x2040_1d': lambda: _case(1, (2040, 1, 1), [(T, RF)], 24),
    'x200_periodic': lambda: _case(2, (200, 8, 1), [(P, P), (T, T)], 25),
}


@pytest.mark.parametrize('name', list(CASES))
def test_c4_partition_parity_fp64(name):
    print('c4 partition', name, flush=True)
    c = CASES[name]()
    gas = orhs.Gas(gamma=c.gamma)
    opts = orhs.Opts(grad='C4')
    g = U.oracle_grid(c)
    info = {}
    ref = orhs.rhs(c.Q, g, gas, opts, 'cgbr', info=info)
    outs = []
    for mask in (-1, NO_PART):
        ctx, _ = U.gpu_context(c, gas, opts)
        ctx.set_line_tiles(mask)
        out = U.gpu_rhs(ctx, c, 'cgbr')
        ctx.close()
        U.compare(out, ref, g, U.RHS_RTOL, U.excused_mask(info, g), label='c4 part %s mask %d' % (name, mask))
        outs.append(out)
    inner = (slice(None),) + g.interior()
    a, b = outs[0][inner], outs[1][inner]
    # per variable, relative to its largest value (or to the largest of all five where it
    # vanishes, as the out-of-plane momentum of a 2D case does)
    scale = np.abs(b).reshape(5, -1).max(axis=1)
    scale = np.where(scale > 0, scale, scale.max())
    rel = np.abs(a - b).reshape(5, -1).max(axis=1) / scale
    print('partition vs tiles', rel.tolist(), flush=True)
    assert rel.max() <= 1e-11
    if name == 'x200_periodic':
        assert np.array_equal(a, b)   # periodic lines never take the partition method


# --- strided directions: register segments joined through their end unknowns (k_grad_c4_seg)
SEG_ON = 0xFFF & ~((1 << 10) | (1 << 11))   # no LDS tiles for the MIG4 gradients along eta / zeta
SEG_OFF = SEG_ON | 0x4000                   # ... and no segment kernel: PCR or one lane per line

STRIDED = {
    'eta384_walls': lambda: _case(2, (12, 384, 1), [(T, T), (RF, T)], 31),           # 392 unknowns, 7 segments
    'eta130_fixed': lambda: _case(2, (16, 130, 1), [(T, T), (FX, T)], 32),           # 138 unknowns, 3 segments
    'eta504': lambda: _case(2, (8, 504, 1), [(T, RF), (T, T)], 33),                  # 512 unknowns, 8 segments
    'eta70_zeta128': lambda: _case(3, (12, 70, 128), [(T, T), (RF, T), (P, P)], 34),  # 78 bounded; 128 cyclic
    'eta8_zeta16': lambda: _case(3, (12, 8, 16), [(T, T), (T, T), (P, P)], 35),       # one segment each
}


@pytest.mark.parametrize('name', list(STRIDED))
def test_c4_strided_segments_parity_fp64(name):
    print('c4 segments', name, flush=True)
    c = STRIDED[name]()
    gas = orhs.Gas(gamma=c.gamma)
    opts = orhs.Opts(grad='C4')
    g = U.oracle_grid(c)
    info = {}
    ref = orhs.rhs(c.Q, g, gas, opts, 'cgbr', info=info)
    outs = []
    for mask in (-1, SEG_ON, SEG_OFF):
        ctx, _ = U.gpu_context(c, gas, opts)
        ctx.set_line_tiles(mask)
        out = U.gpu_rhs(ctx, c, 'cgbr')
        ctx.close()
        U.compare(out, ref, g, U.RHS_RTOL, U.excused_mask(info, g), label='c4 seg %s mask %d' % (name, mask))
        outs.append(out)
    inner = (slice(None),) + g.interior()
    a, b = outs[1][inner], outs[2][inner]
    scale = np.abs(b).reshape(5, -1).max(axis=1)
    scale = np.where(scale > 0, scale, scale.max())
    rel = np.abs(a - b).reshape(5, -1).max(axis=1) / scale
    print('segments vs one lane per line', rel.tolist(), flush=True)
    assert rel.max() <= 1e-11
