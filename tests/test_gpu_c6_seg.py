"""LAD-C6 interface fluxes along eta / zeta in register segments (k_c6_faces_seg: the n - 1
interior faces of a bounded line, or the n faces of a periodic line, 16 to 256 of them; 64
lines per workgroup, one wave per segment of at most 64 faces, the segments joined through
the LU of their end faces; in the last direction of an RK stage the stage combination in
the same pass and the non-physical count in its own),
against the oracle's banded and cyclic solves, through LAD-C6 right-hand sides and RK3
steps (FP64, the tolerances of the other parity tests), beside the lane-per-line kernel it
replaces (mask bit 14).  The LDS tiles, which small grids take, are turned off for the
faces along eta and zeta.

Cases: one segment (44 faces), three with a FIXED face, four (250 faces, and 256: the
longest line), periodic lines of 16 (one segment wrapping onto itself) and 200 faces, a 3D
curvilinear block with bounded eta and periodic zeta lines of 17 faces, and lines of 15 and
299 faces, which stay on the lane-per-line kernel.  The LAD-C6 gradients of periodic lines
of 16 to 256 nodes take the same register segments (the cyclic [1/3, 1, 1/3] system); they
are checked the same way, with the tiles of the gradients turned off too."""
import numpy as np
import pytest

import gpu_util as U
from oracle import grid as ogrid, rhs as orhs
from paper_2511_18042_amd import cases

pytestmark = pytest.mark.gpu

T, P, RF, NS, FX = cases.TRANSMISSIVE, cases.PERIODIC, cases.REFLECTIVE, cases.NOSLIP, cases.FIXED
SEG_ON = 0xFFF & ~((1 << 4) | (1 << 5))   # no LDS tiles for the faces along eta / zeta
SEG_OFF = SEG_ON | 0x4000                 # ... and no segment kernel: one lane per line


def _case(n, bc, seed, hx=0.04):
    c = cases.Case(2, n, bc, h=(hx / n[0], 1.0 / n[1], 1))
    return cases.random_rough_state(c, seed=seed)


def _curv3d():
    c = cases.periodic_case(3, (20, 18, 17), curvilinear=True, amp=0.05)
    c.bc = [(P, P), (NS, T), (P, P)]
    return cases.random_rough_state(c, seed=56)


CASES = {
    'y45_walls': lambda: _case((67, 45, 1), [(RF, T), (T, RF)], 51, hx=1.5),
    'y130_fixed': lambda: _case((10, 130, 1), [(T, T), (FX, T)], 52),
    'y251': lambda: _case((12, 251, 1), [(T, T), (RF, T)], 53),
    'y257': lambda: _case((6, 257, 1), [(T, T), (T, RF)], 54),
    'y16_periodic': lambda: _case((12, 16, 1), [(T, T), (P, P)], 55, hx=0.75),
    'y200_periodic': lambda: _case((10, 200, 1), [(T, T), (P, P)], 57),
    '3d_curv': _curv3d,
    'y16_bounded': lambda: _case((12, 16, 1), [(T, T), (RF, T)], 58, hx=0.75),
    'y300': lambda: _case((12, 300, 1), [(T, T), (RF, T)], 59),
}
UNCHANGED = ('y16_bounded', 'y300')   # 15 and 299 faces: one lane per line


def _gas(c):
    if c.ndim == 3:
        return orhs.Gas(gamma=1.4, viscous=True, Re=300.0, Mref=0.8, Pr=0.72)
    return orhs.Gas(gamma=c.gamma)


def _opts():
    return orhs.Opts(lad='C6', filter_alpha=0.49, C_mu=0.002)


def _rel(a, b):
    scale = np.abs(b).reshape(5, -1).max(axis=1)
    scale = np.where(scale > 0, scale, scale.max())
    return np.abs(a - b).reshape(5, -1).max(axis=1) / scale


@pytest.mark.parametrize('name', list(CASES))
def test_c6_face_segments_rhs_fp64(name):
    print('c6 face segments rhs', name, flush=True)
    c = CASES[name]()
    gas, opts = _gas(c), _opts()
    g = U.oracle_grid(c)
    ref = orhs.rhs(c.Q, g, gas, opts, 'lad')
    outs = []
    for mask in (SEG_ON, SEG_OFF):
        ctx, _ = U.gpu_context(c, gas, opts)
        ctx.set_line_tiles(mask)
        out = U.gpu_rhs(ctx, c, 'lad')
        ctx.close()
        U.compare(out, ref, g, U.RHS_RTOL, label='c6 face seg %s mask %#x' % (name, mask))
        outs.append(out)
    inner = (slice(None),) + g.interior()
    rel = _rel(outs[0][inner], outs[1][inner])
    print('segments vs one lane per line', rel.tolist(), flush=True)
    assert rel.max() <= 1e-11
    if name in UNCHANGED:
        assert np.array_equal(outs[0][inner], outs[1][inner])


@pytest.mark.parametrize('name', ['y45_walls', 'y130_fixed', 'y16_periodic', '3d_curv'])
def test_c6_face_segments_rk3_fp64(name):
    """Two RK3 steps: the last direction's segment solve and the stage combination after it."""
    print('c6 face segments rk3', name, flush=True)
    torch = U.torch_mod()
    c = CASES[name]()
    gas, opts = _gas(c), _opts()
    g = U.oracle_grid(c)
    M = ogrid.node_metrics(g)
    Q, t = c.Q, 0.0
    for _ in range(2):
        Q, t, dt, bad = orhs.rk3_step(Q, t, 10.0, g, gas, opts, 'lad', M)
        assert bad == 0
    outs = []
    for mask in (SEG_ON, SEG_OFF):
        ctx, _ = U.gpu_context(c, gas, opts)
        ctx.set_line_tiles(mask)
        Qd = U.dev(c.Q)
        td = torch.zeros(1, dtype=torch.float64, device='cuda')
        for _ in range(2):
            ctx.rk3_step('lad', Qd, 10.0, td)
        torch.cuda.synchronize()
        assert ctx.poll_status() == 0
        assert abs(td.item() - t) <= 1e-13 * t
        out = Qd.cpu().numpy()
        ctx.close()
        U.compare(out, Q, g, U.STAGE_RTOL, label='c6 face seg rk3 %s mask %#x' % (name, mask))
        outs.append(out)
    inner = (slice(None),) + g.interior()
    rel = _rel(outs[0][inner], outs[1][inner])
    print('rk3 segments vs one lane per line', rel.tolist(), flush=True)
    assert rel.max() <= 1e-12


def test_c6_face_segments_rk3_mixed():
    """FP32 bulk: the same two steps with and without the segment kernel."""
    torch = U.torch_mod()
    c = CASES['3d_curv']()
    gas, opts = _gas(c), _opts()
    g = U.oracle_grid(c)
    outs = []
    for mask in (SEG_ON, SEG_OFF):
        ctx, _ = U.gpu_context(c, gas, opts, precision='mixed')
        ctx.set_line_tiles(mask)
        Qd = U.dev(c.Q)
        td = torch.zeros(1, dtype=torch.float64, device='cuda')
        for _ in range(2):
            ctx.rk3_step('lad', Qd, 10.0, td)
        torch.cuda.synchronize()
        assert ctx.poll_status() == 0
        outs.append(Qd.cpu().numpy())
        ctx.close()
    inner = (slice(None),) + g.interior()
    rel = _rel(outs[0][inner], outs[1][inner])
    print('mixed rk3 segments vs one lane per line', rel.tolist(), flush=True)
    assert rel.max() <= 1e-5


# LAD-C6 gradients of periodic eta / zeta lines in register segments (k_grad_c4_seg with the
# cyclic [1/3, 1, 1/3] tables): no LDS tiles for the gradients and faces along eta / zeta
GSEG_ON = 0xFFF & ~((1 << 1) | (1 << 2) | (1 << 4) | (1 << 5))
GSEG_OFF = GSEG_ON | 0x4000


@pytest.mark.parametrize('name', ['y16_periodic', 'y200_periodic', '3d_curv', 'y300'])
def test_c6_gradient_segments_rhs_fp64(name):
    """Periodic lines of 16 (one segment wrapping onto itself), 200 (four) and 17 nodes (the
    3D block's zeta); the bounded 300-node line stays on one lane per line."""
    print('c6 gradient segments rhs', name, flush=True)
    c = CASES[name]()
    gas, opts = _gas(c), _opts()
    g = U.oracle_grid(c)
    ref = orhs.rhs(c.Q, g, gas, opts, 'lad')
    outs = []
    for mask in (GSEG_ON, GSEG_OFF):
        ctx, _ = U.gpu_context(c, gas, opts)
        ctx.set_line_tiles(mask)
        out = U.gpu_rhs(ctx, c, 'lad')
        ctx.close()
        U.compare(out, ref, g, U.RHS_RTOL, label='c6 gradient seg %s mask %#x' % (name, mask))
        outs.append(out)
    inner = (slice(None),) + g.interior()
    rel = _rel(outs[0][inner], outs[1][inner])
    print('gradient segments vs one lane per line', rel.tolist(), flush=True)
    assert rel.max() <= 1e-11


def test_c6_gradient_segments_rk3_fp64():
    """Two RK3 steps of the 3D block with the gradient and face segments (ghost images of
    the periodic zeta gradients included) against the oracle."""
    torch = U.torch_mod()
    c = CASES['3d_curv']()
    gas, opts = _gas(c), _opts()
    g = U.oracle_grid(c)
    M = ogrid.node_metrics(g)
    Q, t = c.Q, 0.0
    for _ in range(2):
        Q, t, dt, bad = orhs.rk3_step(Q, t, 10.0, g, gas, opts, 'lad', M)
        assert bad == 0
    ctx, _ = U.gpu_context(c, gas, opts)
    ctx.set_line_tiles(GSEG_ON)
    Qd = U.dev(c.Q)
    td = torch.zeros(1, dtype=torch.float64, device='cuda')
    for _ in range(2):
        ctx.rk3_step('lad', Qd, 10.0, td)
    torch.cuda.synchronize()
    assert ctx.poll_status() == 0
    assert abs(td.item() - t) <= 1e-13 * t
    U.compare(Qd.cpu().numpy(), Q, g, U.STAGE_RTOL, label='c6 gradient seg rk3')
    ctx.close()
