"""The kernels' default code forms against their fallbacks.

The defaults are 32-bit offsets from scalar bases in the FP32 LAD sweep and node fluxes, two
nodes per lane in the primitive conversion, and forms of the LAD coefficient kernel (FP32),
node-flux kernel (FP64) and C-GBR direction sweeps (viscous problems) compiled for 3D
curvilinear grids with metrics planar along zeta. The kernels fall back by themselves to
64-bit addressing, one node per lane and the general form for fields of 2^32 bytes or more,
odd node counts, unaligned state, other grids or inviscid problems, and
lg_set_generic_access forces those fallbacks (bit 0 addressing, bit 1 geometry).
On the compression-ramp crop (3D, curvilinear, extruded along zeta) right-hand sides and
RK3 steps must be bitwise equal across the addressing forms, and across the geometry forms
in FP64; the FP32 geometry forms differ by rounding only (the compiler fuses and orders the
arithmetic of the two differently): right-hand sides within 1e-5 of each variable's largest
value, states after three steps within 1e-7 of it and the time within 1e-7 of itself
(measured: 1e-6, 7e-9 and 1.5e-9; the FP32 bulk itself moves the state by about 1e-5 from
the FP64 path)."""
import numpy as np
import pytest

import gpu_util as U
from oracle import rhs as orhs
from paper_2511_18042_amd import cases

pytestmark = pytest.mark.gpu


def _ramp():
    c = cases.ramp3d(40, 32, 16)
    e = c.extra
    gas = orhs.Gas(gamma=1.4, Re=e['Re'], Pr=e['Pr'], Mref=e['Mref'], suth=e['suth'], viscous=True)
    return c, gas, orhs.Opts(grad='C4', p_thr=e['p_thr'])


def _run(c, gas, opts, precision, scheme, generic):
    torch = U.torch_mod()
    ctx, _ = U.gpu_context(c, gas, opts, precision=precision)
    for g in generic:
        ctx.set_generic_access(g)
    rhs = U.gpu_rhs(ctx, c, scheme)
    Qd = U.dev(c.Q)
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    for _ in range(3):
        ctx.rk3_step(scheme, Qd, 10.0, t)
    torch.cuda.synchronize()
    ctx.close()
    return rhs, Qd.cpu().numpy(), float(t.item())


def _rel(a, b):
    """Largest difference per variable over that variable's largest value."""
    d = np.abs(a - b).reshape(a.shape[0], -1).max(axis=1)
    return d / np.abs(b).reshape(b.shape[0], -1).max(axis=1)


@pytest.mark.parametrize('precision', ['mixed', 'fp64'])
@pytest.mark.parametrize('scheme', ['lad', 'hybrid'])
def test_generic_access_matches_default(precision, scheme):
    print('access forms', precision, scheme, flush=True)
    c, gas, opts = _ramp()
    r0, q0, t0 = _run(c, gas, opts, precision, scheme, [])
    r1, q1, t1 = _run(c, gas, opts, precision, scheme, [2, 3])     # general geometry; then every fallback
    r2, q2, t2 = _run(c, gas, opts, precision, scheme, [3, 2])     # general geometry, default addressing
    r3, q3, t3 = _run(c, gas, opts, precision, scheme, [3, False])  # back to the defaults
    # addressing forms: bitwise
    assert np.array_equal(r1, r2) and np.array_equal(q1, q2) and t1 == t2
    assert np.array_equal(r0, r3) and np.array_equal(q0, q3) and t0 == t3 > 0.0
    # geometry forms
    if precision == 'fp64':
        assert np.array_equal(r0, r1) and np.array_equal(q0, q1) and t0 == t1
    else:
        er, eq = _rel(r0, r1), _rel(q0, q1)
        print('geometry forms: rhs', er.tolist(), 'state', eq.tolist(), flush=True)
        assert er.max() <= 1e-5 and eq.max() <= 1e-7
        assert abs(t0 - t1) <= 1e-7 * t0


def test_generic_access_argument_check():
    c, gas, opts = _ramp()
    ctx, _ = U.gpu_context(c, gas, opts, precision='mixed')
    assert ctx._lib.lg_set_generic_access(ctx.handle, 4) != 0
    assert ctx._lib.lg_set_generic_access(ctx.handle, -1) != 0
    assert ctx._lib.lg_set_generic_access(None, 1) != 0
    ctx.close()
