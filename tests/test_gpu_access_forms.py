"""The FP32 kernels' default memory-access forms against their fallbacks.

The defaults are 32-bit offsets from scalar bases in the LAD sweep and two nodes per lane in
the primitive conversion. The kernels fall back by themselves to 64-bit addressing and one
node per lane for fields of 2^32 bytes or more, odd node counts or unaligned state, and
lg_set_generic_access forces those fallbacks. Right-hand sides and RK3 steps on the
compression-ramp crop must then be bitwise equal, in both precisions."""
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


@pytest.mark.parametrize('precision', ['mixed', 'fp64'])
@pytest.mark.parametrize('scheme', ['lad', 'hybrid'])
def test_generic_access_matches_default(precision, scheme):
    print('access forms', precision, scheme, flush=True)
    c, gas, opts = _ramp()
    r0, q0, t0 = _run(c, gas, opts, precision, scheme, [])
    r1, q1, t1 = _run(c, gas, opts, precision, scheme, [True])
    r2, q2, t2 = _run(c, gas, opts, precision, scheme, [True, False])   # back to the default
    assert np.array_equal(r0, r1) and np.array_equal(r0, r2)
    assert np.array_equal(q0, q1) and np.array_equal(q0, q2)
    assert t0 == t1 == t2 > 0.0


def test_generic_access_argument_check():
    c, gas, opts = _ramp()
    ctx, _ = U.gpu_context(c, gas, opts, precision='mixed')
    assert ctx._lib.lg_set_generic_access(ctx.handle, 2) != 0
    assert ctx._lib.lg_set_generic_access(None, 1) != 0
    ctx.close()
