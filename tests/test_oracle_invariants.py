"""Whole-RHS pins of the oracle: free-stream preservation on curved periodic grids,
discrete conservation, design order on smooth waves, stationary contacts, hybrid
flag dilation and the Sod shock tube against the exact solution."""
import numpy as np
import pytest

from oracle import grid as gr, rhs as R, riemann
from paper_2511_18042_amd import cases

GAS = R.Gas(gamma=1.4)


def _grid(c):
    return gr.Grid(c.ndim, c.n, c.bc, c.h, c.coords)


SCHEMES = [('cgbr', 'E6'), ('cgbr', 'C4'), ('lad', 'E6'), ('lad', 'C6'), ('hybrid', 'E6'), ('hybrid', 'C4')]


def _opts(grad, **kw):
    """'C6' selects LAD-C6 (the gradient option is then unused by the LAD scheme)."""
    if grad == 'C6':
        return R.Opts(lad='C6', **kw)
    return R.Opts(grad=grad, **kw)


@pytest.mark.parametrize('ndim,n', [(2, (20, 16)), (3, (12, 10, 9))])
@pytest.mark.parametrize('scheme,grad', [sg for sg in SCHEMES if sg[1] != 'C6'])
@pytest.mark.parametrize('viscous', [False, True])
def test_free_stream_preserved_on_wavy_grid(ndim, n, scheme, grad, viscous):
    c = cases.uniform_state(cases.periodic_case(ndim, n, curvilinear=True, amp=0.1))
    g = _grid(c)
    gas = R.Gas(gamma=1.4, viscous=viscous, Re=100.0, Mref=0.5)
    flags = np.random.default_rng(7).random(g.shape) < 0.05 if scheme == 'hybrid' else None
    L = R.rhs(c.Q, g, gas, _opts(grad, C_mu=0.002), scheme, force_flags=flags)
    assert np.isfinite(L).all()
    assert np.max(np.abs(L)) <= 1e-12, np.max(np.abs(L))


def test_lad_c6_free_stream_error_is_fourth_order_on_wavy_grids():
    """R30: the D4 metrics satisfy the metric identity for D4 differences; under the C6
    differences of LAD-C6 a uniform stream leaves a residual that falls at fourth order."""
    errs = []
    for n in ((20, 16), (40, 32), (80, 64)):
        c = cases.uniform_state(cases.periodic_case(2, n, curvilinear=True, amp=0.1))
        L = R.rhs(c.Q, _grid(c), GAS, _opts('C6'), 'lad')
        errs.append(np.max(np.abs(L)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[0] > 1e-5 and np.all(orders > 3.8), (errs, orders)


@pytest.mark.parametrize('scheme,grad', SCHEMES)
def test_discrete_conservation_periodic(scheme, grad):
    c = cases.random_rough_state(cases.periodic_case(2, (24, 20), curvilinear=True, amp=0.05), seed=3)
    g = _grid(c)
    M = gr.node_metrics(g)
    inner = (slice(None),) + g.interior()
    # the LAD-C6 filter acts on Q, so it keeps sum Q but not the volume-weighted sum on a
    # curved grid: the RK steps are checked without it
    opts = _opts(grad, rho_thr=0.8, p_thr=0.6, filter_alpha=0.5)
    total0 = (c.Q[inner] / M[9][g.interior()]).sum(axis=(1, 2, 3))
    Q, t = c.Q.copy(), 0.0
    for _ in range(4):
        Q, t, dt, bad = R.rk3_step(Q, t, 1.0, g, GAS, opts, scheme, M)
    total = (Q[inner] / M[9][g.interior()]).sum(axis=(1, 2, 3))
    scale = (np.abs(c.Q[inner]) / M[9][g.interior()]).sum(axis=(1, 2, 3))
    assert np.all(np.abs(total - total0) <= 1e-13 * scale), (total - total0) / scale


def _wave(n, kind):
    c = cases.Case(1, (n, 1, 1), [(cases.PERIODIC, cases.PERIODIC)], h=(1.0 / n, 1, 1))
    x, _, _ = cases.cartesian_mesh(c)
    s = np.sin(2 * np.pi * x)
    one = np.ones_like(x)
    if kind == 'entropy':
        W = (1 + 0.2 * s, one, 0 * one, 0 * one, one)
    else:
        W = (one, one, 0.1 * s, 0 * one, one)
    c.Q = cases.conserved(*W, 1.4)
    return c, x


@pytest.mark.parametrize('scheme,grad', [('cgbr', 'E6'), ('cgbr', 'C4'), ('lad', 'E6')])
@pytest.mark.parametrize('viscous', [False, True])
def test_rhs_truncation_order(scheme, grad, viscous):
    """Entropy and shear waves: L1 order 4 (the flux-difference operator of R1 is fourth
    order for E6 and C4 gradients alike).  The MP test switches scheme at smooth extrema,
    which costs one order in the max norm only; it governs the entropy field always and,
    in inviscid flow (R26), every field.  With the wave-appropriate rule of viscous flow
    (Re = 1e12, so the viscous terms stay below 1e-10), the shear field is governed by the
    Omega sensor, which stays below its threshold on a smooth shear wave, and the shear
    wave is fourth order in the max norm as well."""
    gas = R.Gas(gamma=1.4, viscous=True, Re=1e12) if viscous else GAS
    for kind, comp, amp in (('entropy', 0, 0.2), ('shear', 2, 0.1)):
        e1, einf = [], []
        for n in (32, 64, 128):
            c, x = _wave(n, kind)
            L = R.rhs(c.Q, _grid(c), gas, R.Opts(grad=grad), scheme)
            xi = x[0, 0, 5:5 + n]
            ex = -amp * 2 * np.pi * np.cos(2 * np.pi * xi)
            e = L[comp, 0, 0, 5:5 + n] - ex
            e1.append(np.abs(e).mean())
            einf.append(np.abs(e).max())
        o1 = np.log2(np.array(e1[:-1]) / np.array(e1[1:]))
        oinf = np.log2(np.array(einf[:-1]) / np.array(einf[1:]))
        assert np.all(np.abs(o1 - 4.0) < 0.3), (kind, o1)
        if (kind == 'shear' and viscous) or scheme == 'lad':
            assert np.all(np.abs(oinf - 4.0) < 0.3), (kind, oinf)


def test_stationary_contact_is_steady_under_cgbr():
    c = cases.Case(1, (40, 1, 1), [(cases.TRANSMISSIVE,) * 2], h=(1 / 40, 1, 1))
    x, _, _ = cases.cartesian_mesh(c)
    rho = np.where(x < 0.5, 1.0, 0.125)
    z = np.zeros_like(x)
    c.Q = cases.conserved(rho, z, z, z, 0.7 + z, 1.4)
    for grad in ('E6', 'C4'):
        L = R.rhs(c.Q, _grid(c), GAS, R.Opts(grad=grad), 'cgbr')
        assert np.max(np.abs(L)) < 1e-12


def test_hybrid_dilation_pattern():
    """One troubled node selects C-GBR on exactly the interfaces within the dilation box."""
    c = cases.uniform_state(cases.periodic_case(2, (24, 20)))
    g = _grid(c)
    i0, j0 = 5 + 10, 5 + 8
    Q = c.Q.copy()
    Q[:, 0, j0, i0] *= 0.1          # low density (and energy) at one node
    info = {}
    R.rhs(Q, g, GAS, R.Opts(rho_thr=0.5), 'hybrid', info=info)
    f = info['flags']
    assert f.sum() == 1 and f[0, j0, i0]
    gx, gy = info['selectors']
    jj, ii = np.nonzero(gx[0])
    assert set(jj) == set(range(j0 - 3, j0 + 4))
    assert set(ii) == set(range(i0 - 4, i0 + 4))
    jj, ii = np.nonzero(gy[0])
    assert set(ii) == set(range(i0 - 3, i0 + 4))
    assert set(jj) == set(range(j0 - 4, j0 + 4))
    # global mode: the whole field becomes C-GBR
    R.rhs(Q, g, GAS, R.Opts(rho_thr=0.5, hybrid_mode='global'), 'hybrid', info=info)
    assert all(s.all() for s in info['selectors'])


def test_hybrid_without_flags_equals_lad_and_all_flags_equals_cgbr():
    c = cases.random_smooth_state(cases.periodic_case(2, (16, 14), curvilinear=True), seed=5)
    g = _grid(c)
    o = R.Opts()
    Lh0 = R.rhs(c.Q, g, GAS, o, 'hybrid', force_flags=np.zeros(g.shape, bool))
    Lh1 = R.rhs(c.Q, g, GAS, o, 'hybrid', force_flags=np.ones(g.shape, bool))
    assert np.array_equal(Lh0, R.rhs(c.Q, g, GAS, o, 'lad'))
    assert np.array_equal(Lh1, R.rhs(c.Q, g, GAS, o, 'cgbr'))


@pytest.mark.parametrize('grad', ['E6', 'C4'])
def test_sod_against_exact_solution(grad):
    l1 = []
    for n in (100, 200):
        c = cases.sod(n)
        Q, steps, bad = R.run(c.Q.copy(), c.t_end, _grid(c), GAS, R.Opts(grad=grad, cfl=0.5), 'cgbr')
        assert bad == 0
        g = _grid(c)
        W = R.primitives(Q[(slice(None),) + g.interior()], 1.4)[:, 0, 0, :]
        x = (np.arange(n) + 0.5) / n
        ex = riemann.sample((1, 0, 1), (0.125, 0, 0.1), 1.4, (x - 0.5) / 0.2)
        l1.append(np.abs(W[0] - ex[0]).mean())
        assert np.abs(W[4] - ex[2]).mean() < 0.01
    assert l1[1] < 0.65 * l1[0]          # converges at about first order through the discontinuities
    assert l1[1] < 2e-3


@pytest.mark.parametrize('scheme,grad', [('cgbr', 'E6'), ('cgbr', 'C4'), ('lad', 'E6')])
def test_viscous_heating_of_linear_shear(scheme, grad):
    """u = a y, v = w = 0, uniform rho and p: the convective RHS vanishes, the shear stress
    mu a is uniform, and the only RHS is the viscous heating dE/dt = mu a^2 (Eq. tauij),
    with mu = mu_hat(T = 1) = 1/Re (Sutherland is 1 at the reference temperature)."""
    a, Re, Mref, g = 0.8, 50.0, 0.5, 1.4
    c = cases.Case(2, (12, 16, 1), [(cases.PERIODIC,) * 2, (cases.FIXED,) * 2], h=(1 / 12, 1 / 16, 1))
    x, y, _ = cases.cartesian_mesh(c)
    rho = np.ones_like(x)
    p = rho / (g * Mref ** 2)                       # T = gamma M^2 p / rho = 1
    c.Q = cases.conserved(rho, a * y, 0 * x, 0 * x, p, g)
    gas = R.Gas(gamma=g, viscous=True, Re=Re, Mref=Mref)
    L = R.rhs(c.Q, _grid(c), gas, R.Opts(grad=grad), scheme)
    gr_ = _grid(c)
    Li = L[(slice(None),) + gr_.interior()]
    assert np.max(np.abs(Li[:4])) < 1e-12
    assert np.allclose(Li[4], a * a / Re, rtol=1e-11)
