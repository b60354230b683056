"""Pins of the oracle's C-GBR pieces: characteristic transform, GBR linear states,
MP5, HLLC and the Omega sensor (Sec. 2.3)."""
import numpy as np
import pytest

from oracle import gbr

G = 1.4


def _unit(rng, n):
    v = rng.normal(size=(3, n))
    return v / np.linalg.norm(v, axis=0)


def test_tangent_basis_is_orthonormal():
    rng = np.random.default_rng(1)
    n = _unit(rng, 500)
    n[:, :3] = np.eye(3)  # axis-aligned normals (ties in argmin)
    t1, t2 = gbr.tangents(n)
    for a, b in ((n, t1), (n, t2), (t1, t2)):
        assert np.allclose((a * b).sum(0), 0, atol=1e-15)
    for a in (t1, t2):
        assert np.allclose((a * a).sum(0), 1, atol=1e-15)
    # right-handed: t2 = n x t1
    assert np.allclose(np.cross(n.T, t1.T).T, t2, atol=1e-15)


def test_characteristic_round_trip():
    rng = np.random.default_rng(2)
    m = 400
    n = _unit(rng, m)
    t1, t2 = gbr.tangents(n)
    rb = rng.uniform(0.1, 3, m)
    cb = rng.uniform(0.3, 3, m)
    V = np.stack([rng.uniform(0.1, 3, m), *rng.normal(size=(3, m)), rng.uniform(0.1, 3, m)])
    C = gbr.to_characteristic(V, n, t1, t2, rb, cb)
    back = gbr.from_characteristic(C, n, t1, t2, rb, cb)
    assert np.max(np.abs(back - V)) < 1e-14 * np.max(np.abs(V)) * 10
    # matrices: L R = I column by column
    E = np.eye(5)[:, :, None] * np.ones(m)
    for k in range(5):
        LR = gbr.to_characteristic(gbr.from_characteristic(E[k], n, t1, t2, rb, cb), n, t1, t2, rb, cb)
        assert np.allclose(LR, E[k], atol=1e-13)


def test_characteristic_fields_are_the_acoustic_entropy_shear_waves():
    """A pure entropy jump (drho, no du, no dp) only changes C2; a pure shear jump only
    C3/C4; an acoustic right-running perturbation (dp = rho c dun) only C5."""
    n = np.array([[0.6], [0.8], [0.0]])
    t1, t2 = gbr.tangents(n)
    rb, cb = np.array([1.3]), np.array([0.9])
    base = np.array([[1.0], [0.1], [0.2], [0.3], [1.0]])
    def dC(dV):
        return gbr.to_characteristic(base + dV, n, t1, t2, rb, cb) - gbr.to_characteristic(base, n, t1, t2, rb, cb)
    d = dC(np.array([[0.1], [0], [0], [0], [0]]))
    assert np.allclose(d[[0, 2, 3, 4]], 0, atol=1e-15) and abs(d[1, 0]) > 0
    sh = 0.1 * t1
    d = dC(np.vstack([[0], sh, [0]]))
    assert np.allclose(d[[0, 1, 4]], 0, atol=1e-15)
    ac = np.vstack([[0.1 * rb[0] / cb[0]], 0.1 * n, [0.1 * rb[0] * cb[0]]])
    d = dC(ac)
    assert np.allclose(d[[0, 1, 2, 3]], 0, atol=1e-15) and abs(d[4, 0]) > 0


def _conservative_target(f, f2, x):
    """Interface value h(x) whose difference over one cell is f' exactly for cubics:
    h = f - f''/24 (unit spacing)."""
    return f(x) - f2(x) / 24.0


def test_gbr_linear_exact_for_cubics_and_not_quartics():
    x = np.arange(-1, 3, dtype=float)[:, None] + np.linspace(-2, 2, 9)[None, :]
    a = np.array([0.7, -1.1, 0.4, 0.3])
    f = lambda t: a[0] + a[1] * t + a[2] * t ** 2 + a[3] * t ** 3  # noqa: E731
    fp = lambda t: a[1] + 2 * a[2] * t + 3 * a[3] * t ** 2  # noqa: E731
    f2 = lambda t: 2 * a[2] + 6 * a[3] * t  # noqa: E731
    CL, CR = gbr.gbr_linear_states(*(f(x[k]) for k in range(4)), *(fp(x[k]) for k in range(4)))
    target = _conservative_target(f, f2, x[1] + 0.5)
    assert np.allclose(CL, target, atol=1e-13) and np.allclose(CR, target, atol=1e-13)
    q = lambda t: t ** 4  # noqa: E731
    CL, CR = gbr.gbr_linear_states(*(q(x[k]) for k in range(4)), *(4 * x[k] ** 3 for k in range(4)))
    tq = q(x[1] + 0.5) - 12 * (x[1] + 0.5) ** 2 / 24 + 7 * 24 / 5760
    assert not np.allclose(CL, tq, atol=1e-6)


def test_mp5_linear_part_exact_to_degree_four():
    """On smooth data the MP5 value is the 5-point upwind interpolant, which reproduces the
    conservative-FD interface target h = f - f''/24 + 7 f''''/5760 for polynomials of degree <= 4."""
    x0 = np.linspace(-1, 1, 7)
    for deg in range(5):
        c = np.random.default_rng(deg).normal(size=deg + 1)
        P = np.polynomial.Polynomial(c)
        vals = [P(x0 + s) for s in (-2, -1, 0, 1, 2)]
        vor = (2 * vals[0] - 13 * vals[1] + 47 * vals[2] + 27 * vals[3] - 3 * vals[4]) / 60
        xm = x0 + 0.5
        target = P(xm) - P.deriv(2)(xm) / 24 + 7 * P.deriv(4)(xm) / 5760
        assert np.allclose(vor, target, atol=1e-12)
        # monotone smooth data: MP5 returns the linear value
        if deg == 1 and abs(c[1]) > 0:
            val, _ = gbr.mp5(*vals)
            assert np.allclose(val, vor, atol=1e-14)


def test_mp5_creates_no_new_extremum_on_steps():
    rng = np.random.default_rng(3)
    for _ in range(200):
        lo, hi = sorted(rng.uniform(-2, 2, 2))
        k = rng.integers(1, 5)
        v = np.where(np.arange(5) < k, lo, hi) if rng.random() < 0.5 else np.where(np.arange(5) < k, hi, lo)
        val, _ = gbr.mp5(*[np.array([t]) for t in v])
        assert min(v[2], v[3]) - 1e-14 <= val[0] <= max(v[2], v[3]) + 1e-14


def _prim(rho, u, v, w, p):
    return np.array([[rho], [u], [v], [w], [p]], dtype=float)


def test_hllc_consistency_and_rotation():
    rng = np.random.default_rng(4)
    for _ in range(50):
        W = _prim(rng.uniform(0.2, 2), *rng.normal(size=3), rng.uniform(0.2, 2))
        xt = rng.normal(size=(3, 1)) * rng.uniform(0.1, 3)
        F = gbr.hllc(W, W, xt, G)
        assert np.allclose(F, gbr.euler_flux(W, xt, G), rtol=1e-13, atol=1e-13)
    # rotation invariance: rotating the metric and both velocity states rotates the flux
    th = 0.7
    Rm = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    WL = _prim(1.0, 0.3, -0.2, 0.1, 1.0)
    WR = _prim(0.4, -0.5, 0.6, 0.0, 0.3)
    xt = np.array([[1.2], [0.0], [0.0]])
    F = gbr.hllc(WL, WR, xt, G)
    rot = lambda Wk: np.vstack([Wk[0:1], Rm @ Wk[1:4], Wk[4:5]])  # noqa: E731
    Fr = gbr.hllc(rot(WL), rot(WR), Rm @ xt, G)
    assert np.allclose(Fr[[0, 4]], F[[0, 4]], rtol=1e-13)
    assert np.allclose(Fr[1:4], Rm @ F[1:4], rtol=1e-13, atol=1e-14)


def test_hllc_mirror_symmetry():
    WL = _prim(1.0, 0.3, 0.2, 0.0, 1.0)
    WR = _prim(0.2, -0.4, 0.1, 0.0, 0.5)
    xt = np.array([[1.0], [0.0], [0.0]])
    F = gbr.hllc(WL, WR, xt, G)
    mir = lambda Wk: np.vstack([Wk[0:1], -Wk[1:2], Wk[2:5]])  # noqa: E731
    Fm = gbr.hllc(mir(WR), mir(WL), xt, G)
    assert np.allclose(Fm[[0, 2, 3, 4]], -F[[0, 2, 3, 4]], rtol=1e-13, atol=1e-15)
    assert np.allclose(Fm[1], F[1], rtol=1e-13)


def test_hllc_resolves_stationary_contact_exactly():
    WL = _prim(1.0, 0.0, 0.3, -0.2, 0.7)
    WR = _prim(0.125, 0.0, -0.5, 0.1, 0.7)
    xt = np.array([[2.0], [0.0], [0.0]])
    F = gbr.hllc(WL, WR, xt, G)
    assert abs(F[0, 0]) < 1e-15 and abs(F[4, 0]) < 1e-15
    assert np.allclose(F[1:4, 0], [2.0 * 0.7, 0, 0], atol=1e-15)


def test_hllc_resolves_stationary_shock_exactly():
    """Rankine-Hugoniot states of a Mach-3 normal shock in its own frame: the HLLC flux
    equals the (common) physical flux on both sides."""
    M, g = 3.0, G
    r1, p1 = 1.0, 1.0
    u1 = M * np.sqrt(g * p1 / r1)
    r2 = r1 * (g + 1) * M * M / ((g - 1) * M * M + 2)
    p2 = p1 * (2 * g * M * M - (g - 1)) / (g + 1)
    u2 = u1 * r1 / r2
    WL, WR = _prim(r1, u1, 0, 0, p1), _prim(r2, u2, 0, 0, p2)
    xt = np.array([[1.0], [0.0], [0.0]])
    FL = gbr.euler_flux(WL, xt, g)
    assert np.allclose(FL, gbr.euler_flux(WR, xt, g), rtol=1e-13)
    assert np.allclose(gbr.hllc(WL, WR, xt, g), FL, rtol=1e-13)


def test_hllc_supersonic_upwinding():
    WL = _prim(1.0, 5.0, 0, 0, 1.0)
    WR = _prim(0.5, 4.0, 0, 0, 0.6)
    xt = np.array([[1.0], [0], [0]])
    assert np.allclose(gbr.hllc(WL, WR, xt, G), gbr.euler_flux(WL, xt, G), rtol=1e-14)
    assert np.allclose(gbr.hllc(_prim(1, -5, 0, 0, 1), _prim(0.5, -4, 0, 0, 0.6), xt, G),
                       gbr.euler_flux(_prim(0.5, -4, 0, 0, 0.6), xt, G), rtol=1e-14)


def test_minmod_and_median():
    a = np.array([1.0, -2.0, 3.0, 0.0])
    b = np.array([2.0, -1.0, -1.0, 5.0])
    assert np.array_equal(gbr.minmod(a, b), [1.0, -1.0, 0.0, 0.0])
    assert gbr.minmod4(np.array(2.0), np.array(3.0), np.array(1.0), np.array(4.0)) == 1.0
    assert gbr.minmod4(np.array(2.0), np.array(-3.0), np.array(1.0), np.array(4.0)) == 0.0


def test_sensor_detects_pressure_jump_at_rest_and_states_stay_positive():
    """A pressure discontinuity in a fluid at rest (theta = omega = 0) is detected by the
    Omega sensor (pressure switch alone), so the acoustic states are MP5-limited and the
    interface pressures stay positive (Sod and triple-point initial data)."""
    from oracle import grid as gr, rhs as R, derivatives as D
    from paper_2511_18042_amd import cases
    for c in (cases.sod(100), cases.triple_point(112, 48)):
        g = gr.Grid(c.ndim, c.n, c.bc, c.h)
        Q = c.Q.copy()
        gr.fill_ghosts_conserved(Q, g)
        W = R.primitives(Q, 1.4)
        M = gr.node_metrics(g)
        Gd = {l: np.stack([D.e6(W[q], l) for q in range(5)]) for l in range(g.ndim)}
        Dg = __import__('oracle.lad', fromlist=['x']).physical_gradients(Gd, M, g)
        Om = gbr.omega_sensor(W, Dg[1:4], g)
        assert np.nanmax(Om[g.interior()]) > 0.1
        for d in range(g.ndim):
            rec = {}
            F = gbr.gbr_interface_flux(W, Gd[d], gbr.omega_bar(Om, d), M, d, 1.4, record=rec)
            band = g.band(-1, 0)
            assert np.isfinite(F[(slice(None),) + band]).all()
            assert rec['WL'][4][band].min() > 0 and rec['WR'][4][band].min() > 0


def test_inviscid_rule_limits_every_field_by_the_mp_test():
    """Sec. 2.3 limits inviscid flow with the MP criterion alone (R26).  On the Sod and
    triple-point initial data (a pressure jump at rest) every field is then MP5-limited at
    the jump, so the interface pressures stay positive without the Omega sensor; on smooth
    monotone data, where every MP test passes and the sensor stays below its threshold, the
    inviscid rule and the wave-appropriate rule give the same flux."""
    from oracle import grid as gr, rhs as R, derivatives as D
    from oracle.lad import physical_gradients
    from paper_2511_18042_amd import cases
    for c in (cases.sod(100), cases.triple_point(112, 48)):
        g = gr.Grid(c.ndim, c.n, c.bc, c.h)
        Q = c.Q.copy()
        gr.fill_ghosts_conserved(Q, g)
        W = R.primitives(Q, 1.4)
        M = gr.node_metrics(g)
        Gd = {l: np.stack([D.e6(W[q], l) for q in range(5)]) for l in range(g.ndim)}
        for d in range(g.ndim):
            rec = {}
            F = gbr.gbr_interface_flux(W, Gd[d], None, M, d, 1.4, record=rec)
            band = g.band(-1, 0)
            assert np.isfinite(F[(slice(None),) + band]).all()
            assert rec['WL'][4][band].min() > 0 and rec['WR'][4][band].min() > 0
    # smooth monotone ramp in x: MP tests pass, Omega-bar small
    c = cases.Case(1, (40, 1, 1), [(cases.TRANSMISSIVE,) * 2], h=(1 / 40, 1, 1))
    x, _, _ = cases.cartesian_mesh(c)
    W = np.stack([1 + 0.1 * x, 0.2 + 0.05 * x, 0 * x, 0 * x, 1 + 0.05 * x])
    g = gr.Grid(1, c.n, c.bc, c.h)
    M = gr.node_metrics(g)
    G0 = np.stack([D.e6(W[q], 0) for q in range(5)])
    Ob = np.zeros_like(W[0])
    band = g.band(-1, 0)
    Fi = gbr.gbr_interface_flux(W, G0, None, M, 0, 1.4)
    Fv = gbr.gbr_interface_flux(W, G0, Ob, M, 0, 1.4)
    assert np.allclose(Fi[(slice(None),) + band], Fv[(slice(None),) + band], rtol=0, atol=1e-14)
