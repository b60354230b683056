"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds initial conditions and grids only -- none of the method's
arithmetic -- and imports neither the HIP library nor the oracle.  States are the
physical conserved variables Q = (rho, rho u, rho v, rho w, E) on the ghost-padded
node layout (5, Nz, Ny, Nx), five ghost layers per active direction, cell-centred
nodes.  Ghost values of boundaries marked FIXED are set here and never rewritten
by either side; all other ghosts are left at the nearest interior value and are
refilled by the boundary images at every stage.

Workloads (shapes and value ranges of the paper's cases, Sec. 3):
  sod            1D shock tube, Sec. 3.1
  lax, le_blanc  1D shock tubes with the printed states, Sec. 3.1
  shu_osher      1D shock / entropy-wave interaction, Sec. 3.1
  khi            2D Kelvin-Helmholtz instability, Sec. 3.2
  riemann_c3, riemann_c12   2D four-quadrant Riemann problems, Sec. 3.2
  triple_point   2D three-state Riemann problem, Sec. 3.2
  shock_bubble   2D shock / light-cylinder interaction, Sec. 3.2
  quadrants      2D four-quadrant Riemann problems with seeded random states
  ramp3d         3D curvilinear compression-ramp grid with a turbulent-boundary-
                 layer-like state (M 2.9, 24 degrees; Sec. 3.4 shapes)
  wavy / random  smooth periodic test fields on sinusoidally perturbed grids
"""
from dataclasses import dataclass, field

import numpy as np

NG = 5
PERIODIC, TRANSMISSIVE, REFLECTIVE, NOSLIP, FIXED, NOSLIP_ISOTHERMAL = 0, 1, 2, 3, 4, 5


@dataclass
class Case:
    ndim: int
    n: tuple                      # interior nodes (nx, ny, nz)
    bc: list                      # [(lo, hi)] * 3
    h: tuple = (1.0, 1.0, 1.0)    # Cartesian spacings
    coords: object = None         # (3, Nz, Ny, Nx) for curvilinear grids
    Q: object = None              # (5, Nz, Ny, Nx) conserved state incl. ghosts
    gamma: float = 1.4
    t_end: float = 0.0
    x0: tuple = (0.0, 0.0, 0.0)
    extra: dict = field(default_factory=dict)
    wall_T: object = None         # [(lo, hi)] * 3: temperatures of NOSLIP_ISOTHERMAL faces

    @property
    def g(self):
        return tuple(NG if d < self.ndim else 0 for d in range(3))

    @property
    def N(self):
        return tuple(self.n[d] + 2 * self.g[d] for d in range(3))

    @property
    def shape(self):
        N = self.N
        return (N[2], N[1], N[0])

    @property
    def cells(self):
        return int(self.n[0] * self.n[1] * self.n[2])


def node_positions(n, g, x0, h):
    """Cell-centred node coordinates including ghosts: x0 + (i + 1/2) h for i in [-g, n+g)."""
    return x0 + (np.arange(-g, n + g) + 0.5) * h


def cartesian_mesh(case):
    """(x, y, z) node coordinates broadcast to the field shape."""
    g = case.g
    xs = [node_positions(case.n[d], g[d], case.x0[d], case.h[d]) for d in range(3)]
    z, y, x = np.meshgrid(xs[2], xs[1], xs[0], indexing='ij')
    return x, y, z


def conserved(rho, u, v, w, p, gamma):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, E]).astype(np.float64)


def _pad3(n):
    n = tuple(int(v) for v in n)
    return n + (1,) * (3 - len(n))


# ----------------------------------------------------------------- 1D cases
def sod(n=400):
    c = Case(1, _pad3((n,)), [(TRANSMISSIVE, TRANSMISSIVE)], h=(1.0 / n, 1.0, 1.0), t_end=0.2)
    x, _, _ = cartesian_mesh(c)
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    z = np.zeros_like(x)
    c.Q = conserved(rho, z, z, z, p, c.gamma)
    c.extra = dict(left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), x_interface=0.5)
    return c


def shock_tube(n, length, x_face, left, right, t_end, gamma=1.4):
    """1D Riemann problem on [0, length]: (rho, u, p) left / right of x_face; the inflow
    (left) ghosts hold the initial left state (FIXED), the outflow extrapolates."""
    c = Case(1, _pad3((n,)), [(FIXED, TRANSMISSIVE)], h=(length / n, 1.0, 1.0), t_end=t_end, gamma=gamma)
    x, _, _ = cartesian_mesh(c)
    lft = x < x_face
    rho = np.where(lft, left[0], right[0])
    u = np.where(lft, left[1], right[1])
    p = np.where(lft, left[2], right[2])
    z = np.zeros_like(x)
    c.Q = conserved(rho, u, z, z, p, gamma)
    c.extra = dict(left=tuple(left), right=tuple(right), x_interface=x_face)
    return c


def lax(n=200):
    return shock_tube(n, 1.0, 0.5, (0.445, 0.698, 3.528), (0.5, 0.0, 0.571), 0.14)


def le_blanc(n=900):
    """Density and pressure jumps of 1e3 and 1e9, gamma = 5/3, t = 6."""
    return shock_tube(n, 9.0, 3.0, (1.0, 0.0, 2.0 / 3.0 * 1e-1), (1e-3, 0.0, 2.0 / 3.0 * 1e-10), 6.0,
                      gamma=5.0 / 3.0)


SHU_OSHER_POST = (3.857143, 2.629369, 10.33333)


def shu_osher(n=2000):
    """Mach-3 shock at x = -4 entering rho = 1 + 0.2 sin(5x); left ghosts fixed at the post-shock state."""
    c = Case(1, _pad3((n,)), [(FIXED, TRANSMISSIVE)], h=(10.0 / n, 1.0, 1.0),
             x0=(-5.0, 0.0, 0.0), t_end=1.8)
    x, _, _ = cartesian_mesh(c)
    post = x < -4.0
    rho = np.where(post, SHU_OSHER_POST[0], 1.0 + 0.2 * np.sin(5.0 * x))
    u = np.where(post, SHU_OSHER_POST[1], 0.0)
    p = np.where(post, SHU_OSHER_POST[2], 1.0)
    z = np.zeros_like(x)
    c.Q = conserved(rho, u, z, z, p, c.gamma)
    return c


# ----------------------------------------------------------------- 2D cases
def triple_point(nx=1792, ny=768):
    c = Case(2, _pad3((nx, ny)), [(REFLECTIVE, REFLECTIVE), (REFLECTIVE, REFLECTIVE)],
             h=(7.0 / nx, 3.0 / ny, 1.0), t_end=5.0)
    x, y, _ = cartesian_mesh(c)
    rho = np.where(x < 1.0, 1.0, np.where(y < 1.5, 1.0, 0.125))
    p = np.where(x < 1.0, 1.0, 0.1)
    z = np.zeros_like(x)
    c.Q = conserved(rho, z, z, z, p, c.gamma)
    c.extra = dict(rho_thr=0.5 * 0.125, p_thr=0.25 * 0.1)
    return c


def quadrant_states(rng):
    """Four quadrant primitive states (rho, u, v, p) drawn from the configured ranges."""
    st = []
    for _ in range(4):
        st.append((rng.uniform(0.1, 2.0), rng.uniform(-1.0, 1.0), rng.uniform(-1.0, 1.0),
                   rng.uniform(0.1, 2.0)))
    return st


def quadrants(n, states, split=(0.5, 0.5)):
    """2D four-quadrant Riemann problem on [0,1]^2, transmissive boundaries.
    Quadrant order: (x>=sx, y>=sy), (x<sx, y>=sy), (x<sx, y<sy), (x>=sx, y<sy)."""
    c = Case(2, _pad3((n, n)), [(TRANSMISSIVE, TRANSMISSIVE)] * 2, h=(1.0 / n, 1.0 / n, 1.0))
    x, y, _ = cartesian_mesh(c)
    sx, sy = split
    q = np.where(x >= sx, np.where(y >= sy, 0, 3), np.where(y >= sy, 1, 2))
    arr = np.array(states, dtype=np.float64)
    rho, u, v, p = (arr[q, m] for m in range(4))
    c.Q = conserved(rho, u, v, np.zeros_like(rho), p, c.gamma)
    c.extra = dict(rho_thr=0.5 * arr[:, 0].min(), p_thr=0.5 * arr[:, 3].min())
    return c


def riemann_c3(n=400):
    """Strong four-quadrant problem (Schulz-Rinne configuration 3): split at 0.8,
    pressure ratio about 51, t = 0.8."""
    s11 = 4.0 / np.sqrt(11.0)
    st = [(1.5, 0.0, 0.0, 1.5), (33.0 / 62.0, s11, 0.0, 0.3), (77.0 / 558.0, s11, s11, 9.0 / 310.0),
          (33.0 / 62.0, 0.0, s11, 0.3)]
    c = quadrants(n, st, split=(0.8, 0.8))
    c.t_end = 0.8
    return c


def riemann_c12(n=800):
    """Weak four-quadrant problem (the paper's configuration F): split at 0.5, t = 0.25."""
    st = [(0.5313, 0.0, 0.0, 0.4), (1.0, 0.7276, 0.0, 1.0), (0.8, 0.0, 0.0, 1.0), (1.0, 0.0, 0.7276, 1.0)]
    c = quadrants(n, st, split=(0.5, 0.5))
    c.t_end = 0.25
    return c


def khi(n=512):
    """Kelvin-Helmholtz instability on the periodic unit square, t = 0.8: p = 2.5, a
    heavy (rho 2, u 0.5) band 0.25 < y <= 0.75 in light fluid (rho 1, u -0.5), and a
    sin(4 pi x) v perturbation on both interfaces (Gaussian width 0.05 / sqrt 2)."""
    c = Case(2, _pad3((n, n)), [(PERIODIC, PERIODIC)] * 2, h=(1.0 / n, 1.0 / n, 1.0), t_end=0.8)
    x, y, _ = cartesian_mesh(c)
    band = (y > 0.25) & (y <= 0.75)
    rho = np.where(band, 2.0, 1.0)
    u = np.where(band, 0.5, -0.5)
    sig = 0.05 / np.sqrt(2.0)
    v = 0.1 * np.sin(4 * np.pi * x) * (np.exp(-(y - 0.75) ** 2 / (2 * sig ** 2)) +
                                       np.exp(-(y - 0.25) ** 2 / (2 * sig ** 2)))
    p = np.full_like(x, 2.5)
    c.Q = conserved(rho, u, v, np.zeros_like(x), p, c.gamma)
    c.extra = dict(rho_thr=-1.0, p_thr=-1.0)
    return c


SHOCK_BUBBLE_POST = (1.3764, -0.3336, 1.5698 / 1.4)


def shock_bubble(nx=1300, ny=356):
    """Mach 1.22 shock at x/D = 4.5 moving into still air (rho 1, p 1/1.4) towards a light
    cylinder (rho 0.1819, same pressure) of diameter D = 1 centred at (3.5, 0.89), on
    [0, 6.5] x [0, 1.78]; outflow left and right, inviscid walls top and bottom, t = 6."""
    c = Case(2, _pad3((nx, ny)), [(TRANSMISSIVE, TRANSMISSIVE), (REFLECTIVE, REFLECTIVE)],
             h=(6.5 / nx, 1.78 / ny, 1.0), t_end=6.0)
    x, y, _ = cartesian_mesh(c)
    post = x > 4.5
    bubble = (x - 3.5) ** 2 + (y - 0.89) ** 2 < 0.25
    rho = np.where(post, SHOCK_BUBBLE_POST[0], np.where(bubble, 0.1819, 1.0))
    u = np.where(post, SHOCK_BUBBLE_POST[1], 0.0)
    p = np.where(post, SHOCK_BUBBLE_POST[2], 1.0 / 1.4)
    c.Q = conserved(rho, u, np.zeros_like(x), np.zeros_like(x), p, c.gamma)
    c.extra = dict(rho_thr=0.5 * 0.1819, p_thr=-1.0)
    return c


BATCH_SEED = 18042


def batch64(count=64, sizes=(128, 256, 512, 1024), seed=BATCH_SEED, scale=1):
    """The batched serving workload: ``count`` four-quadrant problems with sizes drawn from
    ``sizes`` and per-quadrant states from the same generator.  ``scale`` divides every size
    (used for small test versions of the same draw)."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.array(sizes), count)
    out = []
    for n in ns:
        st = quadrant_states(rng)
        out.append(quadrants(max(8, int(n) // scale), st))
    return out


# ----------------------------------------------------------------- test fields
def wavy_coords(ndim, n, amp=0.1, g=NG):
    """Sinusoidally perturbed periodic grid on the unit square/cube:
    x_m = xi_m + amp prod_k sin(2 pi xi_k) (cell-centred xi)."""
    gs = [g if d < ndim else 0 for d in range(3)]
    n = _pad3(n)
    xi = [node_positions(n[d], gs[d], 0.0, 1.0 / n[d]) if d < ndim else np.zeros(1) for d in range(3)]
    Z, Y, X = np.meshgrid(xi[2], xi[1], xi[0], indexing='ij')
    base = [X, Y, Z]
    prod = np.ones_like(X)
    for d in range(ndim):
        prod = prod * np.sin(2.0 * np.pi * base[d])
    coords = np.stack([base[d] + amp * prod if d < ndim else base[d] for d in range(3)])
    return coords


def periodic_case(ndim, n, curvilinear=False, amp=0.1):
    n = _pad3(n)
    bc = [(PERIODIC, PERIODIC)] * ndim
    h = tuple(1.0 / n[d] if d < ndim else 1.0 for d in range(3))
    c = Case(ndim, n, bc, h=h)
    if curvilinear:
        c.coords = wavy_coords(ndim, n, amp)
    return c


def uniform_state(case, rho=1.0, u=0.5, v=0.3, w=0.2, p=1.0 / 1.4):
    shape = case.shape
    f = lambda a: np.full(shape, float(a))  # noqa: E731
    vv = v if case.ndim >= 2 else 0.0
    ww = w if case.ndim >= 3 else 0.0
    case.Q = conserved(f(rho), f(u), f(vv), f(ww), f(p), case.gamma)
    return case


def random_smooth_state(case, seed, amp=0.2, modes=3):
    """Smooth periodic random primitives (positive rho, p) on a periodic case."""
    rng = np.random.default_rng(seed)
    if case.coords is not None:
        X = [case.coords[d] for d in range(3)]
    else:
        X = list(cartesian_mesh(case))
    def field_(base, a):
        f = np.full(case.shape, base)
        for _ in range(modes):
            k = rng.integers(1, 4, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            arg = ph + sum(2 * np.pi * k[d] * X[d] / (case.n[d] * case.h[d]) for d in range(case.ndim))
            f = f + a * rng.uniform(-1, 1) * np.sin(arg)
        return f
    rho = field_(1.0, amp)
    u = field_(0.3, amp)
    v = field_(-0.2, amp) if case.ndim >= 2 else np.zeros(case.shape)
    w = field_(0.1, amp) if case.ndim >= 3 else np.zeros(case.shape)
    p = field_(1.0, amp)
    case.Q = conserved(rho, u, v, w, p, case.gamma)
    return case


def random_rough_state(case, seed, jumps=True):
    """Random piecewise-smooth data with discontinuities: exercises limiter branches."""
    rng = np.random.default_rng(seed)
    shape = case.shape
    def fld(lo, hi):
        f = rng.uniform(lo, hi, size=shape)
        if jumps:
            blocks = rng.uniform(lo, hi, size=(4,) * 3)
            idx = [np.minimum((np.arange(s) * 4) // max(s, 1), 3) for s in shape]
            f = 0.7 * blocks[np.ix_(*idx)] + 0.3 * f
        return f
    rho = fld(0.3, 2.0)
    u = fld(-1.0, 1.0)
    v = fld(-1.0, 1.0) if case.ndim >= 2 else np.zeros(shape)
    w = fld(-1.0, 1.0) if case.ndim >= 3 else np.zeros(shape)
    p = fld(0.3, 2.0)
    case.Q = conserved(rho, u, v, w, p, case.gamma)
    return case


def entropy_wave(n, t=0.0):
    """rho = 1 + 0.2 sin(2 pi (x - t)), u = 1, p = 1 on a periodic unit interval."""
    c = Case(1, _pad3((n,)), [(PERIODIC, PERIODIC)], h=(1.0 / n, 1.0, 1.0))
    x, _, _ = cartesian_mesh(c)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * (x - t))
    one = np.ones_like(x)
    c.Q = conserved(rho, one, 0 * one, 0 * one, one, c.gamma)
    return c


# ----------------------------------------------------------------- 3D ramp
RAMP_SEED = 2511
RAMP_MACH = 2.9


# integral length scales of the digital-filter inflow in units of the inflow boundary-layer
# thickness (Sec. 4, table of length scales): u, v, w
DF_IX = (0.7, 0.28, 0.28)
DF_IY = ((0.13, 0.23), (0.17, 0.3), (0.1, 0.13))     # (inner, outer)
DF_IZ = (0.15, 0.15, 0.3)


def ramp_df_inflow(c, delta=1.0, M=RAMP_MACH, gamma=1.4):
    """Inputs of the digital-filter inflow generator for a ramp3d case (keyword arguments of
    lgbr.DFInflow / oracle.inflow.DFSpec): the first interior xi column's rows; mean
    rho, U, V, T averaged over the span; Reynolds stresses from a model boundary layer
    (u, v, w rms 0.10, 0.06, 0.08 U_inf times (1 - y/delta)(1 - exp(-y / 0.05 delta)) below
    delta, R21 = -0.4 u_rms v_rms); inner zone up to the displacement thickness of the mean
    profile; the length-scale table in units of delta; the analogy at the free-stream Mach
    number; the free-stream pressure."""
    g = NG
    X, Y = c.coords[0], c.coords[1]
    ny = c.n[1]
    col = Y[g, :, g]                                   # first interior xi column, one z plane
    wall = 0.5 * (col[g - 1] + col[g])                 # the wall face
    y = col[g:g + ny] - wall
    dy = 0.5 * (col[g + 1:g + ny + 1] - col[g - 1:g + ny - 1])
    Q = c.Q[:, g:g + c.n[2], g:g + ny, g]              # (5, nz, ny)
    rho = Q[0].mean(axis=0)
    U = (Q[1] / Q[0]).mean(axis=0)
    V = (Q[2] / Q[0]).mean(axis=0)
    ke = 0.5 * (Q[1] ** 2 + Q[2] ** 2 + Q[3] ** 2) / Q[0]
    p = ((gamma - 1.0) * (Q[4] - ke)).mean(axis=0)
    T = gamma * M * M * p / rho
    f = np.where(y < delta, (1.0 - y / delta) * (1.0 - np.exp(-y / (0.05 * delta))), 0.0)
    urms, vrms, wrms = 0.10 * f, 0.06 * f, 0.08 * f
    rey = np.stack([urms ** 2, -0.4 * urms * vrms, vrms ** 2, wrms ** 2])
    inside = y < delta
    y_lim = float(np.sum(((1.0 - np.clip(U, 0.0, 1.0)) * dy)[inside]))
    return dict(dy=dy, y=y, dz=c.h[2], y_lim=y_lim, Iy=[tuple(v) for v in DF_IY], Iz=list(DF_IZ),
                Ix=list(DF_IX), U_ref=1.0, mean=np.stack([rho, U, V, T]), rey=rey, M_sra=M,
                p=1.0 / (gamma * M * M))


def _stretch(eta, beta):
    """Wall-normal tanh clustering: 0 at the wall (eta = 0), 1 at the top (eta = 1)."""
    return 1.0 + np.tanh(beta * (eta - 1.0)) / np.tanh(beta)


def ramp3d(nx=1024, ny=384, nz=128, seed=RAMP_SEED, Lx=26.2, Ly=7.9, Lz=3.0, angle_deg=24.0,
           y1=0.002, delta=1.0, noise_rms=0.05, M=RAMP_MACH, gamma=1.4, Pr=0.72, wall='adiabatic'):
    """Curvilinear compression-ramp grid and a turbulent-boundary-layer-like state.

    Grid (lengths in units of the inflow boundary-layer thickness delta):
      x_i uniform on [0, Lx]; wall y_w(x) = tan(angle) r log(1 + exp((x - x_c)/r)) with the
      corner at x_c = Lx/2 rounded over r = 0.5; y = y_w + s(eta)(Ly - y_w) with tanh
      clustering s chosen so the first cell centre sits at y1 above the wall; z uniform,
      periodic.  Ghost nodes continue the same maps.
    State (non-dimensional with the free stream: rho = u = T = 1, p = 1/(gamma M^2)):
      u/U = min(1, y_n/delta)^(1/7) above 5 y1 and linear below (y_n = height above the wall),
      directed along the wall tangent with the angle relaxing as exp(-y_n / 2 delta);
      T from the adiabatic Crocco-Busemann relation T = T_aw - (T_aw - 1)(u/U)^2 with
      T_aw = 1 + Pr^(1/3) (gamma - 1) M^2 / 2; uniform p; rho = gamma M^2 p / T.
      Fluctuations: curl of a Gaussian-smoothed (4-cell) normal random vector potential in
      index space, limited to y_n < delta, scaled to noise_rms of U (seeded).
    Boundaries: fixed inflow ghosts (the initial profile), transmissive (supersonic)
    outflow and top, periodic span, and a no-slip wall: adiabatic, or with
    wall='isothermal' held at 1.14 times the recovery temperature T_aw (Sec. 4, M2.9 ramp).
    """
    from scipy.ndimage import gaussian_filter, zoom
    n = (nx, ny, nz)
    c = Case(3, n, [(FIXED, TRANSMISSIVE), (NOSLIP, TRANSMISSIVE), (PERIODIC, PERIODIC)],
             h=(Lx / nx, Ly / ny, Lz / nz), gamma=gamma)
    Taw = 1.0 + Pr ** (1.0 / 3.0) * 0.5 * (gamma - 1.0) * M * M
    if wall == 'isothermal':
        c.bc[1] = (NOSLIP_ISOTHERMAL, TRANSMISSIVE)
        c.wall_T = [(0.0, 0.0), (1.14 * Taw, 0.0), (0.0, 0.0)]
    elif wall != 'adiabatic':
        raise ValueError('wall: adiabatic or isothermal')
    g = NG
    xs = (np.arange(-g, nx + g) + 0.5) * (Lx / nx)
    eta = (np.arange(-g, ny + g) + 0.5) / ny
    zs = (np.arange(-g, nz + g) + 0.5) * (Lz / nz)
    # tanh clustering parameter for the requested first-cell height
    lo, hi = 1e-3, 20.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if _stretch(0.5 / ny, mid) * Ly > y1:
            lo = mid
        else:
            hi = mid
    beta = 0.5 * (lo + hi)
    ta = np.tan(np.radians(angle_deg))
    r = 0.5
    xc = 0.5 * Lx
    yw = ta * r * np.logaddexp(0.0, (xs - xc) / r)
    slope = ta / (1.0 + np.exp(-(xs - xc) / r))
    s = _stretch(eta, beta)
    Z, Sg, X = np.meshgrid(zs, s, xs, indexing='ij')
    _, _, YW = np.meshgrid(zs, s, yw, indexing='ij')
    _, _, SL = np.meshgrid(zs, s, slope, indexing='ij')
    Y = YW + Sg * (Ly - YW)
    c.coords = np.stack([X, Y, Z])
    yn = Y - YW
    # mean profile
    ylin = 5.0 * y1
    frac = np.clip(yn / delta, 0.0, 1.0)
    ulog = frac ** (1.0 / 7.0)
    ulin = (ylin / delta) ** (1.0 / 7.0) * np.clip(yn, 0.0, None) / ylin
    U = np.where(yn >= ylin, ulog, ulin)
    alpha = np.arctan(SL) * np.exp(-np.clip(yn, 0.0, None) / (2.0 * delta))
    u = U * np.cos(alpha)
    v = U * np.sin(alpha)
    w = np.zeros_like(u)
    # divergence-free fluctuations (curl of a smoothed vector potential, index space)
    rng = np.random.default_rng(seed)
    shape = X.shape
    coarse = tuple(max(4, (sz + 3) // 4) for sz in shape)
    psi = []
    for _ in range(3):
        a = gaussian_filter(rng.standard_normal(coarse), sigma=1.0, mode='wrap')
        a = zoom(a, [shape[k] / coarse[k] for k in range(3)], order=1)[:shape[0], :shape[1], :shape[2]]
        psi.append(a)
    def dd(f, ax):
        return 0.5 * (np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax))
    # axes: 0 = z, 1 = y, 2 = x
    fx = dd(psi[2], 1) - dd(psi[1], 0)
    fy = dd(psi[0], 0) - dd(psi[2], 2)
    fz = dd(psi[1], 2) - dd(psi[0], 1)
    mask = (yn > 0.0) & (yn < delta)
    rms = np.sqrt(np.mean((fx ** 2 + fy ** 2 + fz ** 2)[mask]) / 3.0)
    k = noise_rms / max(rms, 1e-300)
    u = u + k * fx * mask
    v = v + k * fy * mask
    w = w + k * fz * mask
    T = Taw - (Taw - 1.0) * np.clip(U, 0.0, 1.0) ** 2
    p = np.full_like(T, 1.0 / (gamma * M * M))
    rho = gamma * M * M * p / T
    c.Q = conserved(rho, u, v, w, p, gamma)
    c.extra = dict(p_thr=0.5 / (gamma * M * M), rho_thr=-1.0, Re=2.0e4, Pr=Pr, Mref=M,
                   suth=110.4 / 108.0, beta_stretch=beta, T_aw=Taw)
    return c
