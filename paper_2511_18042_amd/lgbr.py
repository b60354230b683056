"""ctypes binding of liblgbr.so (include/lgbr.h).  Argument marshalling only: every step of
the right-hand side runs in the HIP library.  Device buffers are torch tensors on the GPU
(``data_ptr()`` is passed through); the HIP stream is torch's current stream unless given.

Raises ``RuntimeError`` when the library is missing: there is no fallback path.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, 'liblgbr.so')

LG_OK, LG_EINVAL, LG_ENOMEM, LG_EHIP, LG_ENONPHYS, LG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
BC_PERIODIC, BC_TRANSMISSIVE, BC_REFLECTIVE, BC_NOSLIP_ADIABATIC, BC_FIXED, BC_NOSLIP_ISOTHERMAL = 0, 1, 2, 3, 4, 5
GRAD_E6, GRAD_C4 = 0, 1
FP64, MIXED = 0, 1
HYB_PERCELL, HYB_GLOBAL = 0, 1
SCHEME_CGBR, SCHEME_LAD, SCHEME_HYBRID = 0, 1, 2
SCHEMES = {'cgbr': SCHEME_CGBR, 'lad': SCHEME_LAD, 'hybrid': SCHEME_HYBRID}

EXPORTS = ('lg_set_allocator', 'lg_strerror', 'lg_create', 'lg_destroy', 'lg_workspace_bytes',
           'lg_metrics_from_coords', 'cgbr_rhs', 'lad_rhs', 'hybrid_rhs', 'rk3_step', 'lg_rk3_stage',
           'lg_compute_dt', 'lg_batch_create', 'lg_batch_run', 'lg_batch_destroy', 'lg_poll_status',
           'lg_prof_start', 'lg_prof_stop', 'lg_set_tuning', 'lg_get_tuning', 'lg_metrics_planar', 'lad_filter',
           'lg_set_line_tiles', 'lg_get_line_tiles', 'lg_set_generic_access', 'lg_switch_stats', 'lg_df_create',
           'lg_df_random_count', 'lg_df_update', 'lg_df_destroy', 'lg_metrics_from_coords_noalloc',
           'lg_prof_stop_launches', 'lg_set_tile_shape', 'lg_get_tile_shape')
KERNEL_CLASSES = ('bc', 'prim', 'flags', 'grad_e6', 'grad_c4', 'sensor', 'visc', 'lad_node', 'lad_raw', 'gauss',
                  'lad_flux', 'sweep_x', 'sweep_y', 'sweep_z', 'combine', 'dt', 'bc_scalar', 'lad_sweep',
                  'c6_faces', 'filter', 'gbr_items', 'hyb_assemble', 'filter_guard')
LAD_E4, LAD_C6 = 0, 1


class LgGrid(ctypes.Structure):
    _fields_ = [('ndim', ctypes.c_int), ('n', ctypes.c_int * 3), ('ng', ctypes.c_int),
                ('bc', (ctypes.c_int * 2) * 3), ('curvilinear', ctypes.c_int), ('h', ctypes.c_double * 3),
                ('wall_T', (ctypes.c_double * 2) * 3)]


class LgGas(ctypes.Structure):
    _fields_ = [('gamma', ctypes.c_double), ('Re', ctypes.c_double), ('Pr', ctypes.c_double),
                ('Mref', ctypes.c_double), ('suth', ctypes.c_double), ('viscous', ctypes.c_int)]


class LgOpts(ctypes.Structure):
    _fields_ = [('grad', ctypes.c_int), ('precision', ctypes.c_int), ('cfl', ctypes.c_double),
                ('omega_thr', ctypes.c_double), ('mp_eps', ctypes.c_double), ('mp_alpha', ctypes.c_double),
                ('C_mu', ctypes.c_double), ('C_beta', ctypes.c_double), ('C_kappa', ctypes.c_double),
                ('hybrid_mode', ctypes.c_int), ('rho_thr', ctypes.c_double), ('p_thr', ctypes.c_double),
                ('dilate', ctypes.c_int), ('seg', ctypes.c_int), ('lad_scheme', ctypes.c_int),
                ('filter_alpha', ctypes.c_double), ('filter_every_stage', ctypes.c_int),
                ('time_scheme', ctypes.c_int)]


_lib = None


def load():
    """Open liblgbr.so (once).  Raises RuntimeError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError('liblgbr.so not built: run python -m paper_2511_18042_amd.build')
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sig = {
        'lg_set_allocator': (I, [P, P, P]),
        'lg_strerror': (ctypes.c_char_p, [I]),
        'lg_create': (I, [ctypes.POINTER(P), ctypes.POINTER(LgGrid), P, P, ctypes.POINTER(LgGas),
                          ctypes.POINTER(LgOpts), P]),
        'lg_destroy': (None, [P]),
        'lg_workspace_bytes': (S, [P]),
        'lg_metrics_planar': (I, [P]),
        'lg_metrics_from_coords': (I, [ctypes.POINTER(LgGrid), P, P, P]),
        'lg_metrics_from_coords_noalloc': (I, [ctypes.POINTER(LgGrid), P, P, P]),
        'cgbr_rhs': (I, [P, P, P]),
        'lad_rhs': (I, [P, P, P]),
        'lad_filter': (I, [P, P]),
        'hybrid_rhs': (I, [P, P, P, P, P]),
        'rk3_step': (I, [P, I, P, D, P]),
        'lg_rk3_stage': (I, [P, I, I, P, P, D]),
        'lg_compute_dt': (I, [P, P, P]),
        'lg_batch_create': (I, [ctypes.POINTER(P), P, P, P, P, I, I, I]),
        'lg_batch_run': (I, [P]),
        'lg_batch_destroy': (None, [P]),
        'lg_df_create': (I, [P, P, ctypes.POINTER(P)]),
        'lg_df_random_count': (I, [P, ctypes.POINTER(ctypes.c_longlong)]),
        'lg_df_update': (I, [P, P, P, D, I]),
        'lg_df_destroy': (None, [P]),
        'lg_poll_status': (I, [P, ctypes.POINTER(I)]),
        'lg_switch_stats': (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), I]),
        'lg_prof_start': (I, [P, I, I]),
        'lg_prof_stop': (I, [P, ctypes.POINTER(D), ctypes.POINTER(I)]),
        'lg_set_tile_shape': (I, [P, I, I]),
        'lg_get_tile_shape': (I, [P, ctypes.POINTER(I), ctypes.POINTER(I)]),
        'lg_prof_stop_launches': (I, [P, ctypes.POINTER(D), ctypes.POINTER(I), ctypes.POINTER(ctypes.c_float),
                                      ctypes.POINTER(I), I, ctypes.POINTER(I)]),
        'lg_set_tuning': (I, [P, I, I, I]),
        'lg_set_line_tiles': (I, [P, I]),
        'lg_get_line_tiles': (I, [P]),
        'lg_set_generic_access': (I, [P, I]),
        'lg_get_tuning': (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class LgError(RuntimeError):
    def __init__(self, code, where):
        msg = load().lg_strerror(code).decode()
        super().__init__('%s failed: %s (%d)' % (where, msg, code))
        self.code = code


def _check(code, where):
    if code != LG_OK:
        raise LgError(code, where)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_grid(ndim, n, bc, h=(1.0, 1.0, 1.0), curvilinear=False, wall_T=None):
    """wall_T[d] = (lo, hi): wall temperatures of BC_NOSLIP_ISOTHERMAL faces."""
    g = LgGrid()
    for d, w in enumerate(wall_T or []):
        g.wall_T[d][0], g.wall_T[d][1] = float(w[0]), float(w[1])
    g.ndim = ndim
    n = tuple(n) + (1,) * (3 - len(n))
    for d in range(3):
        g.n[d] = int(n[d])
        g.h[d] = float(h[d]) if d < len(h) else 1.0
        lo, hi = bc[d] if d < len(bc) else (BC_TRANSMISSIVE, BC_TRANSMISSIVE)
        g.bc[d][0] = int(lo)
        g.bc[d][1] = int(hi)
    g.ng = 5
    g.curvilinear = 1 if curvilinear else 0
    return g


def make_gas(gamma=1.4, Re=1.0, Pr=0.72, Mref=1.0, suth=110.4 / 108.0, viscous=False):
    return LgGas(gamma, Re, Pr, Mref, suth, 1 if viscous else 0)


def make_opts(grad='E6', precision='fp64', cfl=0.2, omega_thr=0.01, mp_eps=1e-20, mp_alpha=4.0,
              C_mu=0.0, C_beta=1.75, C_kappa=0.01, hybrid_mode='percell', rho_thr=-1.0, p_thr=-1.0,
              dilate=3, seg=0, lad='E4', filter_alpha=0.49, filter_every_stage=False, time_scheme='rk3'):
    if time_scheme not in ('rk3', 'rk4'):
        raise ValueError('time_scheme: rk3 or rk4')
    return LgOpts(GRAD_C4 if grad == 'C4' else GRAD_E6, MIXED if precision == 'mixed' else FP64, cfl,
                  omega_thr, mp_eps, mp_alpha, C_mu, C_beta, C_kappa,
                  HYB_GLOBAL if hybrid_mode == 'global' else HYB_PERCELL, rho_thr, p_thr, dilate, seg,
                  LAD_C6 if lad == 'C6' else LAD_E4, float(filter_alpha), 1 if filter_every_stage else 0,
                  1 if time_scheme == 'rk4' else 0)


def metrics_from_coords(grid, coords, metrics, stream=None):
    _check(load().lg_metrics_from_coords(ctypes.byref(grid), _ptr(coords), _ptr(metrics), _stream(stream)),
           'lg_metrics_from_coords')


def metrics_from_coords_noalloc(grid, coords, metrics, stream=None):
    _check(load().lg_metrics_from_coords_noalloc(ctypes.byref(grid), _ptr(coords), _ptr(metrics), _stream(stream)),
           'lg_metrics_from_coords_noalloc')


class Context:
    """One grid + gas + scheme options; owns the library context and its workspace."""

    def __init__(self, grid, gas, opts, metrics=None, coords=None, stream=None):
        lib = load()
        self._lib = lib
        self.grid, self.gas, self.opts = grid, gas, opts
        self._keep = (metrics, coords)
        h = ctypes.c_void_p()
        _check(lib.lg_create(ctypes.byref(h), ctypes.byref(grid), _ptr(metrics), _ptr(coords),
                             ctypes.byref(gas), ctypes.byref(opts), _stream(stream)), 'lg_create')
        self.handle = h

    def close(self):
        if self.handle:
            self._lib.lg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self):
        return int(self._lib.lg_workspace_bytes(self.handle))

    def metrics_planar(self):
        return bool(self._lib.lg_metrics_planar(self.handle) == 1)

    def cgbr_rhs(self, Q, dQ):
        _check(self._lib.cgbr_rhs(self.handle, _ptr(Q), _ptr(dQ)), 'cgbr_rhs')

    def lad_rhs(self, Q, dQ):
        _check(self._lib.lad_rhs(self.handle, _ptr(Q), _ptr(dQ)), 'lad_rhs')

    def lad_filter(self, Q):
        _check(self._lib.lad_filter(self.handle, _ptr(Q)), 'lad_filter')

    def hybrid_rhs(self, Q, dQ, flags_in=None, flags_out=None):
        _check(self._lib.hybrid_rhs(self.handle, _ptr(Q), _ptr(dQ), _ptr(flags_in), _ptr(flags_out)),
               'hybrid_rhs')

    def rhs(self, scheme, Q, dQ, flags_in=None):
        if scheme == 'cgbr':
            self.cgbr_rhs(Q, dQ)
        elif scheme == 'lad':
            self.lad_rhs(Q, dQ)
        else:
            self.hybrid_rhs(Q, dQ, flags_in)

    def rk3_step(self, scheme, Q, t_end, t_dev):
        _check(self._lib.rk3_step(self.handle, SCHEMES[scheme], _ptr(Q), float(t_end), _ptr(t_dev)), 'rk3_step')

    def rk3_stage(self, scheme, stage, Un, Us, dt):
        _check(self._lib.lg_rk3_stage(self.handle, SCHEMES[scheme], int(stage), _ptr(Un), _ptr(Us), float(dt)),
               'lg_rk3_stage')

    def compute_dt(self, Q, dt_dev):
        _check(self._lib.lg_compute_dt(self.handle, _ptr(Q), _ptr(dt_dev)), 'lg_compute_dt')

    def prof_start(self, kernel_class=-1, max_launches=100000):
        k = kernel_class if isinstance(kernel_class, int) else KERNEL_CLASSES.index(kernel_class)
        _check(self._lib.lg_prof_start(self.handle, k, int(max_launches)), 'lg_prof_start')

    def prof_stop(self):
        n = len(KERNEL_CLASSES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int * n)()
        _check(self._lib.lg_prof_stop(self.handle, ms, cnt), 'lg_prof_stop')
        return {KERNEL_CLASSES[k]: (ms[k], cnt[k]) for k in range(n) if cnt[k]}

    def prof_stop_launches(self, cap=100000):
        """(per-class {name: (ms, launches)}, [(class name, ms) of each timed launch])."""
        n = len(KERNEL_CLASSES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int * n)()
        each = (ctypes.c_float * cap)()
        ecls = (ctypes.c_int * cap)()
        got = ctypes.c_int(0)
        _check(self._lib.lg_prof_stop_launches(self.handle, ms, cnt, each, ecls, int(cap), ctypes.byref(got)),
               'lg_prof_stop_launches')
        return ({KERNEL_CLASSES[k]: (ms[k], cnt[k]) for k in range(n) if cnt[k]},
                [(KERNEL_CLASSES[ecls[i]], float(each[i])) for i in range(got.value)])

    def set_tuning(self, seg=0, pcr_blocks=0, zc=0):
        _check(self._lib.lg_set_tuning(self.handle, int(seg), int(pcr_blocks), int(zc)), 'lg_set_tuning')

    def set_tile_shape(self, zm_width=0, line_batch=0):
        _check(self._lib.lg_set_tile_shape(self.handle, int(zm_width), int(line_batch)), 'lg_set_tile_shape')

    def get_tile_shape(self):
        w, b = ctypes.c_int(0), ctypes.c_int(0)
        _check(self._lib.lg_get_tile_shape(self.handle, ctypes.byref(w), ctypes.byref(b)), 'lg_get_tile_shape')
        return w.value, b.value

    def set_line_tiles(self, mask=-1):
        _check(self._lib.lg_set_line_tiles(self.handle, int(mask)), 'lg_set_line_tiles')

    def get_line_tiles(self):
        return int(self._lib.lg_get_line_tiles(self.handle))

    def set_generic_access(self, generic=True):
        """generic: True (every fallback), False (the defaults) or the bit mask of
        lg_set_generic_access (1 addressing and node pairs, 2 general geometry)."""
        mask = (3 if generic else 0) if isinstance(generic, bool) else int(generic)
        _check(self._lib.lg_set_generic_access(self.handle, mask), 'lg_set_generic_access')

    def get_tuning(self):
        a, b, z = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        _check(self._lib.lg_get_tuning(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(z)),
               'lg_get_tuning')
        return a.value, b.value, z.value

    def switch_stats(self, reset=False):
        """(hybrid stages, stages with a troubled node) since creation or the last reset."""
        a, b = ctypes.c_int(0), ctypes.c_int(0)
        _check(self._lib.lg_switch_stats(self.handle, ctypes.byref(a), ctypes.byref(b), 1 if reset else 0),
               'lg_switch_stats')
        return a.value, b.value

    def poll_status(self):
        n = ctypes.c_int(0)
        code = self._lib.lg_poll_status(self.handle, ctypes.byref(n))
        if code not in (LG_OK, LG_ENONPHYS):
            _check(code, 'lg_poll_status')
        return n.value


class LgDFSpec(ctypes.Structure):
    _fields_ = [('ny', ctypes.c_int), ('nz', ctypes.c_int), ('dy', ctypes.c_void_p), ('y', ctypes.c_void_p),
                ('dz', ctypes.c_double), ('y_lim', ctypes.c_double), ('Iy', (ctypes.c_double * 2) * 3),
                ('Iz', ctypes.c_double * 3), ('Ix', ctypes.c_double * 3), ('U_ref', ctypes.c_double),
                ('mean', ctypes.c_void_p), ('rey', ctypes.c_void_p), ('M_sra', ctypes.c_double),
                ('p', ctypes.c_double)]


class DFInflow:
    """Digital-filter inflow generator of a context (lg_df_*): the profile arrays are numpy
    FP64 arrays over the ny inflow rows (mean: rho, U, V, T; rey: R11, R21, R22, R33)."""

    def __init__(self, ctx, dy, y, dz, y_lim, Iy, Iz, Ix, U_ref, mean, rey, M_sra, p):
        import numpy as np
        lib = load()
        self._lib = lib
        self.ctx = ctx
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (dy, y, mean, rey)]
        self._arrs = arrs
        spec = LgDFSpec()
        spec.ny = int(arrs[0].size)
        spec.nz = int(ctx.grid.n[2]) if ctx.grid.ndim == 3 else 1
        spec.dy, spec.y = arrs[0].ctypes.data, arrs[1].ctypes.data
        spec.dz, spec.y_lim = float(dz), float(y_lim)
        for c in range(3):
            spec.Iy[c][0], spec.Iy[c][1] = float(Iy[c][0]), float(Iy[c][1])
            spec.Iz[c], spec.Ix[c] = float(Iz[c]), float(Ix[c])
        spec.U_ref = float(U_ref)
        spec.mean, spec.rey = arrs[2].ctypes.data, arrs[3].ctypes.data
        spec.M_sra, spec.p = float(M_sra), float(p)
        h = ctypes.c_void_p()
        _check(lib.lg_df_create(ctx.handle, ctypes.byref(spec), ctypes.byref(h)), 'lg_df_create')
        self.handle = h

    def random_count(self):
        n = ctypes.c_longlong(0)
        _check(self._lib.lg_df_random_count(self.handle, ctypes.byref(n)), 'lg_df_random_count')
        return n.value

    def update(self, rnd, Q, dt=-1.0, first=False):
        _check(self._lib.lg_df_update(self.handle, _ptr(rnd), _ptr(Q), float(dt), 1 if first else 0),
               'lg_df_update')

    def close(self):
        if self.handle:
            self._lib.lg_df_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent problems advanced ``nsteps`` RK3 steps per graph launch."""

    def __init__(self, contexts, Qs, ts, t_ends, nsteps, scheme):
        lib = load()
        self._lib = lib
        n = len(contexts)
        H = (ctypes.c_void_p * n)(*[c.handle for c in contexts])
        Qp = (ctypes.c_void_p * n)(*[q.data_ptr() for q in Qs])
        Tp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])
        TE = (ctypes.c_double * n)(*[float(x) for x in t_ends])
        self._keep = (contexts, Qs, ts, H, Qp, Tp, TE)
        h = ctypes.c_void_p()
        _check(lib.lg_batch_create(ctypes.byref(h), ctypes.cast(H, ctypes.c_void_p), ctypes.cast(Qp, ctypes.c_void_p),
                                   ctypes.cast(Tp, ctypes.c_void_p), ctypes.cast(TE, ctypes.c_void_p), n,
                                   int(nsteps), SCHEMES[scheme]), 'lg_batch_create')
        self.handle = h

    def run(self):
        _check(self._lib.lg_batch_run(self.handle), 'lg_batch_run')

    def close(self):
        if self.handle:
            self._lib.lg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
