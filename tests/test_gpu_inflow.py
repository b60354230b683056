"""GPU parity of the digital-filter inflow generator (lg_df_*; reading R33, Sec. 4's inflow)
against the oracle: the same normal numbers in, the whole state compared after successive
updates (first, explicit dt, the context's device dt)."""
import numpy as np
import pytest

import gpu_util as U
from oracle import inflow as DF, rhs as orhs
from paper_2511_18042_amd import cases, lgbr

pytestmark = pytest.mark.gpu

FX, NS, P, T = cases.FIXED, cases.NOSLIP, cases.PERIODIC, cases.TRANSMISSIVE


def _case(ndim):
    if ndim == 3:
        c = cases.periodic_case(3, (24, 20, 16))
        c.bc = [(FX, T), (NS, T), (P, P)]
    else:
        c = cases.periodic_case(2, (24, 20))
        c.bc = [(FX, T), (NS, T)]
    cases.random_smooth_state(c, seed=7)
    return c


def _profiles(c):
    ny, h = c.n[1], c.h[1]
    y = (np.arange(ny) + 0.5) * h
    dy = np.full(ny, h) * (1.0 + 0.3 * np.arange(ny) / ny)      # non-uniform spacings
    mean = np.stack([1.0 + 0.2 * y, 0.3 + 0.7 * y, 0.01 * y, 1.1 - 0.1 * y])
    f = np.clip(1.0 - y, 0.0, None) * (1.0 - np.exp(-y / 0.1))
    R11, R22, R33 = (0.1 * f) ** 2, (0.06 * f) ** 2, (0.08 * f) ** 2
    R21 = -0.4 * np.sqrt(R11 * R22)
    return dict(dy=dy, y=y, dz=c.h[2] if c.ndim == 3 else 1.0, y_lim=0.3,
                Iy=[(0.13, 0.23), (0.17, 0.3), (0.1, 0.13)], Iz=[0.15, 0.15, 0.3], Ix=[0.7, 0.28, 0.28],
                U_ref=1.0, mean=mean, rey=np.stack([R11, R21, R22, R33]), M_sra=2.9, p=0.7)


def _oracle_spec(pr, gamma):
    return DF.DFSpec(pr['dy'], pr['y'], pr['dz'], pr['y_lim'], pr['Iy'], pr['Iz'], pr['Ix'], pr['U_ref'],
                     pr['mean'], pr['rey'], gamma, pr['M_sra'], pr['p'])


@pytest.mark.parametrize('ndim', [3, 2])
def test_inflow_updates_match_the_oracle(ndim):
    print('inflow', ndim, flush=True)
    torch = U.torch_mod()
    c = _case(ndim)
    gas = orhs.Gas(gamma=1.4)
    ctx, _ = U.gpu_context(c, gas, orhs.Opts())
    pr = _profiles(c)
    df = lgbr.DFInflow(ctx, **pr)
    spec = _oracle_spec(pr, gas.gamma)
    nz = c.n[2] if ndim == 3 else 1
    shape = (3, c.n[1] + 2 * spec.pad(), nz)
    assert df.random_count() == int(np.prod(shape))
    rng = np.random.default_rng(2024)
    g = U.oracle_grid(c)
    Qd = U.dev(c.Q)
    Qo = c.Q.copy()
    psi = None
    # the context's device dt: one RK3 step of a copy
    Qs = U.dev(c.Q)
    t = torch.zeros(1, dtype=torch.float64, device='cuda')
    ctx.rk3_step('cgbr', Qs, 10.0, t)
    torch.cuda.synchronize()
    dt_dev = float(t.item())
    for step, (dt, dt_o, first) in enumerate(((-1.0, 0.0, True), (0.013, 0.013, False), (-1.0, dt_dev, False))):
        r = rng.standard_normal(shape)
        df.update(U.dev(r), Qd, dt=dt, first=first)
        psi = DF.update(spec, Qo, g, psi, r, dt_o, first)
        torch.cuda.synchronize()
        got = Qd.cpu().numpy()
        for q in range(5):
            scale = max(np.max(np.abs(Qo[q])), 1e-300)
            err = np.max(np.abs(got[q] - Qo[q])) / scale
            assert err <= 1e-13, (ndim, step, q, err)
    df.close()
    ctx.close()


def test_inflow_argument_checks():
    c = _case(3)
    gas = orhs.Gas(gamma=1.4)
    ctx, _ = U.gpu_context(c, gas, orhs.Opts())
    pr = _profiles(c)
    bad = dict(pr, dy=pr['dy'][:-1], y=pr['y'][:-1], mean=pr['mean'][:, :-1], rey=pr['rey'][:, :-1])
    with pytest.raises(lgbr.LgError):
        lgbr.DFInflow(ctx, **bad)                          # rows do not match the grid
    neg = pr['rey'].copy()
    neg[0, 3] = -1e-3
    with pytest.raises(lgbr.LgError):
        lgbr.DFInflow(ctx, **dict(pr, rey=neg))            # negative normal stress
    with pytest.raises(lgbr.LgError):
        lgbr.DFInflow(ctx, **dict(pr, U_ref=0.0))
    ctx.close()
    c.bc = [(T, T), (NS, T), (P, P)]                       # the inflow face must be FIXED
    ctx, _ = U.gpu_context(c, gas, orhs.Opts())
    with pytest.raises(lgbr.LgError):
        lgbr.DFInflow(ctx, **pr)
    ctx.close()
