"""lg_metrics_from_coords_noalloc: the metrics entry point for callers that cannot allocate
(its scratch lives in a static device array) gives bitwise the results of
lg_metrics_from_coords, on two calls in a row (the second on a smaller grid, so it runs on
a scratch that still holds the first call's values), and refuses grids larger than its
scratch before enqueueing anything."""
import ctypes

import numpy as np
import pytest

import gpu_util as U
from paper_2511_18042_amd import cases, lgbr

pytestmark = pytest.mark.gpu


def _metrics_both_ways(c):
    torch = U.torch_mod()
    g = lgbr.make_grid(c.ndim, c.n, c.bc, c.h, curvilinear=True)
    coords = U.dev(c.coords)
    ref = torch.zeros((10,) + tuple(c.shape), dtype=torch.float64, device='cuda')
    out = torch.full_like(ref, float('nan'))
    lgbr.metrics_from_coords(g, coords, ref)
    lgbr.metrics_from_coords_noalloc(g, coords, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_metrics_equal_the_allocating_entry_point_twice():
    first = cases.periodic_case(3, (20, 16, 12), curvilinear=True, amp=0.08)
    second = cases.periodic_case(2, (24, 16), curvilinear=True, amp=0.1)
    assert np.prod(second.shape) < np.prod(first.shape)
    for c in (first, second):
        ref, out = _metrics_both_ways(c)
        assert np.array_equal(ref, out), np.nanmax(np.abs(ref - out))
        assert np.abs(ref[9]).max() > 0.0


def test_noalloc_metrics_refuse_grids_beyond_the_scratch():
    lib = lgbr.load()
    dummy = ctypes.c_void_p(256)                    # never dereferenced: refused first
    g = lgbr.make_grid(2, (1100, 1000), [(0, 0), (0, 0)], curvilinear=True)
    assert 1110 * 1010 > (1 << 20)
    assert lib.lg_metrics_from_coords_noalloc(ctypes.byref(g), dummy, dummy, None) == lgbr.LG_EUNSUPPORTED
    g = lgbr.make_grid(2, (1014, 1014), [(0, 0), (0, 0)], curvilinear=True)
    assert 1024 * 1024 == (1 << 20)                 # the largest accepted padded grid
    torch = U.torch_mod()
    coords = torch.zeros((3, 1, 1024, 1024), dtype=torch.float64, device='cuda')
    ii = torch.arange(1024, dtype=torch.float64, device='cuda')
    coords[0] = ii[None, None, :] * 0.01
    coords[1] = ii[None, :, None] * 0.02
    out = torch.zeros((10, 1, 1024, 1024), dtype=torch.float64, device='cuda')
    lgbr.metrics_from_coords_noalloc(g, coords, out)
    torch.cuda.synchronize()
    J = out[9, 0, 2:-2, 2:-2].cpu().numpy()
    assert np.allclose(J, 1.0 / (0.01 * 0.02), rtol=1e-12)
