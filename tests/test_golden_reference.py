"""The stored 16000-cell Shu-Osher reference (tests/golden/make_shu_osher_reference.py) must
be one the current oracle reproduces: its fingerprint -- the oracle's MIG4 density after 40
steps on 400 cells, written beside the reference -- is recomputed here (CPU)."""
import importlib.util
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
REF = os.path.join(HERE, 'golden', 'shu_osher_ref_16000.npz')


def _generator():
    spec = importlib.util.spec_from_file_location('make_ref', os.path.join(HERE, 'golden',
                                                                           'make_shu_osher_reference.py'))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_shu_osher_reference_matches_the_current_oracle():
    z = np.load(REF)
    if 'fingerprint_rho' not in z.files:
        pytest.skip('the stored reference predates its fingerprint')
    fp = _generator().fingerprint()
    assert np.max(np.abs(fp - z['fingerprint_rho'])) <= 1e-13 * np.max(np.abs(fp))
