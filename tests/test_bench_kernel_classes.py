"""Every library kernel timed on the stepping path has a class in bench.py's rocprofv3
summaries, the classes the library's own launch timing uses (lg_prof_*), so a kernel trace
of a step is attributed in full.  Set-up kernels (metrics, conversions, inflow generation,
one-thread resets) are left out."""
import glob
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import bench  # noqa: E402

SETUP = {'k_convert', 'k_df_eta', 'k_df_ghosts', 'k_df_zeta', 'k_hyb_init', 'k_lad_dx', 'k_metric_inner',
         'k_metric_outer', 'k_planar_dev', 'k_set_dt', 'k_zero_lcount', 'k_zero_status'}


def _kernels():
    names = set()
    for f in glob.glob(os.path.join(os.path.dirname(HERE), 'paper_2511_18042_amd', 'csrc', '*.hip')):
        src = open(f).read()
        for m in re.finditer(r'__global__\s+void\s+(?:__launch_bounds__\([^)]*\)\s*)?'
                             r'(?:__attribute__\(\([^)]*\)\)\)\s*)?(k_\w+)\s*\(', src):
            names.add(m.group(1))
    return names


def test_every_stepping_kernel_has_a_class():
    names = _kernels()
    assert {'k_lad_sweep', 'k_c6_faces_seg', 'k_grad_part', 'k_c6_seg_check'} <= names
    # k_line_tiles is classified by its template's system kind (next test)
    missing = sorted(n for n in names - SETUP - {'k_line_tiles'}
                     if bench.kernel_class('void lg::%s(lg::Prob const*)' % n) is None)
    assert missing == []


def test_line_tile_kinds():
    # k_line_tiles<R, KIND, NT>: gradients (C6, MIG4), faces, filter
    got = [bench.kernel_class('void lg::k_line_tiles<float, %d, 512>(lg::Prob const*, lg::TileArgs)' % k)
           for k in range(4)]
    assert got == ['grad_c4', 'c6_faces', 'filter', 'grad_c4']
