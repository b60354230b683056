"""Build liblgbr.so (HIP for gfx950) in-tree.

    python -m paper_2511_18042_amd.build

Every HIP translation unit is compiled with hipcc for gfx950 only; packed-FP32
instructions are disabled (-Xclang -target-feature -Xclang -packed-fp32-ops).  The
objects are linked into ``paper_2511_18042_amd/liblgbr.so``.  Always recompiles.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, 'csrc')
BUILD = os.path.join(PKG, '_build')
LIB = os.path.join(PKG, 'liblgbr.so')
SOURCES = ['k_basic.hip', 'k_grad.hip', 'k_lad.hip', 'k_sweep.hip', 'k_compact.hip', 'k_inflow.hip', 'noalloc.hip',
           'lgbr.cpp']
ARCH = 'gfx950'


def hipcc():
    h = shutil.which('hipcc') or '/opt/rocm/bin/hipcc'
    if not os.path.exists(h):
        raise RuntimeError('hipcc not found')
    return h


def flags():
    return ['-O3', '-std=c++17', '-fPIC', '--offload-arch=' + ARCH,
            '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
            '-I', os.path.join(ROOT, 'include'), '-I', CSRC]


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + '.o')
    cmd = [hipcc(), '-c', os.path.join(CSRC, src), '-o', obj] + flags()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError('compile failed: %s\n%s\n%s' % (' '.join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + '.tmp'
    cmd = [hipcc(), '-shared', '-fPIC', '--offload-arch=' + ARCH, '-o', tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError('link failed: %s\n%s' % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print('built', LIB)
    return LIB


if __name__ == '__main__':
    build(verbose=True)
    sys.exit(0)
