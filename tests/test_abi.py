"""The C-ABI library loads and exports every entry point that include/lgbr.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2511_18042_amd import lgbr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, 'include', 'lgbr.h')).read()
    src = re.sub(r'/\*.*?\*/', '', src, flags=re.S)
    names = re.findall(r'^\s*(?:lg_status|void|size_t|int|const char\*)\s+\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(',
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ('cgbr_rhs', 'lad_rhs', 'hybrid_rhs', 'rk3_step', 'lg_create', 'lg_batch_create'):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(lgbr.LIB_PATH):
        pytest.skip('liblgbr.so not built')
    lib = ctypes.CDLL(lgbr.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == set(lgbr.EXPORTS)


def test_binding_struct_layout_matches_header(tmp_path):
    """Field offsets and sizes of the ctypes structs equal those the C compiler gives the
    header's structs."""
    import shutil
    import subprocess
    cc = shutil.which('gcc') or shutil.which('cc')
    if cc is None:
        pytest.skip('no C compiler')
    structs = {'lg_grid': lgbr.LgGrid, 'lg_gas': lgbr.LgGas, 'lg_opts': lgbr.LgOpts, 'lg_df_spec': lgbr.LgDFSpec}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lgbr.h"', 'int main(void) {']
    for cname, cls in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines.append('return 0; }')
    src = tmp_path / 'layout.c'
    src.write_text('\n'.join(lines))
    exe = tmp_path / 'layout'
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), 'include')
    subprocess.run([cc, '-I', inc, str(src), '-o', str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split('\n')
    got = {}
    for line in out:
        if line.strip():
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, cls in structs.items():
        assert got[(cname, 'size')] == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert got[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])


def test_strerror_and_argument_errors_without_gpu():
    if not os.path.exists(lgbr.LIB_PATH):
        pytest.skip('liblgbr.so not built')
    lib = lgbr.load()
    assert lib.lg_strerror(lgbr.LG_EINVAL) == b'invalid argument'
    # invalid arguments are rejected before any device work
    h = ctypes.c_void_p()
    g = lgbr.make_grid(2, (3, 40), [(0, 0), (0, 0)], (0.1, 0.1, 1.0))      # n < 5
    code = lib.lg_create(ctypes.byref(h), ctypes.byref(g), None, None, ctypes.byref(lgbr.make_gas()),
                         ctypes.byref(lgbr.make_opts()), None)
    assert code == lgbr.LG_EINVAL
    g = lgbr.make_grid(2, (30, 40), [(0, 1), (1, 1)], (0.1, 0.1, 1.0))     # periodic on one side only
    code = lib.lg_create(ctypes.byref(h), ctypes.byref(g), None, None, ctypes.byref(lgbr.make_gas()),
                         ctypes.byref(lgbr.make_opts()), None)
    assert code == lgbr.LG_EINVAL
    assert lib.cgbr_rhs(None, None, None) == lgbr.LG_EINVAL
    assert lib.lg_set_allocator(ctypes.c_void_p(1), None, None) == lgbr.LG_EINVAL
    assert lib.lg_set_generic_access(None, 1) == lgbr.LG_EINVAL
    assert lib.lg_set_line_tiles(None, -1) == lgbr.LG_EINVAL
