"""Writes tests/golden/shu_osher_ref_16000.npz: the FP64 oracle's MIG4 C-GBR solution of the
Shu-Osher problem (Sec. 3.1) on 16000 cells at t = 1.8, CFL 0.2 -- the reference for the
L1(rho) errors of the 2000-cell runs (the paper's own reference solution is not available).
Calls only the oracle.  Run: python tests/golden/make_shu_osher_reference.py [n]
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import grid as gr, rhs as R  # noqa: E402
from paper_2511_18042_amd import cases  # noqa: E402


def fingerprint(n=400, steps=40):
    """The oracle's MIG4 C-GBR density after ``steps`` RK3 steps of the same problem on ``n``
    cells: stored beside the reference so that a test can tell whether the oracle arithmetic
    that produced it has changed since (a file hash would also change with unrelated edits)."""
    c = cases.shu_osher(n)
    g = gr.Grid(c.ndim, c.n, c.bc, c.h)
    M = gr.node_metrics(g)
    Q, t = c.Q.copy(), 0.0
    for _ in range(steps):
        Q, t, _, _ = R.rk3_step(Q, t, c.t_end, g, R.Gas(gamma=1.4), R.Opts(grad='C4', cfl=0.2), 'cgbr', M)
    inner = (slice(None),) + g.interior()
    return R.primitives(Q[inner], 1.4)[0, 0, 0, :]


def oracle_hash():
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, 'oracle'))):
        if f.endswith('.py'):
            h.update(open(os.path.join(ROOT, 'oracle', f), 'rb').read())
    return h.hexdigest()


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 16000
    c = cases.shu_osher(n)
    g = gr.Grid(c.ndim, c.n, c.bc, c.h)
    M = gr.node_metrics(g)
    gas = R.Gas(gamma=1.4)
    opts = R.Opts(grad='C4', cfl=0.2)
    Q, t, steps = c.Q.copy(), 0.0, 0
    t0 = time.time()
    while t < c.t_end:
        Q, t, dt, bad = R.rk3_step(Q, t, c.t_end, g, gas, opts, 'cgbr', M)
        assert bad == 0
        steps += 1
        if steps % 2000 == 0:
            print('step %d t %.4f (%.0f s)' % (steps, t, time.time() - t0), flush=True)
    inner = (slice(None),) + g.interior()
    W = R.primitives(Q[inner], 1.4)[:, 0, 0, :]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), 'shu_osher_ref_%d.npz' % n)
    np.savez_compressed(out, rho=W[0], u=W[1], p=W[4], t=t, steps=steps, oracle_sha256=oracle_hash(),
                        fingerprint_rho=fingerprint())
    print('wrote', out, 'steps', steps)


if __name__ == '__main__':
    main()
