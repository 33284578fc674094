"""Write the quenched synthetic glasses the parity tests start from.

Calls only the CPU oracle and the seeded input generator: uniform random
positions (aqs_synth.uniform_glass_start, seed words [2507, 20802, tag,
replica]) minimised by the oracle's FIRE to max|F| < 1e-10, then certified
by the oracle's own force evaluation.  Run from the repository root:

    python tests/data/make_inputs.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import aqs_synth as S  # noqa: E402
import oracle as O  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# (name, dim, n, seed words); the paper's sample uses its own potential and
# cell (Sec. 2.2, aqs_synth.paper_sample_start)
GLASSES = [
    ("glass2d_256", 2, 256, (1, 0)),
    ("glass2d_1000", 2, 1000, (11, 0)),
    ("glass2d_1000b", 2, 1000, (11, 1)),
    ("glass3d_1500", 3, 1500, (13, 0)),
    ("glass2d_4096", 2, 4096, (12, 0)),
    ("glass3d_8192", 3, 8192, (14, 0)),
    ("paper2d_400", 2, 400, (15, 0)),
]

QUENCH = O.FireParams(dt0=0.005, dt_max=0.03, f_dec=0.9, alpha0=0.2, f_alpha=0.95, n_delay=5,
                      f_inc=1.2, ftol=1e-10, max_iter=2_000_000)


def make(name, dim, n, seed):
    path = os.path.join(HERE, name + ".npz")
    if name.startswith("paper"):
        s, pot = S.paper_sample_start(*seed), O.paper_binary()
    else:
        s, pot = S.uniform_glass_start(dim, n, *seed), O.kob_andersen()
    H = O.box_matrix(dim, s.L, 0.0)
    t = time.time()
    r = O.fire(s.pos, s.types, H, pot, QUENCH)
    if r.status != O.CONVERGED:
        raise RuntimeError(f"{name}: quench did not converge (status {r.status})")
    fmax = O.max_force(r.pos, s.types, H, pot)
    assert fmax < 1e-10, fmax
    np.savez(path, pos=r.pos, types=s.types, L=s.L, dim=dim, energy=r.E, iters=r.iters,
             seed=np.array(seed))
    print(f"{name}: {r.iters} FIRE iterations, E/N = {r.E / n:.12f}, max|F| = {fmax:.3e}, "
          f"{time.time() - t:.1f} s", flush=True)


if __name__ == "__main__":
    only = sys.argv[1:]
    for g in GLASSES:
        if not only or g[0] in only:
            make(*g)
