"""Writes tests/golden/c4_full_samples.npz: the CPU oracle's solution of the
full 3-D workload (64 x 224 x 80 cells, 4^3 subdomains, overlap 2,
piecewise-constant spaces, 3 smoothing steps) at 4096 seeded sample cells
(pressure and the six face velocities of each), with the norms of the whole
fields.  Calls only the oracle; takes several minutes on one core.

    python tests/golden/make_c4_samples.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from inputs import make_workload  # noqa: E402
from oracle import mrcm  # noqa: E402


def main():
    wl = make_workload("c4")
    t = time.time()
    s = mrcm.solve(wl)
    p = s.pressure()
    f = s.flux()
    rng = np.random.default_rng(20404)
    idx = np.sort(rng.choice(wl.ncells, size=4096, replace=False))
    np.savez_compressed(os.path.join(HERE, "c4_full_samples.npz"), cells=idx.astype(np.int64),
                        pressure=p[idx], flux=f[idx], pressure_norm=np.linalg.norm(p),
                        flux_norm=np.linalg.norm(f), ncells=wl.ncells, nsub=s.part.nsub,
                        n_unknowns=int(s.offset[-1]))
    print("c4 oracle: %.0f s, %d unknowns" % (time.time() - t, int(s.offset[-1])))


if __name__ == "__main__":
    main()
