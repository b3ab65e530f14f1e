"""Writes batch_grain30_map1.npz: the oracle's first iteration map of batch
grain 30, the largest of the seeded 64-grain batch (464x464 cells, h = 0.2,
128 angles, 128 Ozaki poles, s-wave, outer shape minus two holes, no
screening), from its seeded starting field with A_ind = 0 and bulk start
values (Alg. 1), evaluated at sampled cells only (Grain.iterate_cells):
16 seeded cells on the edges of the grain (outer boundary and holes) and 8
seeded interior cells.  Stores Delta_new and j there.

Calls only the oracle (and the seeded inputs).  Run from the repository
root: python tests/golden/make_batch_grain30.py  (a few minutes on one core).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

from helpers import oracle_grain  # noqa: E402
import importlib.util  # noqa: E402

GRAIN = 30
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_grain%d_map1.npz" % GRAIN)


def _workloads():
    spec = importlib.util.spec_from_file_location("_wl", os.path.join(ROOT, "paper_2205_15000_amd", "workloads.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def sample_cells(mask, seed=31, n_edge=16, n_interior=8):
    ny, nx = mask.shape
    pad = np.zeros((ny + 2, nx + 2), dtype=bool)
    pad[1:-1, 1:-1] = mask
    inner = pad[:-2, 1:-1] & pad[2:, 1:-1] & pad[1:-1, :-2] & pad[1:-1, 2:]
    rng = np.random.default_rng(seed)
    edge = np.sort(rng.choice(np.flatnonzero(mask & ~inner), n_edge, replace=False))
    interior = np.sort(rng.choice(np.flatnonzero(mask & inner), n_interior, replace=False))
    return np.concatenate([edge, interior]), n_edge


def main():
    wl = _workloads()
    sp = wl.batch_specs(64)[GRAIN]
    t0 = time.time()
    og = oracle_grain(sp)
    cells, n_edge = sample_cells(og.mask)
    delta = wl.batch_initial_delta(sp, GRAIN)
    A = np.zeros((2, sp["ny"], sp["nx"]))
    dn, j = og.iterate_cells(delta, A, cells)
    np.savez_compressed(OUT, cells=cells, n_edge=n_edge, delta_new=dn, j=j)
    print("wrote %s in %.0f s" % (OUT, time.time() - t0))


if __name__ == "__main__":
    main()
