"""Writes adjoint_<grain>.npz: gradients of one iteration map of the oracle
(Alg. 1, boundary values frozen at those of a first map from bulk starts)
for two small grains, by fourth-order Richardson central differences, at
sampled elements of the inputs, for two losses taken separately:
  L1 = Omega_total (the Eilenberger free energy of the map, Sec. II),
  L2 = h^2 sum over grain cells of |j - j_t|^2 with a seeded target
       j_t = j + N(0, (0.01 max|j|)^2) on grain cells.
The derivative of L with respect to a real input x is
  (8 [L(x + s) - L(x - s)] - [L(x + 2s) - L(x - 2s)]) / (12 s),
which is exact for polynomials of degree four; s = 1e-3.  Elements: 12
seeded grain cells x {Re Delta, Im Delta (a seeded component), A_x, A_y}.

Calls only the oracle (and the seeded inputs).  Run from the repository
root: python tests/golden/make_adjoint_small.py  (a few minutes).
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

from helpers import oracle_grain  # noqa: E402
import importlib.util  # noqa: E402

GRAINS = ("small_polygon_landau", "small_holed_mixed")
STEP = 1e-3
KINDS = ("re", "im", "ax", "ay")


def _workloads():
    spec = importlib.util.spec_from_file_location("_wl", os.path.join(ROOT, "paper_2205_15000_amd", "workloads.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def losses(og, delta, A, bc, jt):
    out = og.iterate(delta, A, bc)
    h2 = og.grid.h ** 2
    j = out["j"]
    m = og.mask
    return out["omega_total"], h2 * float(np.sum((j[:, m] - jt[:, m]) ** 2))


def perturbed(delta, A, comp, cell, kind, s):
    d = delta.copy()
    a = A.copy()
    if kind == "re":
        d.reshape(d.shape[0], -1)[comp, cell] += s
    elif kind == "im":
        d.reshape(d.shape[0], -1)[comp, cell] += 1j * s
    else:
        a.reshape(2, -1)[0 if kind == "ax" else 1, cell] += s
    return d, a


def main():
    wl = _workloads()
    for name in GRAINS:
        sp = wl.spec(name)
        og = oracle_grain(sp)
        delta = wl.initial_delta(name, sp)
        A = wl.initial_A(name, sp)
        bc = og.iterate(delta, A)["bc"]
        j0 = og.iterate(delta, A, bc)["j"]
        rng = np.random.default_rng(41)
        jt = np.where(og.mask[None], j0 + 0.01 * np.abs(j0).max() * rng.standard_normal(j0.shape), 0.0)
        cells = np.sort(rng.choice(np.flatnonzero(og.mask), 12, replace=False))
        comps = rng.integers(og.ncomp, size=len(cells))
        g1 = np.zeros((len(cells), len(KINDS)))
        g2 = np.zeros_like(g1)
        for ic, (c, comp) in enumerate(zip(cells, comps)):
            for ik, kind in enumerate(KINDS):
                vals = {}
                for mult in (1, -1, 2, -2):
                    vals[mult] = losses(og, *perturbed(delta, A, comp, c, kind, mult * STEP), bc, jt)
                for which, gout in ((0, g1), (1, g2)):
                    gout[ic, ik] = (8.0 * (vals[1][which] - vals[-1][which])
                                    - (vals[2][which] - vals[-2][which])) / (12.0 * STEP)
            print(name, "cell", ic + 1, "of", len(cells), flush=True)
        out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_%s.npz" % name)
        np.savez_compressed(out, cells=cells, comps=comps, kinds=np.array(KINDS), step=STEP, jt=jt,
                            grad_omega=g1, grad_jloss=g2)
        print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
