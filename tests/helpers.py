"""Test helpers: build the oracle's grain from a workload description."""
import numpy as np

from oracle import geometry as geo, scf


def oracle_shapes(sp):
    out = []
    for sh in sp["shapes"]:
        add = sh.get("add", True)
        if sh["kind"] == "disc":
            out.append(geo.Disc(sh["cx"], sh["cy"], sh["radius"], add))
        elif sh["kind"] == "regular_polygon":
            out.append(geo.regular_polygon(sh["cx"], sh["cy"], sh["n_edges"], sh["side"], sh.get("rotation", 0.0), add))
        elif sh["kind"] == "mask":
            grid = geo.Grid(sp["nx"], sp["ny"], sp["h"], sp.get("x0"), sp.get("y0"))
            out.append(geo.MaskShape(sh["mask"], grid, add))
        else:
            out.append(geo.Polygon(sh["vx"], sh["vy"], add))
    return out


def oracle_grain(sp):
    return scf.Grain(sp["nx"], sp["ny"], sp["h"], oracle_shapes(sp), sp["n_theta"], sp["n_poles"], sp["t"],
                     components=sp["components"], crystal_rotation=sp.get("crystal_rotation", 0.0),
                     kappa=sp.get("kappa", 0.0), flux_quanta=sp.get("flux_quanta", 0.0),
                     gauge=sp.get("gauge", "symmetric"), charge_sign=sp.get("charge_sign", -1),
                     x0=sp.get("x0"), y0=sp.get("y0"))


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0)
