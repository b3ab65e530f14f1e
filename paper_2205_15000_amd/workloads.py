"""Seeded synthetic workloads: grain descriptions and starting fields.

This module holds inputs only (shapes, grids, parameters, seeded random
starting fields), none of the method's arithmetic; the tests, the smoke
check and the benchmark take their inputs from here so that the HIP path
and the CPU oracle see identical data.  The paper uses no public dataset:
its workloads are synthetic grains, which these recipes stand in for.

DELTA0 is the weak-coupling BCS gap at T = 0, pi exp(-gamma_E) k_B Tc, in
units of 2 pi k_B Tc: the scale of the starting amplitudes and tolerances.
"""
import math

import numpy as np

DELTA0 = 0.28072974178344257
# bulk d-wave gap at t = 0.1 with 64 poles and 64 angles, in units of DELTA0
# (root of the homogeneous gap equation; used only as a starting amplitude)
D_BULK_T01 = 0.8577177
# bulk s-wave gap at t = 0.5 with 16 poles, in units of DELTA0 (the same
# root; starting amplitude of the vortex demonstration)
S_BULK_T05 = 0.9568823
# bulk s-wave gap at t = 0.2 with 24 poles, in units of DELTA0 (starting
# amplitude of the screened annulus)
S_BULK_T02 = 0.9998739


def _disc(cx, cy, r, add=True):
    return {"kind": "disc", "cx": cx, "cy": cy, "radius": r, "add": add}


def _square(cx, cy, side, rotation=0.0, add=True):
    return {"kind": "regular_polygon", "cx": cx, "cy": cy, "n_edges": 4, "side": side,
            "rotation": rotation, "add": add}


def _blob_mask(nx=34, ny=30, h=0.5, seed=17):
    """Seeded non-convex cell mask: three Gaussian bumps minus a hole,
    thresholded, with a 2x2 checkerboard carved into its edge so that the
    contour has squares whose diagonal corners alone are inside."""
    rng = np.random.default_rng(seed)
    xs = -0.5 * nx * h + (np.arange(nx) + 0.5) * h
    ys = -0.5 * ny * h + (np.arange(ny) + 0.5) * h
    X, Y = np.meshgrid(xs, ys)
    f = np.zeros_like(X)
    for _ in range(3):
        cx, cy = rng.uniform(-2.5, 2.5, 2)
        f += np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * rng.uniform(3.0, 4.0) ** 2))
    hole = np.exp(-((X - 1.0) ** 2 + (Y + 0.5) ** 2) / (2 * 1.2 ** 2))
    m = (f - 1.2 * f.max() * hole) > 0.5
    # carve a checkerboard at the rightmost inside cell of the middle row
    j = ny // 2
    i = int(np.nonzero(m[j])[0].max())
    m[j, i], m[j, i - 1], m[j + 1, i], m[j + 1, i - 1] = False, True, True, False
    return m.astype(np.uint8)


SPECS = {
    # s-wave disc R = 10 xi0 on 32x32 (h = 0.625), 32 angles, 16 poles,
    # t = 0.5, no field (the small Picard case, 50 iterations)
    "s_disc_32": dict(nx=32, ny=32, h=0.625, shapes=[_disc(0, 0, 10.0)], n_theta=32, n_poles=16, t=0.5,
                      components=[("s", 1.0)], kappa=0.0, flux_quanta=0.0, gauge="symmetric", charge_sign=-1),
    # d-wave square of side 40 xi0 on 400x400 (h = 0.1) with crystal axes at
    # 45 degrees (four pair-breaking [110] edges), 64 angles, 64 poles,
    # t = 0.1, one flux quantum (symmetric gauge), kappa = 20, one vortex
    "d110_square_400": dict(nx=400, ny=400, h=0.1, shapes=[_square(0, 0, 40.0)], n_theta=64, n_poles=64,
                            t=0.1, components=[("dx2y2", 1.0)], crystal_rotation=0.125, kappa=20.0,
                            flux_quanta=1.0, gauge="symmetric", charge_sign=-1),
    # d-wave disc R = 20 xi0 on 200x200 (h = 0.2), 64 angles, 48 poles,
    # t = 0.2, two flux quanta, kappa = 20 (the differentiated map)
    "d_disc_200": dict(nx=200, ny=200, h=0.2, shapes=[_disc(0, 0, 20.0)], n_theta=64, n_poles=48, t=0.2,
                       components=[("dx2y2", 1.0)], kappa=20.0, flux_quanta=2.0, gauge="symmetric",
                       charge_sign=-1),
    # d-wave square of side 51.2 xi0 on 512x512 (h = 0.1), [110] edges,
    # t = 0.1, kappa = 100; LDOS with 256 angles
    "d110_square_512_ldos": dict(nx=512, ny=512, h=0.1, shapes=[_square(0, 0, 51.2)], n_theta=256, n_poles=64,
                                 t=0.1, components=[("dx2y2", 1.0)], crystal_rotation=0.125, kappa=100.0,
                                 flux_quanta=0.0, gauge="symmetric", charge_sign=-1),
    # the paper's demonstration (Sec. IV, the App. B configuration listing):
    # s-wave disc R = 15 xi0 at 20 points per xi0 (600 x 600, h = 0.05), 32
    # angles, t = 0.5, 1.5 flux quanta (symmetric gauge), penetration depth
    # 5 xi0, one vortex of winding -1 at the centre, no noise; 16 Ozaki poles
    # (their largest energy, 53 x 2 pi Tc, lies above the listing's cutoff
    # of 16)
    "swave_disc_vortex": dict(nx=600, ny=600, h=0.05, shapes=[_disc(0, 0, 15.0)], n_theta=32, n_poles=16, t=0.5,
                              components=[("s", 1.0)], kappa=5.0, flux_quanta=1.5, gauge="symmetric",
                              charge_sign=-1),
    # ---- small parity cases (several tiles, ragged tails, every option) ----
    # d-wave [110] square with field, finite kappa and an off-centre vortex
    "small_d110_field": dict(nx=40, ny=40, h=0.5, shapes=[_square(0, 0, 18.3)], n_theta=16, n_poles=8, t=0.3,
                             components=[("dx2y2", 1.0)], crystal_rotation=0.125, kappa=3.0, flux_quanta=1.5,
                             gauge="symmetric", charge_sign=-1),
    # disc with a square hole, s + d_xy components, solenoid gauge
    "small_holed_mixed": dict(nx=36, ny=36, h=0.5, shapes=[_disc(0, 0, 8.6), _square(1.3, 0.4, 4.0, 0.1, add=False)],
                              n_theta=24, n_poles=6, t=0.4, components=[("s", 1.0), ("dxy", 0.7)],
                              kappa=0.0, flux_quanta=0.6, gauge="solenoid", charge_sign=-1),
    # grain given by its cells only (marching-squares boundary), non-convex
    # with a hole and a saddle square; d-wave, field, finite kappa
    "small_mask_blob": dict(nx=34, ny=30, h=0.5, shapes=[{"kind": "mask", "mask": _blob_mask(), "add": True}],
                            n_theta=16, n_poles=6, t=0.4, components=[("dx2y2", 1.0)], crystal_rotation=0.1,
                            kappa=2.5, flux_quanta=0.7, gauge="symmetric", charge_sign=-1),
    # convex polygon, odd angle count (trapezoid weights), Landau gauge,
    # positive carriers, kappa for the A-solve, 5 poles (padded lanes)
    "small_polygon_landau": dict(nx=30, ny=26, h=0.45,
                                 shapes=[{"kind": "polygon", "vx": [-6.0, 5.5, 6.4, 0.5, -5.8],
                                          "vy": [-5.0, -5.4, 1.0, 5.5, 3.0], "add": True}],
                                 n_theta=15, n_poles=5, t=0.6, components=[("s", 1.0)], kappa=2.0,
                                 flux_quanta=0.8, gauge="landau", charge_sign=1),
}


def spec(name):
    s = dict(SPECS[name])
    s["shapes"] = [dict(sh) for sh in s["shapes"]]
    s["name"] = name
    return s


def centres(sp):
    """Cell centres x0 + (i + 1/2) h, y0 + (j + 1/2) h as [ny][nx] arrays."""
    nx, ny, h = sp["nx"], sp["ny"], sp["h"]
    x0 = sp.get("x0")
    y0 = sp.get("y0")
    x0 = -0.5 * nx * h if x0 is None else x0
    y0 = -0.5 * ny * h if y0 is None else y0
    xs = x0 + (np.arange(nx) + 0.5) * h
    ys = y0 + (np.arange(ny) + 0.5) * h
    return np.meshgrid(xs, ys)


def initial_delta(name, sp=None, seed=None):
    """Seeded starting order parameter, complex [ncomp][ny][nx]
    (values off the grain are ignored by the method)."""
    sp = sp or spec(name)
    nx, ny = sp["nx"], sp["ny"]
    X, Y = centres(sp)
    ncomp = len(sp["components"])
    if name == "s_disc_32":
        rng = np.random.default_rng(1 if seed is None else seed)
        u = rng.uniform(-0.05, 0.05, (ny, nx))
        return (DELTA0 * (1.0 + u))[None].astype(np.complex128)
    if name in ("d110_square_400", "d110_square_512_ldos"):
        rng = np.random.default_rng((2 if name == "d110_square_400" else 7) if seed is None else seed)
        xv, yv = rng.uniform(-5.0, 5.0, 2)
        phase = -np.arctan2(Y - yv, X - xv)
        return (D_BULK_T01 * DELTA0 * np.exp(1j * phase))[None].astype(np.complex128)
    if name == "swave_disc_vortex":
        # bulk amplitude with the phase of one vortex of winding -1 at the centre
        return (S_BULK_T05 * DELTA0 * np.exp(-1j * np.arctan2(Y, X)))[None].astype(np.complex128)
    if name == "d_disc_200":
        rng = np.random.default_rng(4 if seed is None else seed)
        u = rng.uniform(-0.05, 0.05, (ny, nx))
        return (DELTA0 * (0.8 + u))[None].astype(np.complex128)
    # small parity cases: a vortex plus complex noise per component
    rng = np.random.default_rng(11 if seed is None else seed)
    xv, yv = rng.uniform(-2.0, 2.0, 2)
    out = np.empty((ncomp, ny, nx), dtype=np.complex128)
    for c in range(ncomp):
        amp = DELTA0 * (0.9 if c == 0 else 0.3)
        noise = 0.05 * DELTA0 * (rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx)))
        out[c] = amp * np.exp(-1j * np.arctan2(Y - yv, X - xv) + 0.7j * c) + noise
    return out


def initial_A(name, sp=None, seed=None):
    """Starting induced vector potential [2][ny][nx]: zero for the paper
    workloads, a small smooth seeded field for the parity cases."""
    sp = sp or spec(name)
    nx, ny = sp["nx"], sp["ny"]
    if name in ("s_disc_32", "d110_square_400", "d_disc_200", "d110_square_512_ldos", "swave_disc_vortex"):
        return np.zeros((2, ny, nx))
    rng = np.random.default_rng(23 if seed is None else seed)
    X, Y = centres(sp)
    a, b, c, d = rng.uniform(0.1, 0.4, 4)
    return 0.02 * np.stack([np.sin(a * X + b * Y), np.cos(c * X - d * Y)])


def annulus_spec(kappa, flux_quanta, h=0.125, n_theta=64, n_poles=24):
    """The s-wave annulus of Sec. V.A: outer radius 25 xi0, inner radius
    10 xi0, centred in a square grid with 1 xi0 of margin (416 x 416 cells at
    h = 0.125), t = 0.2, symmetric gauge with flux_quanta through the annulus,
    penetration depth kappa xi0."""
    n = int(round(2 * 26.0 / h))
    return dict(nx=n, ny=n, h=h, shapes=[_disc(0, 0, 25.0), _disc(0, 0, 10.0, add=False)], n_theta=n_theta,
                n_poles=n_poles, t=0.2, components=[("s", 1.0)], kappa=kappa, flux_quanta=flux_quanta,
                gauge="symmetric", charge_sign=-1, name="swave_annulus")


def disc_spec(flux_quanta, R=25.0, h=0.125, n_theta=64, n_poles=24):
    """The unscreened s-wave disc of Sec. V.B (radius 25 xi0, t = 0.2,
    infinite penetration depth), centred in a square grid with 1 xi0 of
    margin (416 x 416 cells at h = 0.125), symmetric gauge with flux_quanta
    through the disc."""
    n = int(round(2 * (R + 1.0) / h))
    return dict(nx=n, ny=n, h=h, shapes=[_disc(0, 0, R)], n_theta=n_theta, n_poles=n_poles, t=0.2,
                components=[("s", 1.0)], kappa=0.0, flux_quanta=flux_quanta, gauge="symmetric",
                charge_sign=-1, name="swave_disc_unscreened")


def annulus_initial_delta(sp, winding):
    """Bulk amplitude at t = 0.2 with the phase winding 2 pi winding around
    the grid centre (the hole of the annulus, the vortex of the disc)."""
    X, Y = centres(sp)
    return (S_BULK_T02 * DELTA0 * np.exp(1j * winding * np.arctan2(Y, X)))[None].astype(np.complex128)


def vortex_ldos_energies(n=128):
    """The demonstration's LDOS post-process (Sec. IV listing): n energies
    from 0 to 0.5 (units of 2 pi k_B Tc), endpoints included."""
    return np.linspace(0.0, 0.5, n)


def ldos_energies(n=512):
    """Real energies at the midpoints of n equal intervals of [-2, 2] DELTA0,
    -2 DELTA0 + 4 DELTA0 (k + 1/2) / n, k = 0..n-1: symmetric about zero (the
    two nearest zero are +-2 DELTA0 / n)."""
    return -2.0 * DELTA0 + 4.0 * DELTA0 * (np.arange(n) + 0.5) / n


def batch_specs(n=64, seed0=3):
    """Seeded batch of n grains (grain g uses seed seed0 + g): a disc, a
    square at a random rotation or a convex polygon of 5-9 vertices with
    jittered angles, minus 0-2 disc or square holes; grid N x N with N in
    {64, 80, ..., 512}, h = 0.2, the grain spanning about 80% of the box;
    t ~ U[0.05, 0.9], flux ~ U[0, 5] quanta (symmetric gauge), s or d_{x2-y2}
    with probability 1/2, 32/64/96/128 angles, 32..128 poles in steps of 16,
    infinite penetration depth."""
    out = []
    for g in range(n):
        rng = np.random.default_rng(seed0 + g)
        N = int(rng.choice(np.arange(64, 513, 16)))
        h = 0.2
        L = N * h
        R = 0.4 * L
        kind = int(rng.integers(3))
        if kind == 0:
            shapes = [_disc(0.0, 0.0, R)]
        elif kind == 1:
            shapes = [_square(0.0, 0.0, 0.6 * L, float(rng.uniform(0, 0.25)))]
        else:
            nv = int(rng.integers(5, 10))
            ang = 2 * math.pi * (np.arange(nv) + rng.uniform(-0.3, 0.3, nv)) / nv
            shapes = [{"kind": "polygon", "vx": list(R * np.cos(ang)), "vy": list(R * np.sin(ang)), "add": True}]
        for _ in range(int(rng.integers(3))):
            hr = float(rng.uniform(0.05, 0.12)) * L
            hx, hy = rng.uniform(-0.2, 0.2, 2) * L
            if rng.random() < 0.5:
                shapes.append(_disc(float(hx), float(hy), hr, add=False))
            else:
                shapes.append(_square(float(hx), float(hy), 1.4 * hr, float(rng.uniform(0, 0.25)), add=False))
        sym = "s" if rng.random() < 0.5 else "dx2y2"
        out.append(dict(nx=N, ny=N, h=h, shapes=shapes, n_theta=int(rng.choice([32, 64, 96, 128])),
                        n_poles=int(rng.choice(np.arange(32, 129, 16))), t=float(rng.uniform(0.05, 0.9)),
                        components=[(sym, 1.0)], kappa=0.0, flux_quanta=float(rng.uniform(0, 5)),
                        gauge="symmetric", charge_sign=-1, name="batch%02d" % g))
    return out


def batch_initial_delta(sp, g):
    """Starting field of batch grain g: 0.9 DELTA0 with 5% seeded noise."""
    rng = np.random.default_rng(1000 + g)
    u = rng.uniform(-0.05, 0.05, (sp["ny"], sp["nx"]))
    return (0.9 * DELTA0 * (1.0 + u))[None].astype(np.complex128)
