"""Riccati sweep along the trajectories of one Fermi-surface angle.

Oracle (test infrastructure only).  Complex FP64 throughout.
Follows Sec. II.A (Riccati parametrisation and equations), Sec. III.A
(rotated lattice, bilinear interpolation both ways, boundary-value
interpolation in angle and boundary coordinate) and App. C (implicit
midpoint step in closed form, half-step values, nearest-neighbour
extrapolation at the boundary).
"""
import math
import numpy as np


# --------------------------------------------------------------------------
# interpolation from the reference grid (Sec. III.A)
# --------------------------------------------------------------------------

def masked_bilinear_stencil(grid, mask, px, py):
    """Bilinear weights of the four cell centres around each point, with
    corners that are outside the grain or off the array dropped and the
    rest renormalised.  Reading (the paper is silent near walls): if no
    corner with positive weight survives, the value of the nearest grain
    cell centre is used (ties -> smallest row-major index).
    Returns flat cell indices [N,4] and weights [N,4]."""
    px = np.atleast_1d(np.asarray(px, dtype=np.float64))
    py = np.atleast_1d(np.asarray(py, dtype=np.float64))
    fx = (px - grid.x0) / grid.h - 0.5
    fy = (py - grid.y0) / grid.h - 0.5
    i0 = np.floor(fx).astype(np.int64)
    j0 = np.floor(fy).astype(np.int64)
    wx = fx - i0
    wy = fy - j0
    ci = np.stack([i0, i0 + 1, i0, i0 + 1], axis=1)
    cj = np.stack([j0, j0, j0 + 1, j0 + 1], axis=1)
    w = np.stack([(1 - wx) * (1 - wy), wx * (1 - wy), (1 - wx) * wy, wx * wy], axis=1)
    ok = (ci >= 0) & (ci < grid.nx) & (cj >= 0) & (cj < grid.ny)
    cic = np.clip(ci, 0, grid.nx - 1)
    cjc = np.clip(cj, 0, grid.ny - 1)
    ok &= mask[cjc, cic]
    w = np.where(ok, w, 0.0)
    idx = np.where(ok, cjc * grid.nx + cic, 0)
    tot = w.sum(axis=1)
    good = tot > 0.0
    w[good] /= tot[good][:, None]
    bad = np.nonzero(~good)[0]
    if bad.size:
        X, Y = grid.centres()
        gx = X[mask]
        gy = Y[mask]
        flat = np.nonzero(mask.ravel())[0]
        for b in bad:
            d2 = (gx - px[b]) ** 2 + (gy - py[b]) ** 2
            a = int(np.argmin(d2))  # first minimum = smallest flat index
            idx[b] = [flat[a], 0, 0, 0]
            w[b] = [1.0, 0.0, 0.0, 0.0]
    return idx, w


def clamped_bilinear_stencil(grid, px, py):
    """Plain bilinear weights of the induced vector potential, which lives
    on every cell; points beyond the outermost cell centres are clamped
    onto them (reading; the grain lies inside the array)."""
    px = np.atleast_1d(np.asarray(px, dtype=np.float64))
    py = np.atleast_1d(np.asarray(py, dtype=np.float64))
    fx = np.clip((px - grid.x0) / grid.h - 0.5, 0.0, grid.nx - 1.0)
    fy = np.clip((py - grid.y0) / grid.h - 0.5, 0.0, grid.ny - 1.0)
    i0 = np.minimum(np.floor(fx).astype(np.int64), grid.nx - 2)
    j0 = np.minimum(np.floor(fy).astype(np.int64), grid.ny - 2)
    wx = fx - i0
    wy = fy - j0
    idx = np.stack([j0 * grid.nx + i0, j0 * grid.nx + i0 + 1,
                    (j0 + 1) * grid.nx + i0, (j0 + 1) * grid.nx + i0 + 1], axis=1)
    w = np.stack([(1 - wx) * (1 - wy), wx * (1 - wy), (1 - wx) * wy, wx * wy], axis=1)
    return idx, w


# --------------------------------------------------------------------------
# Riccati step (App. C) and closed forms of Sec. II.A
# --------------------------------------------------------------------------

def riccati_step(gam, dm, zm, h):
    """One implicit-midpoint step of d gamma/ds = i[D* g^2 + 2 z g + D]
    (App. C with v_F = 1): the quadratic c2 g'^2 + c1 g' + c0 = 0 is
    solved in the cancellation-free form g' = 2 c0 / (-c1 + sqrt(disc)).
    Reading: the principal square root is used, with its sign flipped if
    it points away from -c1 (Re(sqrt * conj(-c1)) < 0), which selects the
    root that tends to the old value as h -> 0."""
    c2 = 0.25j * h * np.conj(dm)
    c1 = 2.0 * c2 * gam + 1j * h * zm - 1.0
    c0 = (c1 - c2 * gam + 2.0) * gam - 4.0 * np.conj(c2)
    rt = np.sqrt(c1 * c1 - 4.0 * c2 * c0)
    rt = np.where((rt * np.conj(-c1)).real < 0.0, -rt, rt)
    return 2.0 * c0 / (-c1 + rt)


def bulk_sqrt(z, dabs2):
    """s = sqrt(z^2 - |D|^2) on the branch Im s > 0 (the root that decays
    along the integration direction; retarded for real energies)."""
    s = np.sqrt(z * z - dabs2)
    return np.where(s.imag < 0.0, -s, s)


def bulk_gamma(z, d):
    """Homogeneous solution of the gamma Riccati equation of Sec. II.A,
    D* g^2 + 2 z g + D = 0, on its stable branch, written as -D/(z+s)
    (free of cancellation; zero when D = 0)."""
    s = bulk_sqrt(z, (d * np.conj(d)).real)
    return -d / (z + s)


def bulk_gamma_tilde(z, d):
    """Homogeneous gamma-tilde: the gamma root with D -> -D*."""
    s = bulk_sqrt(z, (d * np.conj(d)).real)
    return np.conj(d) / (z + s)


def green(gam, gamt):
    """g, f, f-tilde from the Riccati parametrisation of Sec. II.A:
    g-hat = -i pi / (1 + gamma gamma~) [[1 - gamma gamma~, 2 gamma],
    [2 gamma~, -1 + gamma gamma~]] and g-hat = [[g, f], [-f~, g~]]."""
    x = gam * gamt
    inv = 1.0 / (1.0 + x)
    g = -1j * math.pi * (1.0 - x) * inv
    f = -2j * math.pi * gam * inv
    ft = 2j * math.pi * gamt * inv
    return g, f, ft


# --------------------------------------------------------------------------
# one angle: node values, march, per-node sums
# --------------------------------------------------------------------------

class AngleSweepData:
    """Value slots of one angle: for every segment its interior lattice
    nodes in order (or, for a segment without interior node, one slot at
    its midpoint), with the interpolation stencils of Delta and A_ind and
    the step sizes of the march."""

    def __init__(self, grid, mask, table, seg_ids=None):
        self.table = table
        if seg_ids is None:
            seg_ids = np.arange(table.nseg)
        self.seg_ids = np.asarray(seg_ids, dtype=np.int64)
        S = len(self.seg_ids)
        n = table.nnodes[self.seg_ids]
        self.n = n
        self.nslot = np.maximum(n, 1)
        W = int(self.nslot.max()) if S else 1
        self.W = W
        line = table.seg_line[self.seg_ids]
        jf = table.jfirst[self.seg_ids]
        s0 = table.smin[self.seg_ids]
        s1 = table.smax[self.seg_ids]
        t = np.arange(W)[None, :]
        valid = t < self.nslot[:, None]
        s_slot = np.where(n[:, None] > 0, table.node_s(jf[:, None] + t), 0.5 * (s0 + s1)[:, None])
        s_slot = np.where(valid, s_slot, 0.0)
        px, py = table.point(line[:, None] * np.ones_like(t), s_slot)
        self.valid = valid
        self.px, self.py = px, py
        flat_x = px[valid]
        flat_y = py[valid]
        self.d_idx, self.d_w = masked_bilinear_stencil(grid, mask, flat_x, flat_y)
        self.a_idx, self.a_w = clamped_bilinear_stencil(grid, flat_x, flat_y)
        # step sizes: step t runs from slot t-1 to slot t (t = 0..n), the
        # first and last ones from / to the boundary points
        h = table.h
        hs = np.full((S, W + 1), h)
        first = np.where(n > 0, table.node_s(jf) - s0, s1 - s0)
        last = np.where(n > 0, s1 - table.node_s(jf + n - 1), 0.0)
        hs[:, 0] = first
        hs[np.arange(S), np.maximum(n, 0)] = np.where(n > 0, last, first)
        stepno = np.arange(W + 1)[None, :]
        self.nsteps = n + 1
        self.step_valid = stepno < self.nsteps[:, None]
        self.hs = np.where(self.step_valid, hs, 0.0)

    def slot_values(self, flat_vals):
        out = np.zeros(self.valid.shape, dtype=flat_vals.dtype)
        out[self.valid] = flat_vals
        return out

    def interpolate(self, delta_k, a_cells_x, a_cells_y, aext_x, aext_y):
        """Delta(p_k, slot) and a(slot) = v_k . A(slot) (Sec. III.A):
        delta_k is the grid field sum_G eta_G(phi_k) Delta_G [ny*nx];
        a_cells_* the induced vector potential [ny*nx]; aext_* the external
        vector potential evaluated at the slots (flat, valid slots)."""
        d = np.sum(delta_k[self.d_idx] * self.d_w, axis=1)
        ax = np.sum(a_cells_x[self.a_idx] * self.a_w, axis=1) + aext_x
        ay = np.sum(a_cells_y[self.a_idx] * self.a_w, axis=1) + aext_y
        a = self.table.epx * ax + self.table.epy * ay
        return self.slot_values(d), self.slot_values(a)

    def midpoints(self, v):
        """Half-step values of each step (App. C): the mean of the values
        at the two ends, where a boundary point takes the value of the
        nearest slot (nearest-neighbour extrapolation)."""
        S, W = v.shape
        last = self.nslot - 1
        prev = np.concatenate([v[:, :1], v], axis=1)          # slot t-1 for step t
        nxt = np.concatenate([v, v[np.arange(S), last][:, None]], axis=1)
        rows = np.arange(S)
        # step n (after the last slot) uses slot n-1 at both ends
        nxt[rows, self.nslot] = v[rows, last]
        # segments without interior node: one step, slot 0 at both ends
        zero = self.n == 0
        prev[zero, 0] = v[zero, 0]
        nxt[zero, 0] = v[zero, 0]
        return 0.5 * (prev + nxt)

    def end_values(self, v):
        """Values at R_min and R_max (nearest slot)."""
        S = v.shape[0]
        return v[:, 0], v[np.arange(S), self.nslot - 1]


def march(data, dnode, anode, eps_j, q, g_start, gt_start):
    """Integrate gamma forward (R_min -> R_max) and gamma~ backward
    (R_max -> R_min) along every segment of one angle (Sec. III.A,
    App. C), for the complex energies eps_j (i eps~_p for Matsubara/Ozaki
    poles, eps + i delta for retarded) with z = eps + q a.
    gamma~ uses the same step with Delta -> -Delta* (tilde symmetry of
    Sec. II), z unchanged.
    Returns gamma and gamma~ at the slots [S, W, E] and the end values
    gamma(R_max), gamma~(R_min) [S, E]."""
    S, W = dnode.shape
    E = eps_j.shape[0]
    dm = data.midpoints(dnode)                       # [S, W+1]
    am = data.midpoints(anode)
    zm = eps_j[None, None, :] + q * am[:, :, None]   # [S, W+1, E]
    hs = data.hs
    gam_nodes = np.zeros((S, W, E), dtype=np.complex128)
    gamt_nodes = np.zeros((S, W, E), dtype=np.complex128)
    g = g_start.copy()
    for t in range(W + 1):
        act = data.step_valid[:, t]
        if not act.any():
            break
        gn = riccati_step(g, dm[:, t, None], zm[:, t, :], hs[:, t, None])
        g = np.where(act[:, None], gn, g)
        if t < W:
            isnode = act & (t < data.n)
            gam_nodes[isnode, t, :] = g[isnode]
    g_end = g
    gt = gt_start.copy()
    for t in range(W, -1, -1):
        act = data.step_valid[:, t]
        if not act.any():
            continue
        gn = riccati_step(gt, -np.conj(dm[:, t, None]), zm[:, t, :], hs[:, t, None])
        gt = np.where(act[:, None], gn, gt)
        if t >= 1:
            isnode = act & (t - 1 < data.n)
            gamt_nodes[isnode, t - 1, :] = gt[isnode]
    gt_end = gt
    return gam_nodes, gamt_nodes, g_end, gt_end


def node_sums(gam_nodes, gamt_nodes, dnode, res, tt):
    """Per-node energy sums over the positive poles (Eqs. gapeq_fixpoint,
    current_density, Eilenberger free energy), using g(-e_n) = g(e_n)*,
    f(-e_n) = f~(e_n)* for the negative half:
      S_f = t~ sum_p R_p (f_p + conj f~_p)
      S_g = t~ sum_p R_p Re g_p
      S_I = 2 pi t~ sum_p R_p Re[(D* f_p + D f~_p) / (pi + i g_p)]
    Reading of the free-energy denominator: pi + i sgn(e_n) g, so that the
    negative-frequency terms are the conjugates of the positive ones."""
    g, f, ft = green(gam_nodes, gamt_nodes)
    d = dnode[:, :, None]
    sf = tt * np.sum(res * (f + np.conj(ft)), axis=-1)
    sg = tt * np.sum(res * g.real, axis=-1)
    si = 2.0 * math.pi * tt * np.sum(res * ((np.conj(d) * f + d * ft) / (math.pi + 1j * g)).real, axis=-1)
    return sf, sg, si


# --------------------------------------------------------------------------
# rotate back (Sec. III.A)
# --------------------------------------------------------------------------

def rotate_back_stencil(table, seg_map, pos_map, cx, cy):
    """For reference-grid points (cx, cy): bilinear weights over the four
    lattice nodes around each point in the rotated frame, with nodes that
    are not interior segment nodes dropped and the rest renormalised.
    Reading: if none with positive weight remains, the nearest interior
    node is used (ties -> smallest (line, node)).
    Returns (segment, slot) index arrays [N,4] and weights [N,4]."""
    cx = np.atleast_1d(cx)
    cy = np.atleast_1d(cy)
    u, v = table.lattice_coords(cx, cy)
    M = table.M
    i0 = np.floor(u).astype(np.int64)
    j0 = np.floor(v).astype(np.int64)
    wu = u - i0
    wv = v - j0
    li = np.stack([i0, i0 + 1, i0, i0 + 1], axis=1)
    lj = np.stack([j0, j0, j0 + 1, j0 + 1], axis=1)
    w = np.stack([(1 - wu) * (1 - wv), wu * (1 - wv), (1 - wu) * wv, wu * wv], axis=1)
    inb = (li >= 0) & (li < M) & (lj >= 0) & (lj < M)
    lic = np.clip(li, 0, M - 1)
    ljc = np.clip(lj, 0, M - 1)
    sg = np.where(inb, seg_map[lic, ljc], -1)
    ps = np.where(inb, pos_map[lic, ljc], -1)
    ok = sg >= 0
    w = np.where(ok, w, 0.0)
    tot = w.sum(axis=1)
    good = tot > 0.0
    w[good] /= tot[good][:, None]
    sg = np.where(ok, sg, 0)
    ps = np.where(ok, ps, 0)
    bad = np.nonzero(~good)[0]
    if bad.size:
        # brute force over every interior node of the angle
        ni, nj = np.nonzero(seg_map >= 0)          # row-major: sorted by (line, node)
        for b in bad:
            d2 = (ni - u[b]) ** 2 + (nj - v[b]) ** 2
            a = int(np.argmin(d2))
            sg[b] = [seg_map[ni[a], nj[a]], 0, 0, 0]
            ps[b] = [pos_map[ni[a], nj[a]], 0, 0, 0]
            w[b] = [1.0, 0.0, 0.0, 0.0]
    return sg, ps, w


# --------------------------------------------------------------------------
# specular boundary condition (Sec. II.A, Sec. III.A)
# --------------------------------------------------------------------------

def bc_taps(tables, k, seg, at_start):
    """Interpolation taps of the start value of one segment (Sec. III.A:
    interpolate between boundary coordinates and azimuthal angles).

    For gamma at R_min (at_start=True): the specularly reflected incoming
    direction is phi_in = 2 theta_t - phi_k (theta_t = wall tangent).
    Reading: with x = phi_in / dphi, angles floor(x) and floor(x)+1 get
    weights 1-frac(x), frac(x); on each of them the two lattice lines that
    bracket R_min get weights from the fractional line coordinate; on each
    line the segment whose end R_max lies nearest R_min is taken, if that
    distance is at most 2h / max(|sin(phi_k' - theta_t)|, 1/8) (the
    spacing of successive line ends along the wall grows like 1/sin).
    gamma~ at R_max is the mirror case: phi_out = 2 theta_t - phi_k and
    the segment whose start lies nearest R_max.
    Returns a list of (angle, segment, weight) with weights summing to one,
    or [] when no tap is accepted (then the bulk value is used)."""
    tab = tables[k]
    nth = len(tables)
    dphi = 2.0 * math.pi / nth
    if at_start:
        px, py = tab.start_point(seg)
        th = tab.tmin[seg]
    else:
        px, py = tab.end_point(seg)
        th = tab.tmax[seg]
    phi_r = math.fmod(2.0 * th - tab.phi, 2.0 * math.pi)
    if phi_r < 0.0:
        phi_r += 2.0 * math.pi
    x = phi_r / dphi
    k0 = int(math.floor(x))
    wphi = x - k0
    taps = []
    for kk, wk in ((k0 % nth, 1.0 - wphi), ((k0 + 1) % nth, wphi)):
        t2 = tables[kk]
        u = ((px - t2.cx) * t2.eqx + (py - t2.cy) * t2.eqy) / t2.h + t2.half
        i0 = int(math.floor(u))
        wu = u - i0
        sn = abs(math.sin(t2.phi - th))
        dacc = 2.0 * t2.h / max(sn, 0.125)
        for ii, wi in ((i0, 1.0 - wu), (i0 + 1, wu)):
            if ii < 0 or ii >= t2.M:
                continue
            cand = np.nonzero(t2.seg_line == ii)[0]
            if cand.size == 0:
                continue
            if at_start:
                ex, ey = t2.end_point(cand)
            else:
                ex, ey = t2.start_point(cand)
            dist = np.hypot(ex - px, ey - py)
            a = int(np.argmin(dist))
            if dist[a] <= dacc:
                taps.append((kk, int(cand[a]), wk * wi))
    tot = sum(t[2] for t in taps)
    if not tot > 0.0:
        return []
    return [(a, b, w / tot) for (a, b, w) in taps]
