"""Grain geometry, reference grid, rotated lattices and trajectory segments.

Oracle (test infrastructure only).  Follows Sec. III.A (square reference
grid of spacing h, per-angle rotated square lattice with the same spacing,
exact boundary location) and App. B (disc / regular polygon / polygon
components combined in order with add or subtract).
"""
import math
import numpy as np


class Disc:
    """Disc component (App. B): centre and radius in units of xi0."""

    def __init__(self, cx, cy, radius, add=True):
        self.cx, self.cy, self.r, self.add = float(cx), float(cy), float(radius), bool(add)

    def inside(self, x, y):
        # closed set: points on the circle count as inside
        dx = x - self.cx
        dy = y - self.cy
        return dx * dx + dy * dy <= self.r * self.r


class Polygon:
    """Convex polygon with counter-clockwise vertices (App. B)."""

    def __init__(self, vx, vy, add=True):
        self.vx = [float(v) for v in vx]
        self.vy = [float(v) for v in vy]
        if len(self.vx) < 3 or len(self.vx) != len(self.vy):
            raise ValueError("polygon needs >= 3 vertices")
        self.add = bool(add)

    def inside(self, x, y):
        # closed convex CCW polygon: on or left of every directed edge
        res = np.ones(np.broadcast(x, y).shape, dtype=bool)
        n = len(self.vx)
        for m in range(n):
            ax, ay = self.vx[m], self.vy[m]
            bx, by = self.vx[(m + 1) % n], self.vy[(m + 1) % n]
            cr = (bx - ax) * (y - ay) - (by - ay) * (x - ax)
            res &= cr >= 0.0
        return res


def regular_polygon(cx, cy, n_edges, side, rotation=0.0, add=True):
    """Regular polygon (App. B): centre, number of edges, side length and a
    rotation in full turns.  Reading (orientation at rotation 0 is not
    printed): the first edge is horizontal at the bottom, so a square with
    rotation 0 has axis-aligned edges.  Vertex m sits at the polar angle
    -pi/2 - pi/n + 2 pi m / n + 2 pi rotation on the circumcircle."""
    n = int(n_edges)
    if n < 3:
        raise ValueError("regular polygon needs >= 3 edges")
    rc = side / (2.0 * math.sin(math.pi / n))
    vx, vy = [], []
    for m in range(n):
        a = -0.5 * math.pi - math.pi / n + 2.0 * math.pi * m / n + 2.0 * math.pi * rotation
        vx.append(cx + rc * math.cos(a))
        vy.append(cy + rc * math.sin(a))
    return Polygon(vx, vy, add)


# Contour pieces of one square of four neighbouring cell centres, by which
# corners are inside (bit 1 lower-left, 2 lower-right, 4 upper-right, 8
# upper-left); the end points are the midpoints of the square's sides
# (B bottom, R right, T top, L left), where the level 1/2 crosses.  Squares
# with only two diagonal corners inside keep those corners apart.
_MS_CASES = {
    1: [("L", "B")], 2: [("B", "R")], 3: [("L", "R")], 4: [("R", "T")],
    5: [("L", "B"), ("R", "T")], 6: [("B", "T")], 7: [("L", "T")], 8: [("T", "L")],
    9: [("B", "T")], 10: [("B", "R"), ("T", "L")], 11: [("R", "T")], 12: [("L", "R")],
    13: [("B", "R")], 14: [("L", "B")],
}


class MaskShape:
    """Component given by a cell mask on the reference grid (App. B allows
    grains of any shape; this is the reading for a grain given only by its
    cells).  Its boundary is the marching-squares contour of the mask at
    level 1/2 over the cell centres, with every cell beyond the array
    outside; inside is the even-odd rule of that closed polyline.  Edges are
    listed square by square, rows of squares bottom to top, each row left to
    right."""

    def __init__(self, mask, grid, add=True):
        m = np.asarray(mask) != 0
        ny, nx = m.shape
        if (nx, ny) != (grid.nx, grid.ny):
            raise ValueError("mask shape does not match the grid")
        h, x0, y0 = grid.h, grid.x0, grid.y0

        def val(i, j):
            return bool(m[j, i]) if 0 <= i < nx and 0 <= j < ny else False

        ax, ay, bx, by = [], [], [], []
        for j in range(-1, ny):
            for i in range(-1, nx):
                case = (1 if val(i, j) else 0) | (2 if val(i + 1, j) else 0) | \
                       (4 if val(i + 1, j + 1) else 0) | (8 if val(i, j + 1) else 0)
                if case in (0, 15):
                    continue
                pts = {"B": (x0 + (i + 1) * h, y0 + (j + 0.5) * h), "T": (x0 + (i + 1) * h, y0 + (j + 1.5) * h),
                       "L": (x0 + (i + 0.5) * h, y0 + (j + 1) * h), "R": (x0 + (i + 1.5) * h, y0 + (j + 1) * h)}
                for a, b in _MS_CASES[case]:
                    ax.append(pts[a][0])
                    ay.append(pts[a][1])
                    bx.append(pts[b][0])
                    by.append(pts[b][1])
        self.ax, self.ay = np.array(ax), np.array(ay)
        self.bx, self.by = np.array(bx), np.array(by)
        self.add = bool(add)

    def inside(self, x, y):
        # even-odd rule: crossings of the ray to +x, each edge half-open in y
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        shp = np.broadcast(x, y).shape
        xf = np.broadcast_to(x, shp).ravel()
        yf = np.broadcast_to(y, shp).ravel()
        res = np.zeros(xf.shape, dtype=bool)
        for c0 in range(0, xf.size, 4096):
            px = xf[c0:c0 + 4096, None]
            py = yf[c0:c0 + 4096, None]
            straddle = (self.ay[None, :] > py) != (self.by[None, :] > py)
            with np.errstate(divide="ignore", invalid="ignore"):
                xi = self.ax + (py - self.ay) * (self.bx - self.ax) / (self.by - self.ay)
            res[c0:c0 + 4096] = (np.count_nonzero(straddle & (px < xi), axis=1) % 2) == 1
        return res.reshape(shp)


def domain(shapes, x, y):
    """The grain D as the ordered fold of its components (App. B):
    an added component is united with D, a subtracted one removed."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = np.zeros(np.broadcast(x, y).shape, dtype=bool)
    for sh in shapes:
        ins = sh.inside(x, y)
        d = (d | ins) if sh.add else (d & ~ins)
    return d


class Grid:
    """Reference grid (Sec. III.A): nx x ny square cells of side h whose
    lower-left corner is (x0, y0); values live at cell centres."""

    def __init__(self, nx, ny, h, x0=None, y0=None):
        self.nx, self.ny, self.h = int(nx), int(ny), float(h)
        self.x0 = -0.5 * nx * h if x0 is None else float(x0)
        self.y0 = -0.5 * ny * h if y0 is None else float(y0)
        self.cx = self.x0 + 0.5 * self.nx * self.h
        self.cy = self.y0 + 0.5 * self.ny * self.h

    def centres(self):
        xs = self.x0 + (np.arange(self.nx) + 0.5) * self.h
        ys = self.y0 + (np.arange(self.ny) + 0.5) * self.h
        X, Y = np.meshgrid(xs, ys)  # [ny][nx], x fastest
        return X, Y

    def mask(self, shapes):
        X, Y = self.centres()
        return domain(shapes, X, Y)

    def lattice_size(self):
        """Side M of the rotated lattice.  Reading: the smallest integer
        >= sqrt(nx^2+ny^2)+3 with M = nx (mod 2), so the lattice covers
        the grid at every angle and, at phi = 0, its nodes coincide with
        the cell centres."""
        m = int(math.ceil(math.sqrt(self.nx * self.nx + self.ny * self.ny) + 3.0))
        if (m - self.nx) % 2 != 0:
            m += 1
        return m


def angle_frame(phi):
    """Unit vectors of the rotated frame for angle phi: e_par along the
    Fermi velocity, e_perp = (sin phi, -cos phi) across the lines."""
    c, s = math.cos(phi), math.sin(phi)
    return (c, s), (s, -c)


def _primitive_hits(shapes, bx, by, ex, ey):
    """All intersections of the line B + s e with component boundaries,
    as (s, tangent angle) pairs."""
    hits = []
    for sh in shapes:
        if isinstance(sh, Disc):
            dx, dy = bx - sh.cx, by - sh.cy
            bq = dx * ex + dy * ey
            cq = dx * dx + dy * dy - sh.r * sh.r
            disc = bq * bq - cq
            if disc > 0.0:
                rt = math.sqrt(disc)
                for s in (-bq - rt, -bq + rt):
                    px, py = bx + s * ex, by + s * ey
                    tang = math.atan2(py - sh.cy, px - sh.cx) + 0.5 * math.pi
                    hits.append((s, tang))
        elif isinstance(sh, MaskShape):
            # the same line / edge formula as for polygon edges, per contour edge
            dx, dy = sh.bx - sh.ax, sh.by - sh.ay
            den = ex * dy - ey * dx
            ok = den != 0.0
            with np.errstate(divide="ignore", invalid="ignore"):
                wx, wy = sh.ax - bx, sh.ay - by
                s_all = (wx * dy - wy * dx) / den
                t_all = (wx * ey - wy * ex) / den
            for m in np.nonzero(ok & (t_all >= 0.0) & (t_all <= 1.0))[0]:
                hits.append((float(s_all[m]), math.atan2(float(dy[m]), float(dx[m]))))
        else:
            n = len(sh.vx)
            for m in range(n):
                ax, ay = sh.vx[m], sh.vy[m]
                dx, dy = sh.vx[(m + 1) % n] - ax, sh.vy[(m + 1) % n] - ay
                den = ex * dy - ey * dx
                if den == 0.0:
                    continue
                wx, wy = ax - bx, ay - by
                s = (wx * dy - wy * dx) / den
                t = (wx * ey - wy * ex) / den
                if 0.0 <= t <= 1.0:
                    hits.append((s, math.atan2(dy, dx)))
    hits.sort(key=lambda p: p[0])
    return hits


def line_segments(shapes, bx, by, ex, ey, h):
    """Maximal parameter intervals [s_min, s_max] of the line B + s e that
    lie in D (Sec. II.A trajectory coordinate, Sec. III.A exact boundary).

    Reading: the sorted boundary intersections cut the line into
    intervals; an interval belongs to D when its midpoint does; adjacent
    D-intervals merge.  Intervals shorter than 1e-9 h are ignored.
    Returns a list of (s_min, s_max, tangent_min, tangent_max)."""
    hits = _primitive_hits(shapes, bx, by, ex, ey)
    segs = []
    tol = 1e-9 * h
    start = None
    end = None
    for a in range(len(hits) - 1):
        sa, ta = hits[a]
        sb, tb = hits[a + 1]
        if sb - sa <= tol:
            continue
        sm = 0.5 * (sa + sb)
        ins = bool(domain(shapes, bx + sm * ex, by + sm * ey))
        if ins:
            if start is None:
                start = (sa, ta)
            end = (sb, tb)
        elif start is not None:
            segs.append((start[0], end[0], start[1], end[1]))
            start = None
    if start is not None:
        segs.append((start[0], end[0], start[1], end[1]))
    return segs


class AngleTable:
    """Trajectory segments of one Fermi-surface angle (Sec. III.A, Fig. 2):
    the lines of the rotated lattice, their segments inside D, and the
    lattice nodes strictly inside each segment."""

    def __init__(self, grid, shapes, phi):
        self.phi = phi
        self.M = M = grid.lattice_size()
        h = grid.h
        (self.epx, self.epy), (self.eqx, self.eqy) = angle_frame(phi)
        half = 0.5 * (M - 1)
        seg_line, smin, smax, tmin, tmax, jfirst, nnodes = [], [], [], [], [], [], []
        for i in range(M):
            u = (i - half) * h
            bx = grid.cx + u * self.eqx
            by = grid.cy + u * self.eqy
            for (s0, s1, t0, t1) in line_segments(shapes, bx, by, self.epx, self.epy, h):
                jf = int(math.floor(s0 / h + half)) + 1
                jl = int(math.ceil(s1 / h + half)) - 1
                seg_line.append(i)
                smin.append(s0)
                smax.append(s1)
                tmin.append(t0)
                tmax.append(t1)
                jfirst.append(jf)
                nnodes.append(max(0, jl - jf + 1))
        self.seg_line = np.array(seg_line, dtype=np.int64)
        self.smin = np.array(smin, dtype=np.float64)
        self.smax = np.array(smax, dtype=np.float64)
        self.tmin = np.array(tmin, dtype=np.float64)
        self.tmax = np.array(tmax, dtype=np.float64)
        self.jfirst = np.array(jfirst, dtype=np.int64)
        self.nnodes = np.array(nnodes, dtype=np.int64)
        self.h = h
        self.half = half
        self.cx, self.cy = grid.cx, grid.cy

    @property
    def nseg(self):
        return len(self.seg_line)

    def point(self, i, s):
        """Position of parameter s on line i."""
        u = (np.asarray(i) - self.half) * self.h
        return (self.cx + u * self.eqx + s * self.epx,
                self.cy + u * self.eqy + s * self.epy)

    def node_s(self, j):
        return (np.asarray(j) - self.half) * self.h

    def start_point(self, k):
        return self.point(self.seg_line[k], self.smin[k])

    def end_point(self, k):
        return self.point(self.seg_line[k], self.smax[k])

    def lattice_coords(self, x, y):
        """(line, node) lattice coordinates of a point (real-valued)."""
        dx = np.asarray(x) - self.cx
        dy = np.asarray(y) - self.cy
        return (dx * self.eqx + dy * self.eqy) / self.h + self.half, \
               (dx * self.epx + dy * self.epy) / self.h + self.half

    def node_map(self):
        """Dense (line, node) -> (segment, position in segment) map; -1
        where the lattice node is not strictly inside a segment."""
        seg = -np.ones((self.M, self.M), dtype=np.int64)
        pos = -np.ones((self.M, self.M), dtype=np.int64)
        for k in range(self.nseg):
            i = self.seg_line[k]
            jf = self.jfirst[k]
            n = self.nnodes[k]
            if n > 0:
                seg[i, jf:jf + n] = k
                pos[i, jf:jf + n] = np.arange(n)
        return seg, pos
