"""One iteration map of Alg. 1, the Picard self-consistency loop, and the
LDOS post-process.

Oracle (test infrastructure only).  Follows Alg. 1 (Sec. III.A), Eqs.
gapeq_fixpoint and current_density (Sec. II), the Eilenberger free-energy
form (Sec. II), App. D (A-solve), App. E (Picard on the concatenated x) and
the LDOS definition of Sec. II with the burn-in of App. B; App. E also
gives Polyak's heavy-ball accelerator.
"""
import math
import numpy as np

from . import tables, geometry, sweep, fields


class Grain:
    """A grain with its numerics.  components: list of (basis name or None,
    critical temperature relative to Tc).  eta may be given directly as a
    complex [ncomp][n_theta] table (then the names are ignored)."""

    def __init__(self, nx, ny, h, shapes, n_theta, n_poles, t,
                 components=(("s", 1.0),), crystal_rotation=0.0, kappa=0.0,
                 flux_quanta=0.0, gauge="symmetric", charge_sign=-1,
                 x0=None, y0=None, eta=None):
        self.grid = geometry.Grid(nx, ny, h, x0, y0)
        self.shapes = list(shapes)
        self.mask = self.grid.mask(self.shapes)
        self.area = h * h * float(self.mask.sum())
        self.n_theta = int(n_theta)
        self.n_poles = int(n_poles)
        self.t = float(t)
        self.tt = self.t / (2.0 * math.pi)
        self.kappa = float(kappa)
        self.flux = float(flux_quanta)
        self.gauge = gauge
        self.q = float(charge_sign)
        self.phi = tables.fs_angles(self.n_theta)
        self.wk = tables.fs_weights(self.n_theta)
        self.zp, self.rp = tables.ozaki_poles(self.n_poles)
        self.tc = np.array([c[1] for c in components], dtype=np.float64)
        self.ncomp = len(components)
        if eta is None:
            eta = np.array([tables.basis(c[0], self.phi, crystal_rotation) for c in components])
        self.eta = np.asarray(eta, dtype=np.complex128).reshape(self.ncomp, self.n_theta)
        self.tables = [geometry.AngleTable(self.grid, self.shapes, p) for p in self.phi]
        self._data = {}
        self._rb = {}
        self._taps = {}
        self._maps = {}

    # -- cached per-angle geometry ---------------------------------------
    def maps(self, k):
        if k not in self._maps:
            self._maps[k] = self.tables[k].node_map()
        return self._maps[k]

    def data(self, k):
        if k not in self._data:
            self._data[k] = sweep.AngleSweepData(self.grid, self.mask, self.tables[k])
        return self._data[k]

    def rb_stencil(self, k):
        """Rotate-back stencil of every grain cell for angle k."""
        if k not in self._rb:
            X, Y = self.grid.centres()
            seg, pos = self.maps(k)
            self._rb[k] = sweep.rotate_back_stencil(self.tables[k], seg, pos, X[self.mask], Y[self.mask])
        return self._rb[k]

    def taps(self, k, at_start):
        key = (k, at_start)
        if key not in self._taps:
            self._taps[key] = [sweep.bc_taps(self.tables, k, s, at_start)
                               for s in range(self.tables[k].nseg)]
        return self._taps[key]

    def gap_denominator(self):
        """ln(t / t_c,G) + pi T sum_n 1/|e_n| = ln(t/t_c,G) + 2 pi sum_p R_p/z_p
        (Eq. gapeq_fixpoint with the Ozaki poles)."""
        return np.log(self.t / self.tc) + 2.0 * math.pi * np.sum(self.rp / self.zp)

    def steps_per_sweep(self):
        """Trajectory steps of one iteration: gamma and gamma~ each take
        n+1 steps per segment and positive pole."""
        nst = sum(int(np.sum(tb.nnodes + 1)) for tb in self.tables)
        return 2 * self.n_poles * nst

    # -- node values of one angle ----------------------------------------
    def node_values(self, k, data, delta, A_ind):
        """Delta(p_k, slot) and a(slot) on the value slots of angle k."""
        ny, nx = self.grid.ny, self.grid.nx
        dk = np.tensordot(self.eta[:, k], delta.reshape(self.ncomp, ny * nx), axes=(0, 0))
        fx = data.px[data.valid]
        fy = data.py[data.valid]
        ex, ey = fields.external_A(self.gauge, self.flux, self.area, self.grid.cx, self.grid.cy, fx, fy)
        return data.interpolate(dk, A_ind[0].ravel(), A_ind[1].ravel(), ex, ey)

    def start_values(self, k, data, dnode, anode, eps, bc_prev):
        """Start values of gamma at R_min and gamma~ at R_max: the bulk
        roots at the segment ends in the first iteration (reading), then
        the specular taps of the previous iteration's end values (Jacobi
        update, Alg. 1), bulk where no tap exists."""
        d0, d1 = data.end_values(dnode)
        a0, a1 = data.end_values(anode)
        z0 = eps[None, :] + self.q * a0[:, None]
        z1 = eps[None, :] + self.q * a1[:, None]
        g0 = sweep.bulk_gamma(z0, d0[:, None])
        gt0 = sweep.bulk_gamma_tilde(z1, d1[:, None])
        if bc_prev is None:
            return g0, gt0
        gend, gtend = bc_prev
        for row, s in enumerate(data.seg_ids):
            tp = self.taps(k, True)[s]
            if tp:
                g0[row] = sum(w * gend[kk][ss] for (kk, ss, w) in tp)
            tp = self.taps(k, False)[s]
            if tp:
                gt0[row] = sum(w * gtend[kk][ss] for (kk, ss, w) in tp)
        return g0, gt0

    # -- the iteration map ------------------------------------------------
    def iterate(self, delta, A_ind, bc_prev=None):
        """One pass of the loop body of Alg. 1 with Delta and A_ind given:
        for every angle and positive pole sweep gamma, gamma~, form the
        Green's functions, sum over poles, rotate back and accumulate;
        then the gap update, current and free-energy density.
        Returns a dict with delta_new [ncomp,ny,nx], j [2,ny,nx],
        omega_density [ny,nx], omega_total, bc (end values per angle)."""
        ny, nx = self.grid.ny, self.grid.nx
        delta = np.asarray(delta, dtype=np.complex128).reshape(self.ncomp, ny, nx)
        A_ind = np.asarray(A_ind, dtype=np.float64).reshape(2, ny, nx)
        m = self.mask
        ncell = int(m.sum())
        num = np.zeros((self.ncomp, ncell), dtype=np.complex128)
        jx = np.zeros(ncell)
        jy = np.zeros(ncell)
        icell = np.zeros(ncell)
        eps = 1j * self.zp * self.tt
        gend, gtend = [], []
        for k in range(self.n_theta):
            data = self.data(k)
            dnode, anode = self.node_values(k, data, delta, A_ind)
            g0, gt0 = self.start_values(k, data, dnode, anode, eps, bc_prev)
            gn, gtn, ge, gte = sweep.march(data, dnode, anode, eps, self.q, g0, gt0)
            gend.append(ge)
            gtend.append(gte)
            sf, sg, si = sweep.node_sums(gn, gtn, dnode, self.rp, self.tt)
            seg, pos, w = self.rb_stencil(k)
            cf = np.sum(sf[seg, pos] * w, axis=1)
            cg = np.sum(sg[seg, pos] * w, axis=1)
            ci = np.sum(si[seg, pos] * w, axis=1)
            wk = self.wk[k]
            num += wk * np.conj(self.eta[:, k])[:, None] * cf[None, :]
            jx += 4.0 * self.q * wk * math.cos(self.phi[k]) * cg
            jy += 4.0 * self.q * wk * math.sin(self.phi[k]) * cg
            icell += wk * ci
        return self._finish(delta, A_ind, num, jx, jy, icell, (gend, gtend))

    def green_average(self, delta, A_ind, bc_prev=None):
        """Fermi-surface average <g>(R, i eps~_p) of the quasiclassical
        Green's function g = -i pi (1 - gamma gamma~)/(1 + gamma gamma~)
        (Sec. II.A) at each positive pole, from the same marches as
        iterate() with the given start values; the angle average rotates
        the per-node g back with the gap's stencils and weights (Sec. III.A).
        Returns complex [n_poles, ny, nx], zero off the grain."""
        ny, nx = self.grid.ny, self.grid.nx
        delta = np.asarray(delta, dtype=np.complex128).reshape(self.ncomp, ny, nx)
        A_ind = np.asarray(A_ind, dtype=np.float64).reshape(2, ny, nx)
        m = self.mask
        eps = 1j * self.zp * self.tt
        out = np.zeros((len(eps), int(m.sum())), dtype=np.complex128)
        for k in range(self.n_theta):
            data = self.data(k)
            dnode, anode = self.node_values(k, data, delta, A_ind)
            g0, gt0 = self.start_values(k, data, dnode, anode, eps, bc_prev)
            gn, gtn, _, _ = sweep.march(data, dnode, anode, eps, self.q, g0, gt0)
            g, _, _ = sweep.green(gn, gtn)                 # [S, W, E]
            seg, pos, w = self.rb_stencil(k)
            cell = np.sum(g[seg, pos, :] * w[:, :, None], axis=1)   # [ncell, E]
            out += self.wk[k] * cell.T
        res = np.zeros((len(eps), ny, nx), dtype=np.complex128)
        res[:, m] = out
        return res

    def _finish(self, delta, A_ind, num, jx, jy, icell, bc):
        ny, nx = self.grid.ny, self.grid.nx
        m = self.mask
        den = self.gap_denominator()
        dnew = np.zeros((self.ncomp, ny, nx), dtype=np.complex128)
        for c in range(self.ncomp):
            dnew[c][m] = num[c] / den[c]
        j = np.zeros((2, ny, nx))
        j[0][m] = jx
        j[1][m] = jy
        dcell = delta[:, m]
        d2avg = np.zeros(dcell.shape[1])
        for k in range(self.n_theta):
            dk = np.tensordot(self.eta[:, k], dcell, axes=(0, 0))
            d2avg += self.wk[k] * (dk * np.conj(dk)).real
        om = np.zeros((ny, nx))
        om[m] = (np.sum((dcell * np.conj(dcell)).real * np.log(self.t / self.tc)[:, None], axis=0)
                 + 2.0 * math.pi * np.sum(self.rp / self.zp) * d2avg - icell)
        h = self.grid.h
        total = h * h * om.sum()
        if self.kappa > 0.0:
            b = fields.curl(A_ind[0], A_ind[1], h)
            total += h * h * np.sum(0.5 * self.kappa ** 2 * b * b)
        return {"delta_new": dnew, "j": j, "omega_density": om,
                "omega_total": total, "bc": bc}

    def iterate_cells(self, delta, A_ind, cells):
        """The same map evaluated only at the given grain cells (flat
        row-major indices), from bulk start values: only the segments that
        feed those cells are swept.  Used to check full-size runs on
        samples.  Returns (delta_new [ncomp,n], j [2,n])."""
        ny, nx = self.grid.ny, self.grid.nx
        delta = np.asarray(delta, dtype=np.complex128).reshape(self.ncomp, ny, nx)
        A_ind = np.asarray(A_ind, dtype=np.float64).reshape(2, ny, nx)
        cells = np.asarray(cells, dtype=np.int64)
        X, Y = self.grid.centres()
        cx = X.ravel()[cells]
        cy = Y.ravel()[cells]
        n = len(cells)
        num = np.zeros((self.ncomp, n), dtype=np.complex128)
        jx = np.zeros(n)
        jy = np.zeros(n)
        eps = 1j * self.zp * self.tt
        for k in range(self.n_theta):
            tab = self.tables[k]
            segm, posm = self.maps(k)
            seg, pos, w = sweep.rotate_back_stencil(tab, segm, posm, cx, cy)
            need = np.unique(seg)
            data = sweep.AngleSweepData(self.grid, self.mask, tab, need)
            row = np.searchsorted(need, seg)
            dnode, anode = self.node_values(k, data, delta, A_ind)
            g0, gt0 = self.start_values(k, data, dnode, anode, eps, None)
            gn, gtn, _, _ = sweep.march(data, dnode, anode, eps, self.q, g0, gt0)
            sf, sg, si = sweep.node_sums(gn, gtn, dnode, self.rp, self.tt)
            cf = np.sum(sf[row, pos] * w, axis=1)
            cg = np.sum(sg[row, pos] * w, axis=1)
            wk = self.wk[k]
            num += wk * np.conj(self.eta[:, k])[:, None] * cf[None, :]
            jx += 4.0 * self.q * wk * math.cos(self.phi[k]) * cg
            jy += 4.0 * self.q * wk * math.sin(self.phi[k]) * cg
        den = self.gap_denominator()
        return num / den[:, None], np.stack([jx, jy])

    # -- Luttinger-Ward free energy (Sec. II) ------------------------------
    def condensation_base(self, delta):
        """The terms of the free-energy density (Eq. qcLWFE) before the
        propagator term: sum_G |Delta_G|^2 ln(t/t_c,G) + pi T sum_n
        <|Delta(p)|^2>/|e_n|, the latter as 2 pi sum_p R_p/z_p times the
        quadrature mean of |sum_G eta_G(phi_k) Delta_G|^2.  [ny, nx], zero
        off the grain."""
        ny, nx = self.grid.ny, self.grid.nx
        delta = np.asarray(delta, dtype=np.complex128).reshape(self.ncomp, ny, nx)
        m = self.mask
        dcell = delta[:, m]
        d2avg = np.zeros(dcell.shape[1])
        for k in range(self.n_theta):
            dk = np.tensordot(self.eta[:, k], dcell, axes=(0, 0))
            d2avg += self.wk[k] * (dk * np.conj(dk)).real
        out = np.zeros((ny, nx))
        out[m] = (np.sum((dcell * np.conj(dcell)).real * np.log(self.t / self.tc)[:, None], axis=0)
                  + 2.0 * math.pi * np.sum(self.rp / self.zp) * d2avg)
        return out

    def free_energy_lw(self, delta, A_ind, n_lambda, bc_iters):
        """Luttinger-Ward form of the free energy (Eqs. qcLWFE and
        qcLWFE_I): the propagator term is
          I(R) = int_0^1 dlambda T sum_n <Delta*(p,R) f_lambda + Delta(p,R) f~_lambda>,
        with f_lambda, f~_lambda the propagators of the Eilenberger equation
        solved with the scaled gap lambda Delta (A unscaled).  With f(-e) =
        f~(e)* the sum over both signs of e_n is twice the real part of the
        positive poles', and <Delta*(p) t~ sum_p R_p (f + conj f~)> =
        sum_G conj(Delta_G) Num_G, with Num_G the gap numerator of
        Eq. gapeq_fixpoint; so per lambda
          I_lambda(R) = 2 sum_G den_G Re[conj(Delta_G(R)) Delta_new,G[lambda Delta](R)].
        Readings: Delta and the propagators meet at the reference cell
        (after the rotate-back, as in the gap update); the lambda integral
        is Gauss-Legendre with n_lambda nodes on [0, 1]; for each lambda the
        boundary values start from the bulk roots of lambda Delta and take
        bc_iters burn-in sweeps (App. B) before the sweep that is used.
        Returns (omega_density [ny, nx], omega_total) with the magnetic term
        h^2 sum (kappa^2/2)|B_ind|^2 as in the Eilenberger form."""
        ny, nx = self.grid.ny, self.grid.nx
        delta = np.asarray(delta, dtype=np.complex128).reshape(self.ncomp, ny, nx)
        A_ind = np.asarray(A_ind, dtype=np.float64).reshape(2, ny, nx)
        m = self.mask
        den = self.gap_denominator()
        x, w = np.polynomial.legendre.leggauss(int(n_lambda))
        lam = 0.5 * (x + 1.0)
        wl = 0.5 * w
        integral = np.zeros((ny, nx))
        for lv, wv in zip(lam, wl):
            dl = lv * delta
            bc = None
            for _ in range(int(bc_iters)):
                bc = self.iterate(dl, A_ind, bc)["bc"]
            dn = self.iterate(dl, A_ind, bc)["delta_new"]
            term = np.zeros((ny, nx))
            for c in range(self.ncomp):
                term += 2.0 * den[c] * (np.conj(delta[c]) * dn[c]).real
            integral += wv * term
        om = self.condensation_base(delta) - np.where(m, integral, 0.0)
        h = self.grid.h
        total = h * h * om.sum()
        if self.kappa > 0.0:
            b = fields.curl(A_ind[0], A_ind[1], h)
            total += h * h * np.sum(0.5 * self.kappa ** 2 * b * b)
        return om, total

    # -- LDOS ---------------------------------------------------------------
    def ldos(self, delta, A_ind, energies, broadening, bc_iters):
        """Angle-averaged local density of states N(R, e)/N_F =
        <-Im g^R / pi> (Sec. II) with z = e + i delta + q a, Delta and A
        frozen.  bc_iters sweeps only update the boundary values (burn-in,
        App. B); one more sweep gives the output.  Returns [E, ny, nx]."""
        ny, nx = self.grid.ny, self.grid.nx
        delta = np.asarray(delta, dtype=np.complex128).reshape(self.ncomp, ny, nx)
        A_ind = np.asarray(A_ind, dtype=np.float64).reshape(2, ny, nx)
        eps = np.asarray(energies, dtype=np.float64) + 1j * broadening
        m = self.mask
        ncell = int(m.sum())
        bc = None
        vals = [self.data(k) for k in range(self.n_theta)]
        nodev = [self.node_values(k, vals[k], delta, A_ind) for k in range(self.n_theta)]
        for it in range(bc_iters + 1):
            gend, gtend = [], []
            out = np.zeros((len(eps), ncell))
            for k in range(self.n_theta):
                data = vals[k]
                dnode, anode = nodev[k]
                g0, gt0 = self.start_values(k, data, dnode, anode, eps, bc)
                gn, gtn, ge, gte = sweep.march(data, dnode, anode, eps, self.q, g0, gt0)
                gend.append(ge)
                gtend.append(gte)
                if it == bc_iters:
                    g, _, _ = sweep.green(gn, gtn)
                    nval = -g.imag / math.pi                  # [S, W, E]
                    seg, pos, w = self.rb_stencil(k)
                    cell = np.sum(nval[seg, pos, :] * w[:, :, None], axis=1)  # [ncell, E]
                    out += self.wk[k] * cell.T
            bc = (gend, gtend)
        res = np.zeros((len(eps), ny, nx))
        res[:, m] = out
        return res


def rel_norm(new, old, p=2):
    """Global error of Eq. global_error: ||new - old||_p / ||old||_p
    (0 when both vanish, inf when only the old one does)."""
    a = np.asarray(new - old).ravel()
    b = np.asarray(old).ravel()
    if p == np.inf or p == 0:
        num, den = np.max(np.abs(a)) if a.size else 0.0, np.max(np.abs(b)) if b.size else 0.0
    else:
        num = np.sum(np.abs(a) ** p) ** (1.0 / p)
        den = np.sum(np.abs(b) ** p) ** (1.0 / p)
    if den == 0.0:
        return 0.0 if num == 0.0 else math.inf
    return num / den


def polyak_step(x, v, gx, alpha, beta):
    """Polyak's heavy-ball update of App. E: the velocity v relaxes with
    drag beta toward alpha times the difference d = g(x) - x, and x moves
    by the new velocity.  Returns (x_next, v_next)."""
    v_next = (1.0 - beta) * v + alpha * (gx - x)
    return x + v_next, v_next


BB_STEP_MIN, BB_STEP_MAX = 1e-3, 1e2  # App. E's default bounds of the BB step


def bb_step_size(alpha, d, d_prev, i, amin=BB_STEP_MIN, amax=BB_STEP_MAX):
    """Barzilai-Borwein step size of App. E for accelerated iteration i
    (counted from 0): alpha_{i+1} = alpha_i s_i with s_i = |d_{i-1}|^2 /
    |d_{i-1}.(d_i - d_{i-1})| for odd i and |d_{i-1}.(d_i - d_{i-1})| /
    |d_i - d_{i-1}|^2 for even i, clamped to [amin, amax].  A zero
    denominator keeps alpha_i.  d_prev is None for the first iteration,
    which keeps the initial step."""
    if d_prev is None:
        return alpha
    diff = d - d_prev
    pd = abs(float(np.dot(d_prev, diff)))
    num, den = (float(np.dot(d_prev, d_prev)), pd) if i % 2 == 1 else (pd, float(np.dot(diff, diff)))
    if den == 0.0:
        return alpha
    return min(max(alpha * num / den, amin), amax)


# App. E's CongAcc defaults: first step, step factor k, minimum similarity,
# step bounds
CONG_STEP, CONG_K, CONG_SMIN, CONG_STEP_MIN, CONG_STEP_MAX = 0.5, 1.234, 0.7, 1e-3, 1e2
# Similarities at or below -1 + CONG_ANTI count as anti-parallel m and d.
CONG_ANTI = 1e-9


def similarity_weight(mm, md, dd, smin, n_bisect=60):
    """The weight w* in [0, 1] at which the cosine similarity of
    w m + (1 - w) d with d equals smin (App. E), by bisection, from the dot
    products m.m, m.d and d.d.  At w = 0 the similarity is 1; the caller
    applies it only when the similarity at w = 1 is below smin."""
    def sim(w):
        uu = w * w * mm + 2.0 * w * (1.0 - w) * md + (1.0 - w) * (1.0 - w) * dd
        return (w * md + (1.0 - w) * dd) / math.sqrt(uu * dd) if uu > 0.0 else 1.0
    lo, hi = 0.0, 1.0
    for _ in range(n_bisect):
        mid = 0.5 * (lo + hi)
        if sim(mid) >= smin:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def congacc_component(m, d, alpha, w, first, k=CONG_K, smin=CONG_SMIN, amin=CONG_STEP_MIN, amax=CONG_STEP_MAX,
                      stats=None):
    """CongAcc (App. E) for one component c of x (the real or imaginary part
    of one order-parameter component, or one component of A): the cosine
    similarity s of the moving average m with the difference d scales the
    step, alpha <- alpha k^s (clamped); the weight w is kept while s >= smin
    and otherwise replaced by similarity_weight; m <- w m + (1 - w) d.  The
    first iteration takes w = 0 (so m = d) and keeps alpha; a similarity
    with a zero vector is read as 0.
    When m and d are anti-parallel (s <= -1 + CONG_ANTI) the blend
    w m + (1 - w) d is a multiple of d that changes sign at one weight: its
    similarity with d jumps from 1 to -1 there, so the equation for w* has
    no root, and a bisection would stop where the blend vanishes.  That
    case takes w = 0: the average restarts from d (and alpha has just
    shrunk by k^-1).
    stats (a dict, optional) counts the weights set by bisection ("bisect")
    and by the anti-parallel rule ("anti").  Returns (m_next, alpha_next,
    w_next); the step is x <- x + alpha_next m_next."""
    if first:
        return d.copy(), alpha, 0.0
    mm, md, dd = float(np.dot(m, m)), float(np.dot(m, d)), float(np.dot(d, d))
    s = md / math.sqrt(mm * dd) if mm > 0.0 and dd > 0.0 else 0.0
    alpha = min(max(alpha * k ** s, amin), amax)
    if s < smin and mm > 0.0 and dd > 0.0:
        if s <= -1.0 + CONG_ANTI:
            w = 0.0
            key = "anti"
        else:
            w = similarity_weight(mm, md, dd, smin)
            key = "bisect"
        if stats is not None:
            stats[key] = stats.get(key, 0) + 1
    return w * m + (1.0 - w) * d, alpha, w


def scf(grain, delta, A_ind, n_iter, alpha=1.0, burnin=0, norm_p=2, accelerator="picard", beta=0.5, stats=None):
    """Self-consistency (App. E) on x = (Re Delta_G, Im Delta_G on grain
    cells, kappa^2 A_ind on all cells), with A from the current of the same
    iteration (App. D).  accelerator "picard": x <- x + alpha (g(x) - x);
    "polyak": the heavy-ball step (polyak_step) with step size alpha and
    drag beta, the velocity starting at zero.  The kappa^2 scale of A drops
    out of both updates, which are linear in x.  "bb": x <- x + alpha_i d
    with the Barzilai-Borwein step (bb_step_size) from the dot products of
    the concatenated d, where kappa^2 does enter; alpha is the first step.
    "congacc": per component of x (congacc_component), alpha the first step
    of every component; kappa^2 drops out again.  During the first `burnin`
    iterations Delta and A stay fixed and only the boundary values update
    (App. B).
    Convergence is checked before the accelerator moves x (Alg. 1): eps_Delta
    and eps_A are Eq. global_error of g(x) against x, i.e. ||d|| / ||x|| per
    field; eps_j and eps_Omega compare with the previous iteration.
    kappa <= 0 (no screening) has no induced vector potential: A_ind is set
    to zero before the first sweep and stays zero (eps_A = 0).
    stats: optional dict passed to congacc_component; it also collects the
    components whose weight was bisected ("bisect_components").  Returns the final
    fields, the per-iteration history of (eps_Delta, eps_j, eps_A,
    eps_Omega, Omega) and the boundary values of the last sweep."""
    if accelerator not in ("picard", "polyak", "bb", "congacc"):
        raise ValueError("unknown accelerator %r" % (accelerator,))
    ny, nx = grain.grid.ny, grain.grid.nx
    delta = np.array(delta, dtype=np.complex128).reshape(grain.ncomp, ny, nx)
    A = np.array(A_ind, dtype=np.float64).reshape(2, ny, nx)
    if grain.kappa <= 0.0:
        A[:] = 0.0
    m = grain.mask
    bc = None
    hist = []
    j_old = None
    om_old = None
    v_d = np.zeros_like(delta)
    v_a = np.zeros_like(A)
    a_bb, d_prev, i_bb = alpha, None, 0
    ncomp_x = 2 * grain.ncomp + 2
    cg = [None] * ncomp_x, [alpha] * ncomp_x, [0.0] * ncomp_x  # m, alpha, w per component
    cg_first = True
    ksc = grain.kappa ** 2 if grain.kappa > 0.0 else 1.0
    for it in range(n_iter):
        out = grain.iterate(delta, A, bc)
        bc = out["bc"]
        j = out["j"]
        om = out["omega_total"]
        if it < burnin:
            hist.append((0.0, 0.0, 0.0, 0.0, om))
            j_old, om_old = j, om
            continue
        ax, ay = fields.solve_A(j[0], j[1], m, grain.grid.h, grain.kappa)
        A_new = np.stack([ax, ay])
        if accelerator == "congacc":
            dD = out["delta_new"] - delta
            dA = A_new - A
            parts = []
            for g_ in range(grain.ncomp):
                parts += [dD[g_][m].real.copy(), dD[g_][m].imag.copy()]
            parts += [dA[0].ravel().copy(), dA[1].ravel().copy()]
            d_new = delta.copy()
            A_next = A.copy()
            for c, dc in enumerate(parts):
                nb = stats.get("bisect", 0) if stats is not None else 0
                mc, ac, wc = congacc_component(cg[0][c], dc, cg[1][c], cg[2][c], cg_first, stats=stats)
                if stats is not None and stats.get("bisect", 0) > nb:
                    stats.setdefault("bisect_components", set()).add(c)
                cg[0][c], cg[1][c], cg[2][c] = mc, ac, wc
                step = ac * mc
                if c < 2 * grain.ncomp:
                    g_, im = divmod(c, 2)
                    d_new[g_][m] += 1j * step if im else step
                else:
                    A_next[c - 2 * grain.ncomp] += step.reshape(ny, nx)
            cg_first = False
        elif accelerator == "bb":
            dD = out["delta_new"] - delta
            dA = A_new - A
            dvec = np.concatenate([dD[:, m].real.ravel(), dD[:, m].imag.ravel(), ksc * dA.ravel()])
            a_bb = bb_step_size(a_bb, dvec, d_prev, i_bb)
            d_prev, i_bb = dvec, i_bb + 1
            d_new = delta + a_bb * dD
            A_next = A + a_bb * dA
        elif accelerator == "polyak":
            d_new, v_d = polyak_step(delta, v_d, out["delta_new"], alpha, beta)
            A_next, v_a = polyak_step(A, v_a, A_new, alpha, beta)
        else:
            d_new = delta + alpha * (out["delta_new"] - delta)
            A_next = A + alpha * (A_new - A)
        d_new[:, ~m] = 0.0
        e_d = rel_norm(out["delta_new"][:, m], delta[:, m], norm_p)
        e_a = rel_norm(A_new, A, norm_p)
        e_j = rel_norm(j, j_old, norm_p) if j_old is not None else math.inf
        e_o = abs(om - om_old) / abs(om_old) if (om_old is not None and om_old != 0.0) else math.inf
        hist.append((e_d, e_j, e_a, e_o, om))
        delta, A = d_new, A_next
        j_old, om_old = j, om
    return delta, A, hist, bc
