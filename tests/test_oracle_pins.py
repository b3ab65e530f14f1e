"""Further pins of the oracle: the external gauges, the LDOS post-process,
the gauge covariance of the whole map with an induced vector potential, the
continuity equation, the sampled-cell evaluation, and closed-form segment
end points of the trajectory tables."""
import math

import numpy as np
import pytest

from oracle import geometry as geo, sweep, scf, bulk, fields


# --------------------------------------------------- external field (App. F)
@pytest.mark.parametrize("gauge", ["symmetric", "landau"])
def test_uniform_gauges_have_the_flux_density_of_the_unit_table(gauge):
    """alpha flux quanta through the area A give B = alpha Phi0 / A; with
    B0 = Phi0 / (pi xi0^2) that is pi alpha / A.  Both linear gauges have
    this curl everywhere (central differences are exact on linear fields),
    and the line integral around a circle is B times its area."""
    area, alpha, cx, cy = 37.5, 1.7, 0.3, -0.2
    h = 0.25
    x = cx + (np.arange(40) - 19.5) * h
    X, Y = np.meshgrid(x, x)
    ax, ay = fields.external_A(gauge, alpha, area, cx, cy, X, Y)
    b = fields.curl(ax, ay, h)
    assert np.max(np.abs(b[1:-1, 1:-1] - math.pi * alpha / area)) < 1e-12
    th = np.linspace(0, 2 * math.pi, 4001)[:-1]
    R = 2.0
    px, py = cx + R * np.cos(th), cy + R * np.sin(th)
    qx, qy = fields.external_A(gauge, alpha, area, cx, cy, px, py)
    circ = np.sum(qx * (-np.sin(th)) + qy * np.cos(th)) * R * (2 * math.pi / len(th))
    assert abs(circ - math.pi * alpha / area * math.pi * R * R) < 1e-12


def test_solenoid_gauge_is_curl_free_and_encloses_alpha_quanta():
    """The solenoid field alpha/(2r) phi-hat: zero curl off the centre, and
    a line integral of pi alpha (alpha flux quanta in units of A0 xi0 =
    Phi0/pi) around any loop that encloses the centre, zero otherwise."""
    alpha = 0.8
    errs = []
    for h in (0.1, 0.05):
        n = int(round(2.0 / h)) + 1
        x = 3.0 + (np.arange(n) - (n - 1) / 2) * h      # a patch away from the centre
        X, Y = np.meshgrid(x, x - 2.0)
        ax, ay = fields.external_A("solenoid", alpha, 10.0, 0.0, 0.0, X, Y)
        b = fields.curl(ax, ay, h)
        errs.append(np.max(np.abs(b[1:-1, 1:-1])))
    # the central differences of a curl-free field: O(h^2) remainder only
    assert errs[1] < 1e-3 * alpha and 3.5 < errs[0] / errs[1] < 4.5, errs
    th = np.linspace(0, 2 * math.pi, 2001)[:-1]
    for (ox, oy, R, inside) in ((0.4, -0.3, 1.5, True), (3.0, 1.0, 1.0, False)):
        px, py = ox + R * np.cos(th), oy + R * np.sin(th)
        qx, qy = fields.external_A("solenoid", alpha, 10.0, 0.0, 0.0, px, py)
        circ = np.sum(qx * (-np.sin(th)) + qy * np.cos(th)) * R * (2 * math.pi / len(th))
        assert abs(circ - (math.pi * alpha if inside else 0.0)) < 1e-9


# ----------------------------------------------------- LDOS (Sec. II, App. B)
def _bcs_dos(e, broad, d):
    z = e + 1j * broad
    s = np.sqrt(z * z - d * d + 0j)
    s = np.where(s.imag < 0, -s, s)              # retarded branch, Im s > 0
    return (z / s).real


@pytest.mark.parametrize("bc_iters", [0, 2])
def test_ldos_of_a_uniform_s_wave_grain_is_the_bcs_density_of_states(bc_iters):
    """A uniform s-wave gap with no field: the bulk root is left unchanged
    by every step and by specular reflection, so every grain cell carries the
    bulk density of states N/N_F = Re[z / sqrt(z^2 - |Delta|^2)] with
    z = e + i delta, for any number of burn-in sweeps."""
    gr = scf.Grain(22, 22, 0.6, [geo.Disc(0.1, -0.2, 6.0)], 12, 4, 0.5)
    d0 = 0.26 * np.exp(0.7j)
    delta = np.where(gr.mask, d0, 0)[None]
    e = np.array([-0.5, -0.2, 0.0, 0.1, 0.25, 0.27, 0.4])
    broad = 0.02
    out = gr.ldos(delta, np.zeros((2, 22, 22)), e, broad, bc_iters)
    ref = _bcs_dos(e, broad, abs(d0))
    assert np.max(np.abs(out[:, gr.mask] - ref[:, None])) < 1e-12
    assert np.all(out[:, ~gr.mask] == 0.0)


def test_ldos_zero_energy_peak_on_a_110_edge_needs_the_burn_in():
    """d-wave with [110] edges: every reflection changes the sign of the gap,
    and the converged boundary values give N(0)/N_F = sqrt(|D_phi|^2 +
    delta^2)/delta on each trajectory at the wall.  A wall cell sits within a
    cell of the wall, so its angle average approaches <sqrt(|D_phi|^2 +
    delta^2)>/delta (bounded above by it); without burn-in the starts are
    bulk roots and the cell shows the gapped bulk value instead."""
    t, npol, nth = 0.1, 4, 16
    gr = scf.Grain(40, 40, 0.3, [geo.regular_polygon(0, 0, 4, 11.7)], nth, npol, t,
                   components=(("dx2y2", 1.0),), crystal_rotation=0.125)
    d0 = 0.25
    delta = np.where(gr.mask, d0, 0)[None].astype(complex)
    broad = 0.08
    X, Y = gr.grid.centres()
    # grain cells next to the middle of the bottom edge
    row = np.nonzero(gr.mask.any(axis=1))[0][0]
    cols = np.nonzero(gr.mask[row] & (np.abs(X[row]) < 1.5))[0]
    zes = np.sum(gr.wk * np.sqrt((d0 * np.abs(gr.eta[0])) ** 2 + broad ** 2)) / broad
    bulk_v = np.sum(gr.wk * broad / np.sqrt((d0 * np.abs(gr.eta[0])) ** 2 + broad ** 2))
    n0 = gr.ldos(delta, np.zeros((2, 40, 40)), [0.0], broad, 0)[0, row, cols]
    n8 = gr.ldos(delta, np.zeros((2, 40, 40)), [0.0], broad, 8)[0, row, cols]
    assert np.all(n8 > 0.6 * zes) and np.all(n8 < 1.02 * zes), (n8, zes)
    assert np.all(n0 < 0.5 * n8), (n0, n8, bulk_v)


# ----------------------------------- gauge covariance with A_ind (Sec. V.A)
def _gauge_case(h, shift):
    """Disc grain with a smooth complex gap, a smooth induced A and an
    external solenoid field; shift = 0 or 1 applies the gauge
    transformation Delta -> Delta e^{i L}, A_ind -> A_ind + (q/2) grad L."""
    R = 5.2
    n = int(round(2 * (R + 0.8) / h))
    gr = scf.Grain(n, n, h, [geo.Disc(0.0, 0.0, R)], 16, 4, 0.5, components=(("s", 1.0),),
                   kappa=3.0, flux_quanta=0.3, gauge="solenoid")
    X, Y = gr.grid.centres()
    delta = (0.24 + 0.03 * np.cos(0.5 * X) + 0.02j * np.sin(0.4 * Y)) * np.exp(0.15j * X)
    A = np.stack([0.03 * np.sin(0.3 * Y + 0.2), 0.02 * np.cos(0.25 * X)])
    lam = 0.35 * X - 0.2 * Y + 0.3 * np.sin(0.4 * X + 0.3 * Y)
    glx = 0.35 + 0.12 * np.cos(0.4 * X + 0.3 * Y)
    gly = -0.2 + 0.09 * np.cos(0.4 * X + 0.3 * Y)
    if shift:
        delta = delta * np.exp(1j * lam)
        A = A + 0.5 * gr.q * np.stack([glx, gly])
    delta = np.where(gr.mask, delta, 0)[None]
    return gr, delta, A, lam


def _frozen_iterations(gr, delta, A, n):
    bc = None
    for _ in range(n):
        o = gr.iterate(delta, A, bc)
        bc = o["bc"]
    return o


def test_gauge_transformation_with_induced_field_is_covariant_to_second_order():
    """(Delta e^{iL}, A_ind + (q/2) grad L) gives Delta_new e^{iL} with the
    same j and free-energy density: exact for the continuum equations,
    O(h^2) for the discrete map (bilinear interpolation of the phase, and
    the boundary taps between lines), after the boundary values have
    forgotten the bulk-root starts (frozen fields, several sweeps).  This
    exercises the clamped bilinear A_ind stencil and the q v.A term of z: a
    wrong sign or factor there breaks the covariance at O(1)."""
    errs = []
    for h in (0.5, 0.25):
        res = []
        for shift in (0, 1):
            gr, d, A, lam = _gauge_case(h, shift)
            res.append(_frozen_iterations(gr, d, A, 4))
        o0, o1 = res
        m = gr.mask
        X, Y = gr.grid.centres()
        inner = m & (np.hypot(X, Y) < 3.5)
        dn0 = o0["delta_new"][0] * np.exp(1j * lam)
        e_d = np.max(np.abs(o1["delta_new"][0] - dn0)[inner]) / np.max(np.abs(dn0[m]))
        e_j = np.max(np.abs(o1["j"] - o0["j"])[:, inner]) / np.max(np.abs(o0["j"][:, m]))
        errs.append((e_d, e_j))
    (d1, j1), (d2, j2) = errs
    # h = 0.5 / 0.25 / 0.125 give 1.5e-2 / 4.1e-3 / 1.3e-3 (Delta_new) and
    # 1.6e-2 / 5.3e-3 / 2.0e-3 (j)
    assert d2 < 6e-3 and j2 < 8e-3, errs
    assert d1 / d2 > 3.0 and j1 / j2 > 2.5, errs


def test_wrong_charge_in_the_gauge_shift_is_not_covariant():
    """Control for the test above: the opposite shift of A breaks it."""
    h = 0.5
    gr, d0_, A0, lam = _gauge_case(h, 0)
    _, d1_, A1, _ = _gauge_case(h, 1)
    A_bad = 2 * A0 - A1                          # A_ind - (q/2) grad L
    o0 = _frozen_iterations(gr, d0_, A0, 4)
    o1 = _frozen_iterations(gr, d1_, A_bad, 4)
    m = gr.mask
    X, Y = gr.grid.centres()
    inner = m & (np.hypot(X, Y) < 3.5)
    e_j = np.max(np.abs(o1["j"] - o0["j"])[:, inner]) / np.max(np.abs(o0["j"][:, m]))
    assert e_j > 0.2


# ------------------------------------------- continuity equation (Sec. II)
def test_current_divergence_equals_the_gap_equation_source():
    """Along a trajectory the Riccati equations give v.grad g = i(D f~ - D* f)
    (z drops out), so for any Delta and A the current of Eq. current_density
    and the gap-equation numerator of Eq. gapeq_fixpoint obey
      div j = 4 q sum_G den_G Im(conj(Delta_G) Delta_G,new)
    at every point, per angle and pole; it vanishes at self-consistency
    (current conservation).  The discrete map satisfies it to O(h^2): the
    residual falls about fourfold when h halves."""
    res = []
    for h in (0.4, 0.2):
        R = 5.0
        n = int(round(2 * (R + 0.6) / h))
        gr = scf.Grain(n, n, h, [geo.Disc(0.0, 0.0, R)], 16, 4, 0.5, components=(("s", 1.0),),
                       kappa=2.0, flux_quanta=0.0)
        X, Y = gr.grid.centres()
        delta = np.where(gr.mask, (0.22 + 0.04 * np.cos(0.6 * X) * np.sin(0.5 * Y)) * np.exp(0.25j * X + 0.1j * Y),
                         0)[None]
        A = np.stack([0.04 * np.sin(0.3 * Y), 0.03 * np.cos(0.35 * X)])
        o = _frozen_iterations(gr, delta, A, 3)
        jx, jy = o["j"]
        div = np.zeros_like(jx)
        div[1:-1, 1:-1] = (jx[1:-1, 2:] - jx[1:-1, :-2] + jy[2:, 1:-1] - jy[:-2, 1:-1]) / (2 * h)
        src = 4 * gr.q * gr.gap_denominator()[0] * np.imag(np.conj(delta[0]) * o["delta_new"][0])
        inner = gr.mask & (np.hypot(X, Y) < 3.0)
        scale = np.max(np.abs(src[inner]))
        res.append((np.max(np.abs(div - src)[inner]) / scale, scale))
    (r1, s1), (r2, s2) = res
    assert s1 > 1e-3
    assert r2 < 2e-2 and r1 / r2 > 3.0, res


# --------------------------------------------- sampled cells (full sizes)
def test_iterate_cells_equals_the_full_map_at_its_cells():
    """iterate_cells sweeps only the segments feeding the sampled cells; from
    bulk starts it must give the full map's values there."""
    gr = scf.Grain(26, 24, 0.5, [geo.Disc(0.2, 0.1, 5.8), geo.regular_polygon(1.0, -0.5, 4, 2.5, 0.1, add=False)],
                   12, 5, 0.4, components=(("s", 1.0), ("dxy", 0.7)), kappa=2.0, flux_quanta=0.6)
    rng = np.random.default_rng(8)
    X, Y = gr.grid.centres()
    delta = np.stack([0.22 * np.exp(-1j * np.arctan2(Y - 0.4, X + 0.3)), 0.05 * np.exp(0.3j * X)])
    delta = np.where(gr.mask[None], delta + 0.01 * rng.standard_normal(delta.shape), 0)
    A = np.stack([0.03 * np.sin(0.4 * Y), 0.02 * np.cos(0.3 * X)])
    full = gr.iterate(delta, A)
    cells = np.sort(rng.choice(np.flatnonzero(gr.mask), 30, replace=False))
    dn, j = gr.iterate_cells(delta, A, cells)
    scale = np.max(np.abs(full["delta_new"]))
    assert np.max(np.abs(dn - full["delta_new"].reshape(2, -1)[:, cells])) < 1e-13 * scale
    assert np.max(np.abs(j - full["j"].reshape(2, -1)[:, cells])) < 1e-13 * np.max(np.abs(full["j"]))


# ----------------------------------- trajectory end points (Sec. III.A)
@pytest.mark.parametrize("phi", [0.0, 0.37, 1.2, 2.9])
def test_disc_segment_ends_are_the_chord_ends(phi):
    """A line at distance u from the centre of a disc of radius R meets it
    at s = s_c +- sqrt(R^2 - u^2) (s_c the foot of the centre on the line)."""
    grid = geo.Grid(30, 30, 0.5)
    cx, cy, R = 0.4, -0.3, 6.1
    tab = geo.AngleTable(grid, [geo.Disc(cx, cy, R)], phi)
    ex, ey = math.cos(phi), math.sin(phi)
    for s in range(tab.nseg):
        px, py = tab.point(tab.seg_line[s], 0.0)
        # offset of the line from the disc centre, and the foot's parameter
        dx, dy = cx - px, cy - py
        sc = dx * ex + dy * ey
        u2 = dx * dx + dy * dy - sc * sc
        half = math.sqrt(R * R - u2)
        assert abs(tab.smin[s] - (sc - half)) < 1e-10 and abs(tab.smax[s] - (sc + half)) < 1e-10


@pytest.mark.parametrize("phi", [0.21, 0.9, 2.2])
def test_square_segment_ends_are_the_edge_crossings(phi):
    """An axis-aligned square [-a, a]^2 crossed by the line p + s e: the
    inside interval is the intersection of the slabs |p_x + s e_x| <= a and
    |p_y + s e_y| <= a."""
    grid = geo.Grid(28, 28, 0.5)
    a = 5.3
    tab = geo.AngleTable(grid, [geo.regular_polygon(0.0, 0.0, 4, 2 * a)], phi)
    ex, ey = math.cos(phi), math.sin(phi)
    for s in range(tab.nseg):
        px, py = tab.point(tab.seg_line[s], 0.0)
        lo, hi = -math.inf, math.inf
        for p, e in ((px, ex), (py, ey)):
            t1, t2 = (-a - p) / e, (a - p) / e
            lo, hi = max(lo, min(t1, t2)), min(hi, max(t1, t2))
        assert abs(tab.smin[s] - lo) < 1e-10 and abs(tab.smax[s] - hi) < 1e-10


# ------------------------------- Luttinger-Ward free energy (Sec. II)
@pytest.mark.parametrize("bc_iters", [0, 1])
def test_luttinger_ward_form_of_a_uniform_s_wave_state_is_the_bulk_free_energy(bc_iters):
    """In a uniform s-wave state f_lambda = pi lambda Delta/sqrt(e^2 +
    lambda^2 |Delta|^2), so int_0^1 dlambda (Delta* f_lambda + Delta
    f~_lambda) = 2 pi (Omega_n - |e_n|) and Eq. qcLWFE becomes
    |D|^2 ln t + pi T sum_n |D|^4 / (|e_n| (Omega_n + |e_n|)^2) (Eq. FEbulk):
    -0.020601374 at t = 0.5 with 16 poles at the BCS gap.  The integrand is
    analytic in lambda, so 12 Gauss-Legendre nodes reach rounding level; 4
    do not."""
    gr = scf.Grain(32, 32, 0.625, [geo.Disc(0, 0, 10)], 32, 16, 0.5)
    db = bulk.bulk_gap(0.5, 16)
    delta = np.where(gr.mask, db * np.exp(0.3j), 0)[None]
    ref = bulk.bulk_free_energy(db, 0.5, 16)
    assert abs(ref + 0.020601374) < 1e-9
    om, tot = gr.free_energy_lw(delta, np.zeros((2, 32, 32)), 12, bc_iters)
    assert np.max(np.abs(om[gr.mask] - ref)) < 1e-14
    assert np.all(om[~gr.mask] == 0.0)
    assert abs(tot - gr.area * ref) < 1e-12 * abs(gr.area * ref)
    om4, _ = gr.free_energy_lw(delta, np.zeros((2, 32, 32)), 4, bc_iters)
    assert np.max(np.abs(om4[gr.mask] - ref)) > 1e-8


def test_luttinger_ward_equals_the_eilenberger_form_in_a_uniform_d_wave_square():
    """d_{x2-y2} in an axis-aligned square keeps its bulk state exactly (no
    pair breaking at [100] edges), so both forms of the free energy give the
    angle-resolved bulk value (Eq. FEbulk with |Delta(p)|^2 = |eta|^2 D^2);
    near the gap nodes the lambda integrand is less smooth and needs 24
    nodes."""
    t, npol, nth = 0.2, 16, 16
    gr = scf.Grain(30, 30, 0.5, [geo.regular_polygon(0, 0, 4, 12.0)], nth, npol, t, components=(("dx2y2", 1.0),))
    e2 = np.abs(gr.eta[0]) ** 2
    db = bulk.bulk_gap(t, npol, e2, gr.wk)
    delta = np.where(gr.mask, db, 0)[None].astype(complex)
    A = np.zeros((2, 30, 30))
    ref = bulk.bulk_free_energy(db, t, npol, e2, gr.wk)
    eil = gr.iterate(delta, A)["omega_density"]
    om, _ = gr.free_energy_lw(delta, A, 24, 1)
    assert np.max(np.abs(eil[gr.mask] - ref)) < 1e-14
    assert np.max(np.abs(om[gr.mask] - ref)) < 1e-14


def test_luttinger_ward_propagator_term_is_linear_in_the_lambda_integrand():
    """The lambda integral of Eq. qcLWFE_I at one node reduces to the gap
    numerator of the scaled sweep: with a single Gauss-Legendre node
    (lambda = 1/2, weight 1) the propagator term is 2 den Re(conj(Delta)
    Delta_new[Delta/2]) at every cell, for any state (here a vortex with a
    field)."""
    gr = scf.Grain(24, 24, 0.5, [geo.Disc(0, 0, 5.4)], 12, 5, 0.4, kappa=2.0, flux_quanta=0.7)
    X, Y = gr.grid.centres()
    delta = np.where(gr.mask, 0.22 * np.exp(-1j * np.arctan2(Y - 0.3, X + 0.4)), 0)[None]
    A = np.stack([0.03 * np.sin(0.4 * Y), 0.02 * np.cos(0.3 * X)])
    om, tot = gr.free_energy_lw(delta, A, 1, 0)
    dn = gr.iterate(0.5 * delta, A)["delta_new"]
    term = 2 * gr.gap_denominator()[0] * np.real(np.conj(delta[0]) * dn[0])
    base = gr.condensation_base(delta)
    assert np.max(np.abs(om - (base - np.where(gr.mask, term, 0)))) < 1e-15


# ---- eigen-truncated A-solve and magnetic moment (App. D, Sec. V.A) ----

def test_truncation_rank_is_the_smallest_count_meeting_the_tolerance():
    """N* of App. D on a hand-made spectrum: lam^2 = 16, 4, 1, 1/4 (total
    21.25); the tail norms sqrt(sum_{n>=k} lam^2 / total) are 1, 0.497,
    0.2425, 0.1085, 0 for k = 0..4, in whatever order and sign the
    eigenvalues come."""
    lam = [0.5, -2.0, 4.0, 1.0]
    assert fields.truncation_rank(lam, 1.1) == 0
    assert fields.truncation_rank(lam, 0.5) == 1
    assert fields.truncation_rank(lam, 0.3) == 2
    assert fields.truncation_rank(lam, 0.11) == 3
    assert fields.truncation_rank(lam, 0.1) == 4
    assert fields.truncation_rank(lam, 1e-12) == 4


def _random_current(n, seed):
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(np.arange(n) - n / 2 + 0.5, np.arange(n) - n / 2 + 0.5)
    mask = X ** 2 + Y ** 2 < (0.45 * n) ** 2
    return rng.standard_normal((n, n)), rng.standard_normal((n, n)), mask


def test_eigen_A_with_every_mode_is_the_direct_sum():
    """With every eigenpair kept, sum_k lam_k T_k J T_k is the full
    correlation with G (App. D): the eigen path equals the direct double
    sum on a 24 x 24 grid to rounding, for both components."""
    jx, jy, mask = _random_current(24, 5)
    ax, ay = fields.solve_A(jx, jy, mask, 0.4, 2.5, method="direct")
    ex, ey, nstar = fields.solve_A_eigen(jx, jy, mask, 0.4, 2.5, 1e-300)
    assert nstar == 24
    assert np.max(np.abs(ex - ax)) <= 1e-11 * np.max(np.abs(ax))
    assert np.max(np.abs(ey - ay)) <= 1e-11 * np.max(np.abs(ay))


def test_eigen_A_truncation_error_is_bounded_by_the_tolerance():
    """Keeping N* modes changes the kernel by dK with ||dK||_F <= eps ||G||_F
    (the criterion of App. D), so each A element moves by at most
    2 kappa^-2 ||dK||_F ||j'||_2 (Cauchy-Schwarz; every offset appears at
    most four times).  Checked at eps = 1e-3 on a 32 x 32 grid, where the
    truncation keeps only a few modes."""
    n, h, kappa, eps = 32, 0.5, 1.5, 1e-3
    jx, jy, mask = _random_current(n, 6)
    ax, ay = fields.solve_A(jx, jy, mask, h, kappa, method="direct")
    ex, ey, nstar = fields.solve_A_eigen(jx, jy, mask, h, kappa, eps)
    assert 1 <= nstar < n // 2
    G = fields.green_matrix(n, h)
    lam, V = fields.green_eigen(n, h, eps)
    dK = np.linalg.norm(G - (V * lam) @ V.T)
    assert dK < eps * np.linalg.norm(G)
    for a, e, j in ((ax, ex, jx), (ay, ey, jy)):
        jp = np.where(mask, j - j[mask].mean(), 0.0)
        bound = 2.0 / kappa ** 2 * dK * np.linalg.norm(jp)
        assert 0.0 < np.max(np.abs(e - a)) <= bound


def test_magnetic_moment_of_a_rigidly_rotating_disc():
    """j = w z x R on a disc of radius R (Sec. V.A, Eq. magnetic_moment_def):
    m_z / m0 = (1 / 2A) int r^2 w dR = w R^2 / 4 in the continuum; the cell
    sum converges to it as h -> 0."""
    errs = []
    for h in (0.4, 0.2, 0.1):
        n = int(round(24.0 / h))
        g = geo.Grid(n, n, h)
        X, Y = g.centres()
        mask = g.mask([geo.Disc(0.0, 0.0, 10.0)])
        w = 0.3
        m = fields.magnetic_moment(-w * Y, w * X, mask, X, Y, g.cx, g.cy)
        errs.append(abs(m - w * 100.0 / 4.0) / (w * 100.0 / 4.0))
    assert errs[-1] < 1e-2 and errs[-1] < errs[0]


def test_magnetic_moment_of_an_annulus_with_azimuthal_current():
    """Uniform azimuthal current j0 on R< <= r <= R>: m_z / m0 =
    j0 2 pi (R>^3 - R<^3) / 3 / (2 pi (R>^2 - R<^2))."""
    h, n, r1, r2, j0 = 0.1, 240, 4.0, 11.0, 0.7
    g = geo.Grid(n, n, h)
    X, Y = g.centres()
    mask = g.mask([geo.Disc(0.0, 0.0, r2), geo.Disc(0.0, 0.0, r1, False)])
    r = np.hypot(X, Y)
    jx, jy = -j0 * Y / r, j0 * X / r
    m = fields.magnetic_moment(jx, jy, mask, X, Y, g.cx, g.cy)
    ref = j0 * (r2 ** 3 - r1 ** 3) / (3.0 * (r2 ** 2 - r1 ** 2))
    assert abs(m - ref) < 5e-3 * ref


def test_magnetic_moment_is_origin_independent_without_net_current():
    """sum over cells of (R - O) x j does not depend on O when sum j = 0."""
    n, h = 30, 0.5
    g = geo.Grid(n, n, h)
    X, Y = g.centres()
    mask = g.mask([geo.Disc(0.0, 0.0, 6.5)])
    rng = np.random.default_rng(8)
    jx, jy = rng.standard_normal((2, n, n))
    jx = np.where(mask, jx - jx[mask].mean(), 0.0)
    jy = np.where(mask, jy - jy[mask].mean(), 0.0)
    m0 = fields.magnetic_moment(jx, jy, mask, X, Y, g.cx, g.cy)
    m1 = fields.magnetic_moment(jx, jy, mask, X, Y, g.cx + 3.7, g.cy - 1.2)
    assert abs(m1 - m0) < 1e-12 * max(abs(m0), 1.0)


# ------------------------------------- screened annulus (Sec. V.A closed forms)
from oracle import annulus  # noqa: E402

_RING = (25.0, 10.0)


@pytest.mark.parametrize("lam,alpha,n", [(2.0, 0.5, 0), (5.0, 0.0, -1), (20.0, 1.3, -2), (7.0, -0.8, 1)])
def test_annulus_field_solves_the_london_maxwell_equation(lam, alpha, n):
    """A(R) of the annulus solves -(A'' + A'/R - A/R^2) = -(A + n Phi0 /
    (2 pi R)) / lam^2 (central differences, step 1e-3); A is continuous at
    R<, where the hole's uniform field takes over; B = (1/R) d(R A)/dR equals
    the applied alpha Phi0 / A at R>, and the flux through the hole plus the
    flux through the annulus equals the line integral 2 pi R> A(R>)."""
    Ro, Ri = _RING
    f = lambda R: annulus.field(R, Ro, Ri, lam, alpha, n)[0]  # noqa: E731
    e = 1e-3
    for R in np.linspace(Ri + 0.5, Ro - 0.5, 9):
        lap = (f(R + e) - 2 * f(R) + f(R - e)) / e ** 2 + (f(R + e) - f(R - e)) / (2 * e * R) - f(R) / R ** 2
        rhs = (f(R) + n * math.pi / (2 * math.pi * R)) / lam ** 2
        assert abs(lap - rhs) < 1e-5 * max(abs(rhs), 1e-3), (R, lap, rhs)
    a_in = annulus.field(Ri - 1e-12, Ro, Ri, lam, alpha, n)[0]
    assert abs(f(Ri) - a_in) < 1e-9 * max(abs(a_in), 1e-3)
    b_out = ((Ro + e) * f(Ro + e) - (Ro - e) * f(Ro - e)) / (2 * e * Ro)
    area = math.pi * (Ro ** 2 - Ri ** 2)
    assert abs(b_out - alpha * math.pi / area) < 1e-6 + 1e-6 * abs(alpha)
    assert abs(annulus.field(Ro, Ro, Ri, lam, alpha, n)[1] - alpha * math.pi / area) < 1e-9
    from scipy.integrate import quad
    flux = annulus.field(1.0, Ro, Ri, lam, alpha, n)[1] * math.pi * Ri ** 2
    flux += quad(lambda R: 2 * math.pi * R * annulus.field(R, Ro, Ri, lam, alpha, n)[1], Ri, Ro, limit=200)[0]
    assert abs(flux - 2 * math.pi * Ro * f(Ro)) < 1e-8 * max(abs(flux), 1.0)


@pytest.mark.parametrize("lam0,Y", [(2.0, 1.0), (5.0, 0.99886), (20.0, 0.83), (100.0, 1.0)])
def test_annulus_moment_equals_the_moment_of_its_current(lam0, Y):
    """d_alpha alpha + d_n n equals (pi / A) int R^2 j(R) dR over the
    annulus, with j the linear-response current of the closed-form field
    (Sec. V.A, Eq. magnetic_moment_def in polar coordinates), for several
    (alpha, n); it is linear in both."""
    from scipy.integrate import quad
    Ro, Ri = _RING
    area = math.pi * (Ro ** 2 - Ri ** 2)
    for alpha, n in ((0.5, 0), (0.0, -1), (1.3, -2), (-0.4, 3)):
        m, da, dn = annulus.moment(Ro, Ri, lam0, Y, alpha, n)
        ref = math.pi / area * quad(lambda R: R * R * annulus.current(R, Ro, Ri, lam0, Y, alpha, n),
                                    Ri, Ro, limit=200)[0]
        assert abs(m - ref) < 1e-9 * max(abs(ref), 1e-6), (alpha, n, m, ref)
        assert abs(m - (da * alpha + dn * n)) < 1e-15 + 1e-12 * abs(m)
    # diamagnetic: a positive field gives a negative moment without winding
    assert annulus.moment(Ro, Ri, lam0, Y, 1.0, 0)[0] < 0


def test_annulus_moment_without_screening():
    """lam0 -> infinity: the field is the applied one, A = B R / 2, and
    m/m0 = -(pi Y / A) (B (R>^4 - R<^4) / 8 + n (R>^2 - R<^2) / 4) with
    B = alpha pi / A; the closed form tends to it as 1/lam0^2."""
    Ro, Ri = _RING
    area = math.pi * (Ro ** 2 - Ri ** 2)
    Y, alpha, n = 0.9, 0.7, -1
    B = alpha * math.pi / area
    ref = -(math.pi * Y / area) * (B * (Ro ** 4 - Ri ** 4) / 8 + n * (Ro ** 2 - Ri ** 2) / 4)
    errs = [abs(annulus.moment(Ro, Ri, lam0, Y, alpha, n)[0] / ref - 1) for lam0 in (300.0, 3000.0)]
    assert errs[1] < 1e-4 and errs[1] < 0.03 * errs[0], errs


# ------------------------------------ unscreened disc (Sec. V.B closed forms)
from oracle import disc as odisc  # noqa: E402


@pytest.mark.parametrize("R,Y", [(25.0, 0.998859), (15.0, 0.83), (8.0, 1.0)])
def test_disc_free_energy_is_the_kinetic_energy_of_its_superflow(R, Y):
    """Eq. lFEkin with rho_s = 2 N_F Y v_F v_F^T and p_s = (hbar / 2) q phi-hat
    gives, averaged over the Fermi circle (<(v.e)^2> = v_F^2 / 2) and with
    hbar v_F = 2 pi k_B T_c xi0, the density Y q^2 / 8 in units of
    N_F (2 pi k_B T_c)^2, q = n / r + alpha r / R^2 in 1/xi0.  Its disc
    average reproduces dw alpha^2 for n = 0 and, for n = -1, the terms of
    Eq. 1vor that depend on alpha (the r^-2 term is the core's)."""
    from scipy.integrate import quad
    area = math.pi * R * R
    for alpha in (0.5, 1.0, 2.7):
        for n in (0, -1):
            dens = lambda r: Y / 8.0 * ((alpha * r / R ** 2) ** 2 + 2 * n * alpha / R ** 2)  # noqa: E731
            avg = quad(lambda r: dens(r) * 2 * math.pi * r, 0.0, R)[0] / area
            ref = odisc.free_energy_shift(R, Y, alpha, n) - odisc.free_energy_shift(R, Y, 0.0, n)
            assert abs(avg - ref) < 1e-12 * abs(ref), (alpha, n, avg, ref)
    assert odisc.kinetic_coefficient(R, Y) == pytest.approx(Y / (16 * R * R), rel=1e-15)


@pytest.mark.parametrize("kappa,alpha,n", [(5.0, 0.3, 0), (5.0, 0.0, -1), (20.0, 1.3, -2), (3.0, -0.6, 1)])
def test_annulus_free_energy_is_stationary_at_the_london_field(kappa, alpha, n):
    """The London field minimises kinetic + magnetic energy (its Euler-Lagrange
    equation is Eq. LMeqRing with 1 / lambda^2 = Y / kappa^2): adding
    eps dA (dA smooth, zero at R> and inside the hole's edge region, so the
    applied flux stays) changes the functional by O(eps^2) only, while the
    same variation of a field off the solution changes it at first order.
    A wrong relative factor between the two terms (kappa^2 against 1/8pi, or
    Y/2) moves the minimiser off the London field and fails this.  The
    functional here is integrated on its own grid; free_energy_shift must
    agree with it at the London field."""
    Ro, Ri, Y = 25.0, 10.0, 0.9
    lam = kappa / math.sqrt(Y)
    area = math.pi * (Ro ** 2 - Ri ** 2)
    b_ext = alpha * math.pi / area
    r = np.linspace(Ri, Ro, 20001)
    dr = r[1] - r[0]
    A0 = np.array([annulus.field(x, Ro, Ri, lam, alpha, n)[0] for x in r])
    bh = annulus.field(0.5 * Ri, Ro, Ri, lam, alpha, n)[1]
    dA = np.sin(np.pi * (r - Ri) / (Ro - Ri)) ** 2  # zero with its slope at both ends

    def functional(Af):
        B = np.gradient(r * Af, dr) / r
        kin = 0.5 * Y * (Af + n / (2 * r)) ** 2
        mag = 0.5 * kappa ** 2 * (B - b_ext) ** 2
        f = (kin + mag) * 2 * np.pi * r
        return np.sum(0.5 * (f[1:] + f[:-1])) * dr + 0.5 * kappa ** 2 * (bh - b_ext) ** 2 * math.pi * Ri ** 2

    eps = 1e-3 * max(np.max(np.abs(A0)), 1e-3)
    f0 = functional(A0)
    tot, kin, mag = annulus.free_energy_shift(Ro, Ri, kappa, Y, alpha, n, kappa)
    assert abs(f0 - tot) < 1e-6 * abs(tot), (f0, tot)
    d1 = (functional(A0 + eps * dA) - functional(A0 - eps * dA)) / (2 * eps)
    d2 = (functional(A0 + eps * dA) - 2 * f0 + functional(A0 - eps * dA)) / eps ** 2
    assert d2 > 0
    assert abs(d1) < 1e-6 * d2 * max(np.max(np.abs(A0)), 1.0), (d1, d2)
    # a field off the solution (the applied one alone) is not stationary
    Aoff = A0 + 0.05 * np.max(np.abs(A0) + 1e-3) * dA
    d1off = (functional(Aoff + eps * dA) - functional(Aoff - eps * dA)) / (2 * eps)
    assert abs(d1off) > 1e-3 * d2 * 0.05 * np.max(np.abs(A0) + 1e-3)
