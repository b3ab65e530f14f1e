"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

FP64: <= 1e-10 normwise relative (and elementwise against the field's max).
Mixed FP32-sweep / FP64-sum: within the bound derived from FP32 rounding
(checked at 2e-5 * DELTA0 absolute on Delta, about 1e-4 relative).
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2205_15000_amd import workloads as wl  # noqa: E402
from oracle import fields, scf as oscf  # noqa: E402
from helpers import oracle_grain, rel_err  # noqa: E402

SMALL = ["s_disc_32", "small_d110_field", "small_holed_mixed", "small_polygon_landau", "small_mask_blob"]
FP64_TOL = 1e-10


def _qs():
    import paper_2205_15000_amd as qs
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return qs


def _dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda()


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _close(a, b, tol):
    a = np.asarray(a)
    b = np.asarray(b)
    scale = max(np.max(np.abs(b)), 1e-300)
    return rel_err(a, b) <= tol and np.max(np.abs(a - b)) <= tol * scale


@pytest.mark.parametrize("name", SMALL)
def test_iteration_map_fp64_matches_oracle(name):
    qs = _qs()
    sp = wl.spec(name)
    _note("case %s fp64: 3 chained sweeps" % name)
    g = qs.Grain(sp, "fp64")
    og = oracle_grain(sp)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    dd, ad = _dev(d0, torch.complex128), _dev(a0, torch.float64)
    bc = None
    for it in range(3):
        dn, j, om, od = g.sweep(dd, ad, omega_density=True)
        ref = og.iterate(d0, a0, bc)
        bc = ref["bc"]
        m = og.mask
        assert _close(dn.cpu().numpy()[:, m], ref["delta_new"][:, m], FP64_TOL), (it, rel_err(dn.cpu().numpy(), ref["delta_new"]))
        assert np.all(dn.cpu().numpy()[:, ~m] == 0)
        if np.max(np.abs(ref["j"])) > 1e-12:
            assert _close(j.cpu().numpy(), ref["j"], FP64_TOL), (it, rel_err(j.cpu().numpy(), ref["j"]))
        else:
            assert np.max(np.abs(j.cpu().numpy())) < 1e-13
        assert _close(od.cpu().numpy(), ref["omega_density"], FP64_TOL)
        assert abs(om - ref["omega_total"]) <= FP64_TOL * abs(ref["omega_total"])
    g.close()


@pytest.mark.parametrize("n_poles,epl", [(8, 1), (8, 2), (8, 4), (8, 8), (64, 1), (64, 2), (64, 4), (48, 3),
                                         (7, 3), (48, 0)])
def test_every_lane_shape_matches_oracle(n_poles, epl):
    """Forced energies per lane cover every lanes-per-segment G of the
    per-node pole-sum reduction: 8 poles give G = 8, 4, 2, 1 and 64 poles
    G = 64, 32, 16; three energies per lane with 48 poles (G = 16, the
    automatic choice) and with 7 (G = 4, two padded energies) (two chained
    sweeps, FP64, against the oracle)."""
    qs = _qs()
    name = "small_d110_field"
    sp = dict(wl.spec(name), n_poles=n_poles)
    _note("case %s fp64, %d poles, %d energies per lane" % (name, n_poles, epl))
    g = qs.Grain(sp, "fp64")
    g.set_lanes(epl)
    e, G = g.lanes()
    want = epl if epl else 3
    assert e == want and G == 1 << max(0, math.ceil(math.log2(math.ceil(n_poles / want))))
    og = oracle_grain(sp)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    dd, ad = _dev(d0, torch.complex128), _dev(a0, torch.float64)
    bc = None
    for it in range(2):
        dn, j, om, od = g.sweep(dd, ad, omega_density=True)
        ref = og.iterate(d0, a0, bc)
        bc = ref["bc"]
        m = og.mask
        assert _close(dn.cpu().numpy()[:, m], ref["delta_new"][:, m], FP64_TOL), (it, G)
        assert _close(j.cpu().numpy(), ref["j"], FP64_TOL), (it, G)
        assert _close(od.cpu().numpy(), ref["omega_density"], FP64_TOL), (it, G)
    g.close()


@pytest.mark.parametrize("name", ["s_disc_32", "small_d110_field", "small_holed_mixed", "small_mask_blob"])
def test_iteration_map_mixed_precision_error(name):
    qs = _qs()
    sp = wl.spec(name)
    _note("case %s mixed: 3 chained sweeps" % name)
    g = qs.Grain(sp, "mixed")
    og = oracle_grain(sp)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    dd, ad = _dev(d0, torch.complex128), _dev(a0, torch.float64)
    bc = None
    for it in range(3):
        dn, j, om = g.sweep(dd, ad)
        ref = og.iterate(d0, a0, bc)
        bc = ref["bc"]
        m = og.mask
        err = np.max(np.abs(dn.cpu().numpy()[:, m] - ref["delta_new"][:, m]))
        assert err < 2e-5 * wl.DELTA0, err
        jerr = np.max(np.abs(j.cpu().numpy() - ref["j"]))
        assert jerr < 2e-5 * max(np.max(np.abs(ref["j"])), 1e-3), jerr
        assert abs(om - ref["omega_total"]) < 1e-5 * abs(ref["omega_total"])
    g.close()


@pytest.mark.parametrize("name", ["small_d110_field", "small_polygon_landau"])
def test_A_solve_matches_oracle(name):
    qs = _qs()
    sp = wl.spec(name)
    _note("case %s: A-solve" % name)
    g = qs.Grain(sp, "fp64")
    og = oracle_grain(sp)
    rng = np.random.default_rng(99)
    jj = rng.standard_normal((2, sp["ny"], sp["nx"]))
    A, B = g.solve_A(_dev(jj, torch.float64))
    ax, ay = fields.solve_A(jj[0], jj[1], og.mask, sp["h"], sp["kappa"], method="direct")
    assert _close(A.cpu().numpy()[0], ax, FP64_TOL)
    assert _close(A.cpu().numpy()[1], ay, FP64_TOL)
    assert _close(B.cpu().numpy(), fields.curl(ax, ay, sp["h"]), FP64_TOL)
    g.close()


def test_scf_50_picard_iterations_match_oracle():
    qs = _qs()
    name = "s_disc_32"
    sp = wl.spec(name)
    _note("case %s: 50 Picard iterations fp64" % name)
    g = qs.Grain(sp, "fp64")
    og = oracle_grain(sp)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    dd, ad = _dev(d0, torch.complex128), _dev(a0, torch.float64)
    it, res, conv = g.scf(dd, ad, 50)
    assert it == 50 and not conv
    dref, aref, hist, _ = oscf.scf(og, d0, a0, 50)
    m = og.mask
    assert _close(dd.cpu().numpy()[:, m], dref[:, m], FP64_TOL)
    h = np.array(hist)
    for c in (0, 3, 4):
        fin = np.isfinite(h[:, c])
        assert np.all(np.isfinite(res[:, c]) == fin)
        assert np.max(np.abs(res[fin, c] - h[fin, c]) / np.maximum(np.abs(h[fin, c]), 1e-300)) < 1e-8
    g.close()


def test_scf_with_A_solve_matches_oracle():
    qs = _qs()
    name = "small_d110_field"
    sp = wl.spec(name)
    _note("case %s: 6 Picard iterations with A, fp64" % name)
    g = qs.Grain(sp, "fp64")
    og = oracle_grain(sp)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    dd, ad = _dev(d0, torch.complex128), _dev(a0, torch.float64)
    it, res, conv = g.scf(dd, ad, 6, alpha=0.7, burnin=1)
    dref, aref, hist, _ = oscf.scf(og, d0, a0, 6, alpha=0.7, burnin=1)
    m = og.mask
    assert _close(dd.cpu().numpy()[:, m], dref[:, m], FP64_TOL)
    assert _close(ad.cpu().numpy(), aref, FP64_TOL)
    h = np.array(hist)
    fin = np.isfinite(h)
    assert np.max(np.abs(res[fin] - h[fin]) / np.maximum(np.abs(h[fin]), 1e-12)) < 1e-8
    g.close()


def test_scf_polyak_matches_oracle():
    """Polyak's heavy ball (App. E) with the A-solve: 8 iterations after a
    burn-in, then the same grain run again (the velocity restarts at zero)
    and switched back to Picard."""
    qs = _qs()
    name = "small_d110_field"
    sp = wl.spec(name)
    _note("case %s: 8 Polyak iterations with A, fp64" % name)
    g = qs.Grain(sp, "fp64")
    g.set_accelerator("polyak", beta=0.4)
    og = oracle_grain(sp)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    m = og.mask
    for rerun in range(2):
        g.reset_bc()
        dd, ad = _dev(d0, torch.complex128), _dev(a0, torch.float64)
        it, res, conv = g.scf(dd, ad, 8, alpha=1.5, burnin=1)
        dref, aref, hist, _ = oscf.scf(og, d0, a0, 8, alpha=1.5, burnin=1, accelerator="polyak", beta=0.4)
        assert _close(dd.cpu().numpy()[:, m], dref[:, m], FP64_TOL)
        assert _close(ad.cpu().numpy(), aref, FP64_TOL)
        h = np.array(hist)
        fin = np.isfinite(h)
        assert np.max(np.abs(res[fin] - h[fin]) / np.maximum(np.abs(h[fin]), 1e-12)) < 1e-8
    # and back to Picard
    g.set_accelerator("picard")
    g.reset_bc()
    dd, ad = _dev(d0, torch.complex128), _dev(a0, torch.float64)
    g.scf(dd, ad, 3, alpha=0.7)
    dref, aref, _, _ = oscf.scf(og, d0, a0, 3, alpha=0.7)
    assert _close(dd.cpu().numpy()[:, m], dref[:, m], FP64_TOL)
    with pytest.raises(qs.QcError):
        g.set_accelerator("polyak", beta=1.5)
    g.close()


def test_scf_barzilai_borwein_matches_oracle():
    """Barzilai-Borwein steps (App. E) with the A-solve and kappa^2 in the
    dot products: 10 iterations after a burn-in, FP64, against the oracle;
    run twice on the same grain (the step restarts at alpha)."""
    qs = _qs()
    name = "small_d110_field"
    sp = wl.spec(name)
    _note("case %s: 10 BB iterations with A, fp64" % name)
    g = qs.Grain(sp, "fp64")
    g.set_accelerator("bb")
    og = oracle_grain(sp)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    m = og.mask
    for rerun in range(2):
        g.reset_bc()
        dd, ad = _dev(d0, torch.complex128), _dev(a0, torch.float64)
        it, res, conv = g.scf(dd, ad, 10, alpha=0.8, burnin=1)
        dref, aref, hist, _ = oscf.scf(og, d0, a0, 10, alpha=0.8, burnin=1, accelerator="bb")
        assert _close(dd.cpu().numpy()[:, m], dref[:, m], FP64_TOL)
        assert _close(ad.cpu().numpy(), aref, FP64_TOL)
        h = np.array(hist)
        fin = np.isfinite(h)
        assert np.max(np.abs(res[fin] - h[fin]) / np.maximum(np.abs(h[fin]), 1e-12)) < 1e-8
    g.close()


def test_scf_congacc_matches_oracle():
    """CongAcc (App. E) per component, with the A-solve, FP64, against the
    oracle: 10 iterations after a burn-in on a one-component grain with a
    field, 12 on a two-component grain without screening (A held at zero)
    with a first step large enough that the similarity of every Delta
    component falls below the minimum at least once, so the weights of the
    second component are set by bisection too.  The number of bisected
    weights equals the oracle's."""
    qs = _qs()
    for name, n_it, alpha in (("small_d110_field", 10, 0.5), ("small_holed_mixed", 12, 1.0)):
        sp = wl.spec(name)
        _note("case %s: %d CongAcc iterations, alpha %g, fp64" % (name, n_it, alpha))
        g = qs.Grain(sp, "fp64")
        g.set_accelerator("congacc")
        og = oracle_grain(sp)
        d0 = wl.initial_delta(name, sp)
        a0 = wl.initial_A(name, sp)
        m = og.mask
        dd, ad = _dev(d0, torch.complex128), _dev(a0, torch.float64)
        it, res, conv = g.scf(dd, ad, n_it, alpha=alpha, burnin=1)
        st = {}
        dref, aref, hist, _ = oscf.scf(og, d0, a0, n_it, alpha=alpha, burnin=1, accelerator="congacc", stats=st)
        assert _close(dd.cpu().numpy()[:, m], dref[:, m], FP64_TOL)
        assert _close(ad.cpu().numpy(), aref, FP64_TOL)
        h = np.array(hist)
        fin = np.isfinite(h)
        assert np.max(np.abs(res[fin] - h[fin]) / np.maximum(np.abs(h[fin]), 1e-12)) < 1e-8
        bis, anti = g.accel_stats()
        assert st.get("bisect", 0) >= 1 and bis == st.get("bisect", 0) and anti == st.get("anti", 0)
        if g.ncomp == 2:
            assert {2, 3} <= st["bisect_components"]
        with pytest.raises(qs.QcError):
            g.scf(dd, ad, 2, norm_p=1)
        g.close()


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", 2e-4)])
def test_ldos_matches_oracle(precision, tol):
    qs = _qs()
    name = "small_d110_field"
    sp = wl.spec(name)
    _note("case %s: LDOS %s" % (name, precision))
    g = qs.Grain(sp, precision)
    og = oracle_grain(sp)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    en = np.linspace(-0.4, 0.4, 7)
    out = g.ldos(_dev(d0, torch.complex128), _dev(a0, torch.float64), en, 0.02, 2)
    ref = og.ldos(d0, a0, en, 0.02, 2)
    assert _close(out.cpu().numpy(), ref, tol), rel_err(out.cpu().numpy(), ref)
    g.close()


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("mixed", 2e-4)])
def test_ldos_far_from_the_gap_matches_oracle(precision, tol):
    """LDOS at energies far outside the gap (up to about 20 times the gap)
    with a small broadening: there h Re(z)/2 exceeds (1 + h Im z)/2, so the
    discriminant of the implicit-midpoint step (App. C) has a negative real
    part and its root is taken on the other branch; the step's stable root
    must still be the oracle's."""
    qs = _qs()
    name = "small_d110_field"
    sp = wl.spec(name)
    _note("case %s: LDOS far from the gap %s" % (name, precision))
    g = qs.Grain(sp, precision)
    og = oracle_grain(sp)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    en = np.array([-6.0, -3.0, -1.2, 0.1, 1.2, 3.0, 6.0])
    out = g.ldos(_dev(d0, torch.complex128), _dev(a0, torch.float64), en, 0.005, 2)
    ref = og.ldos(d0, a0, en, 0.005, 2)
    assert np.all(np.isfinite(out.cpu().numpy()))
    assert _close(out.cpu().numpy(), ref, tol), rel_err(out.cpu().numpy(), ref)
    g.close()


@pytest.mark.parametrize("name,precision", [("small_d110_field", "fp64"), ("s_disc_32", "fp64"),
                                            ("small_d110_field", "mixed")])
def test_ldos_angle_pairs_equal_every_angle(name, precision):
    """LDOS with an energy set symmetric about zero (e and -e, zero included)
    and 5 boundary iterations: with angle pairs the boundary and output
    sweeps march the lower angle of each pair (the upper one's store filled
    from its mirror at -e; its LDOS share read at -e through the lower
    angle's corners).  The LDOS equals that of the run without pairs (1e-12
    FP64, 1e-6 mixed), for one output block (9 energies), for several
    (131 energies in the caller's shuffled order: blocks of 64 holding
    whole pairs, zero last), and for an asymmetric set, which runs
    unpaired."""
    qs = _qs()
    sp = wl.spec(name)
    _note("case %s %s: LDOS with and without angle pairs" % (name, precision))
    d0 = _dev(wl.initial_delta(name, sp), torch.complex128)
    a0 = _dev(wl.initial_A(name, sp), torch.float64)
    tol = 1e-12 if precision == "fp64" else 1e-6
    shuffled = np.random.default_rng(4).permutation(np.linspace(-0.5, 0.5, 131))
    for en in (np.linspace(-0.45, 0.45, 9), shuffled, np.array([-0.3, 0.05, 0.2, 0.31])):
        out = []
        for pair in (True, False):
            g = qs.Grain(sp, precision)
            g.set_pairing(pair)
            out.append(g.ldos(d0, a0, en, 0.02, 5).cpu().numpy())
            g.close()
        assert _close(out[0], out[1], tol), rel_err(out[0], out[1])


def test_uniform_s_wave_is_an_exact_fixed_point_on_gpu():
    qs = _qs()
    from oracle import bulk
    sp = wl.spec("s_disc_32")
    _note("case s_disc_32: bulk fixed point")
    g = qs.Grain(sp, "fp64")
    db = bulk.bulk_gap(0.5, 16)
    d = torch.full((1, 32, 32), db, dtype=torch.complex128, device="cuda")
    A = torch.zeros((2, 32, 32), dtype=torch.float64, device="cuda")
    for _ in range(2):
        dn, j, om = g.sweep(d, A)
    m = oracle_grain(sp).mask
    assert np.max(np.abs(dn.cpu().numpy()[0][m] - db)) < 1e-13
    assert np.max(np.abs(j.cpu().numpy())) < 1e-15
    assert abs(om / (0.625 ** 2 * m.sum()) - bulk.bulk_free_energy(db, 0.5, 16)) < 1e-13
    g.close()


def test_state_roundtrip_and_reset():
    qs = _qs()
    name = "small_holed_mixed"
    sp = wl.spec(name)
    _note("case %s: boundary-store get/set" % name)
    g = qs.Grain(sp, "fp64")
    d0 = _dev(wl.initial_delta(name, sp), torch.complex128)
    a0 = _dev(wl.initial_A(name, sp), torch.float64)
    g.sweep(d0, a0)
    st = g.get_state()
    r1 = g.sweep(d0, a0)[0].cpu().numpy()
    g.set_state(st)
    r2 = g.sweep(d0, a0)[0].cpu().numpy()
    assert np.array_equal(r1, r2)
    g.reset_bc()
    r3 = g.sweep(d0, a0)[0].cpu().numpy()
    g.reset_bc()
    r4 = g.sweep(d0, a0)[0].cpu().numpy()
    assert np.array_equal(r3, r4) and not np.array_equal(r3, r1)
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_d110_square_400_sampled_cells(precision):
    """The 400x400 [110] square with a vortex, field and kappa = 20 in the
    launch configuration of the benchmark: the first iteration map from
    bulk start values checked at sampled grain cells against the oracle,
    which sweeps only the trajectories feeding those cells."""
    qs = _qs()
    name = "d110_square_400"
    sp = wl.spec(name)
    _note("case %s %s: full-size first sweep" % (name, precision))
    g = qs.Grain(sp, precision)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    dn, j, om = g.sweep(_dev(d0, torch.complex128), _dev(a0, torch.float64))
    og = oracle_grain(sp)
    rng = np.random.default_rng(31)
    cells = np.sort(rng.choice(np.nonzero(og.mask.ravel())[0], 6, replace=False))
    cells = np.concatenate([cells, [0, 399, 400 * 200 + 200]])  # two corners and the centre
    _note("  oracle on cells %s" % cells.tolist())
    dref, jref = og.iterate_cells(d0, a0, cells)
    dg = dn.cpu().numpy().reshape(1, -1)[:, cells]
    jg = j.cpu().numpy().reshape(2, -1)[:, cells]
    if precision == "fp64":
        assert np.max(np.abs(dg - dref)) <= FP64_TOL * np.max(np.abs(dref))
        assert np.max(np.abs(jg - jref)) <= FP64_TOL * np.max(np.abs(jref))
    else:
        assert np.max(np.abs(dg - dref)) < 2e-5 * wl.DELTA0
        assert np.max(np.abs(jg - jref)) < 2e-5 * max(np.max(np.abs(jref)), 1e-3)
    assert math.isfinite(om)
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_d110_square_400_three_maps_match_oracle(precision):
    """The 400x400 [110] square with a vortex, field and kappa = 20 in the
    benchmark's launch configuration: three iteration maps chained as
    Picard with step 1 and the A-solve between them, so the second and third
    maps start from the specular boundary taps of the previous one, against
    the oracle's values stored by tests/golden/make_d110_square_400.py at
    every cell of the four [110] edges (corners included) and 200 interior
    cells: Delta_new, j and Omega_total of each map.  FP64 within 1e-10
    (normwise and elementwise against the largest value); the mixed path
    within 2e-5 Delta0 on Delta and 1e-4 of the largest |j| on j."""
    import os
    qs = _qs()
    name = "d110_square_400"
    sp = wl.spec(name)
    gold = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name + "_iter3.npz"))
    cells = gold["cells"]
    _note("case %s %s: three chained maps vs the oracle at %d cells" % (name, precision, len(cells)))
    g = qs.Grain(sp, precision)
    d = _dev(wl.initial_delta(name, sp), torch.complex128)
    a = _dev(wl.initial_A(name, sp), torch.float64)
    for i in range(len(gold["omega_total"])):
        dn, j, om = g.sweep(d, a)
        dg = dn.cpu().numpy().reshape(1, -1)[:, cells]
        jg = j.cpu().numpy().reshape(2, -1)[:, cells]
        dref, jref, oref = gold["delta_new"][i], gold["j"][i], gold["omega_total"][i]
        if precision == "fp64":
            assert _close(dg, dref, FP64_TOL), (i, rel_err(dg, dref))
            assert _close(jg, jref, FP64_TOL), (i, rel_err(jg, jref))
            assert abs(om - oref) <= FP64_TOL * abs(oref), (i, om, oref)
        else:
            assert np.max(np.abs(dg - dref)) <= 2e-5 * wl.DELTA0, (i, np.max(np.abs(dg - dref)) / wl.DELTA0)
            assert np.max(np.abs(jg - jref)) <= 1e-4 * np.max(np.abs(jref)), (i, np.max(np.abs(jg - jref)))
            assert abs(om - oref) <= 1e-5 * abs(oref), (i, om, oref)
        a, _ = g.solve_A(j, B=False)
        d = dn
    g.close()


@pytest.mark.parametrize("name,precision", [("small_d110_field", "fp64"), ("small_mask_blob", "fp64"),
                                            ("small_holed_mixed", "fp64"), ("small_d110_field", "mixed")])
def test_green_average_matches_oracle(name, precision):
    """<g>(R, i eps~_p) per pole: from bulk starts, then with the boundary
    store of one sweep; the call must leave the store unchanged."""
    qs = _qs()
    sp = wl.spec(name)
    _note("case %s %s: green average" % (name, precision))
    g = qs.Grain(sp, precision)
    og = oracle_grain(sp)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    dd, ad = _dev(d0, torch.complex128), _dev(a0, torch.float64)
    tol = FP64_TOL if precision == "fp64" else 2e-5
    m = og.mask
    got = g.green_average(dd, ad).cpu().numpy()
    ref = og.green_average(d0, a0, None)
    assert got.shape == ref.shape
    assert _close(got[:, m], ref[:, m], tol), rel_err(got[:, m], ref[:, m])
    assert np.all(got[:, ~m] == 0)
    g.sweep(dd, ad)
    bc = og.iterate(d0, a0, None)["bc"]
    st0 = g.get_state().cpu().numpy().copy()
    got = g.green_average(dd, ad).cpu().numpy()
    ref = og.green_average(d0, a0, bc)
    assert _close(got[:, m], ref[:, m], tol), rel_err(got[:, m], ref[:, m])
    assert np.array_equal(g.get_state().cpu().numpy(), st0)
    g.close()


def _degenerate(case):
    base = wl.spec("small_d110_field")
    if case == "tiny_disc":
        return dict(base, nx=10, ny=10, h=0.5, n_theta=8, n_poles=4,
                    shapes=[{"kind": "disc", "cx": 0.1, "cy": -0.05, "radius": 0.9, "add": True}])
    if case == "square_fills_array":
        return dict(base, nx=24, ny=24, h=0.5,
                    shapes=[{"kind": "regular_polygon", "cx": 0.0, "cy": 0.0, "n_edges": 4, "side": 12.0,
                             "rotation": 0.0, "add": True}])
    if case == "thin_sliver":
        c, s = math.cos(0.3), math.sin(0.3)
        pts = [(-6.0, -0.15), (6.0, -0.15), (6.0, 0.15), (-6.0, 0.15)]
        return dict(base, shapes=[{"kind": "polygon", "vx": [c * x - s * y for x, y in pts],
                                   "vy": [s * x + c * y for x, y in pts], "add": True}])
    if case in ("normal_state", "single_pole"):
        return dict(base, n_poles=1) if case == "single_pole" else dict(base)
    raise ValueError(case)


@pytest.mark.parametrize("case", ["tiny_disc", "square_fills_array", "thin_sliver", "normal_state", "single_pole"])
def test_degenerate_inputs_match_oracle(case):
    """A disc of a few cells, a sliver a fraction of a cell wide (segments
    without interior nodes), a grain reaching the array edge on all sides,
    Delta = 0 (normal state: no current, no condensation energy) and a
    single pole (one lane per segment): two chained FP64 sweeps against
    the oracle."""
    qs = _qs()
    sp = _degenerate(case)
    sp["name"] = case
    _note("degenerate case %s" % case)
    og = oracle_grain(sp)
    m = og.mask
    assert m.sum() > 0
    d0 = wl.initial_delta(case, sp)
    if case == "normal_state":
        d0 = np.zeros_like(d0)
    a0 = wl.initial_A(case, sp)
    g = qs.Grain(sp, "fp64")
    dd, ad = _dev(d0, torch.complex128), _dev(a0, torch.float64)
    bc = None
    for it in range(2):
        dn, j, om, od = g.sweep(dd, ad, omega_density=True)
        ref = og.iterate(d0, a0, bc)
        bc = ref["bc"]
        if case == "normal_state":
            assert np.max(np.abs(dn.cpu().numpy())) == 0.0
        else:
            assert _close(dn.cpu().numpy()[:, m], ref["delta_new"][:, m], FP64_TOL), (case, it)
        assert _close(j.cpu().numpy(), ref["j"], FP64_TOL), (case, it)
        assert _close(od.cpu().numpy(), ref["omega_density"], FP64_TOL), (case, it)
        assert abs(om - ref["omega_total"]) <= FP64_TOL * abs(ref["omega_total"])
    g.close()



@pytest.mark.parametrize("name,precision", [("small_d110_field", "fp64"), ("small_holed_mixed", "fp64"),
                                            ("small_polygon_landau", "fp64"), ("small_d110_field", "mixed")])
def test_luttinger_ward_free_energy_matches_oracle(name, precision):
    """The Luttinger-Ward free energy (Sec. II, Eqs. qcLWFE and qcLWFE_I):
    4 Gauss-Legendre couplings with 2 burn-in sweeps each, density and total
    against the oracle (FP64 1e-10; mixed 1e-4 of the largest density).  The
    call leaves the grain's boundary store as it found it."""
    qs = _qs()
    sp = wl.spec(name)
    _note("case %s %s: Luttinger-Ward free energy" % (name, precision))
    g = qs.Grain(sp, precision)
    og = oracle_grain(sp)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    dd, ad = _dev(d0, torch.complex128), _dev(a0, torch.float64)
    g.sweep(dd, ad)
    st = g.get_state().clone()
    tot, dens = g.free_energy_lw(dd, ad, 4, 2, density=True)
    ref_d, ref_t = og.free_energy_lw(d0, a0, 4, 2)
    got = dens.cpu().numpy()
    if precision == "fp64":
        assert _close(got, ref_d, FP64_TOL), rel_err(got, ref_d)
        assert abs(tot - ref_t) <= FP64_TOL * abs(ref_t)
    else:
        assert np.max(np.abs(got - ref_d)) <= 1e-4 * np.max(np.abs(ref_d))
        assert abs(tot - ref_t) <= 1e-4 * abs(ref_t)
    assert torch.equal(g.get_state(), st)
    with pytest.raises(qs.QcError):
        g.free_energy_lw(dd, ad, 0, 2)
    g.close()


@pytest.mark.parametrize("name,precision", [("s_disc_32", "fp64"), ("small_d110_field", "fp64"),
                                            ("small_holed_mixed", "fp64"), ("small_d110_field", "mixed")])
def test_angle_pairs_equal_the_full_sweep(name, precision):
    """Paired sweeps (one march per pair of opposite directions) against
    sweeps of every angle: three chained maps (so the second and third read
    boundary values the pairs filled in) give the same Delta_new, j and
    Omega to rounding (1e-12 FP64, 1e-5 mixed), and the stores agree."""
    qs = _qs()
    sp = wl.spec(name)
    _note("case %s %s: angle pairs vs every angle" % (name, precision))
    d0 = _dev(wl.initial_delta(name, sp), torch.complex128)
    a0 = _dev(wl.initial_A(name, sp), torch.float64)
    out = []
    for pair in (True, False):
        g = qs.Grain(sp, precision)
        avail, on, _ = g.pairing()
        assert avail and on
        g.set_pairing(pair)
        _, on, swept = g.pairing()
        assert on == pair
        d, a = d0.clone(), a0.clone()
        res = []
        for _ in range(3):
            dn, j, om = g.sweep(d, a)
            res.append((dn.cpu().numpy(), j.cpu().numpy(), om))
            d = dn
        res.append(g.get_state().cpu().numpy())
        out.append((res, swept))
        g.close()
    (p, swept), (f, full) = out
    assert 2 * swept == full
    tol = 1e-12 if precision == "fp64" else 1e-5
    for i in range(3):
        assert _close(p[i][0], f[i][0], tol), (i, rel_err(p[i][0], f[i][0]))
        assert _close(p[i][1], f[i][1], tol), (i, rel_err(p[i][1], f[i][1]))
        assert abs(p[i][2] - f[i][2]) <= tol * abs(f[i][2])
    if precision == "fp64":
        sp_ = p[3].view(np.float64)
        sf_ = f[3].view(np.float64)
        assert np.max(np.abs(sp_ - sf_)) <= 1e-12 * np.max(np.abs(sf_))


@pytest.mark.parametrize("name,precision,epl", [("s_disc_32", "fp64", 0), ("small_d110_field", "fp64", 0),
                                                ("small_polygon_landau", "fp64", 2), ("small_d110_field", "mixed", 0),
                                                ("d110_square_400", "fp64", 0), ("d110_square_400", "mixed", 0)])
def test_split_launch_shape_equals_one_shape(name, precision, epl):
    """The SCF sweep with its longest segments on twice the lanes (half the
    energies per lane) against the same sweep in one lane shape: three
    chained maps give the same Delta_new, j and Omega up to the order of the
    pole sums (1e-13 FP64; mixed 1e-6, where the FP32 terms may round
    differently in the two instantiations), and the split is in use.  The
    5-pole polygon at 2 energies per lane pads 3 lanes of its wide shape;
    at its automatic 3 per lane the split does not apply."""
    qs = _qs()
    sp = wl.spec(name)
    _note("case %s %s: split launch shape vs one shape" % (name, precision))
    d0 = _dev(wl.initial_delta(name, sp), torch.complex128)
    a0 = _dev(wl.initial_A(name, sp), torch.float64)
    if name == "small_polygon_landau":
        g = qs.Grain(sp, precision)
        assert g.lanes()[0] % 2 == 1 and g.split()[1] == 0
        g.close()
    out = []
    for frac in (0.8, 0.0):
        g = qs.Grain(sp, precision)
        g.set_lanes(epl)
        for bad in (-0.1, 1.5, float("nan")):
            with pytest.raises(qs.QcError):
                g.set_split(bad)
        g.set_split(frac)
        f, n_wide = g.split()
        assert f == frac
        if frac > 0:
            assert n_wide > 0, n_wide
        else:
            assert n_wide == 0
        d, a = d0.clone(), a0.clone()
        res = []
        for _ in range(3):
            dn, j, om = g.sweep(d, a)
            res.append((dn.cpu().numpy(), j.cpu().numpy(), om))
            d = dn
        out.append(res)
        g.close()
    p, f = out
    tol = 1e-13 if precision == "fp64" else 1e-6
    for i in range(3):
        assert _close(p[i][0], f[i][0], tol), (i, rel_err(p[i][0], f[i][0]))
        assert _close(p[i][1], f[i][1], tol), (i, rel_err(p[i][1], f[i][1]))
        assert abs(p[i][2] - f[i][2]) <= tol * abs(f[i][2])


@pytest.mark.parametrize("name", ["small_polygon_landau", "small_mask_blob"])
def test_angle_pairs_unavailable_where_the_tables_do_not_mirror(name):
    """An odd angle count, and a cell-mask boundary whose corners give
    direction-dependent wall tangents: every angle is swept."""
    qs = _qs()
    sp = wl.spec(name)
    g = qs.Grain(sp, "fp64")
    assert g.pairing()[:2] == (False, False)
    with pytest.raises(qs.QcError):
        g.set_pairing(True)
    g.close()


@pytest.mark.parametrize("name,eps", [("small_d110_field", 1e-6), ("small_d110_field", 1e-3),
                                      ("small_d110_field", 1e-300)])
def test_eigen_truncated_A_solve_matches_oracle(name, eps):
    """The separable, eigen-truncated A-solve (App. D) on a square grid: the
    modes kept and A against the oracle's (numpy eigh) at 1e-10 of the
    largest |A|, for the default tolerance, a coarse one and every mode;
    eps = 0 restores the FFT solve."""
    qs = _qs()
    sp = wl.spec(name)
    _note("case %s: eigen-truncated A-solve, eps %g" % (name, eps))
    g = qs.Grain(sp, "fp64")
    og = oracle_grain(sp)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    _, j, _ = g.sweep(_dev(d0, torch.complex128), _dev(a0, torch.float64))
    jj = j.cpu().numpy()
    g.set_A_solver(eps)
    A, B = g.solve_A(j)
    ax, ay, nstar = fields.solve_A_eigen(jj[0], jj[1], og.mask, sp["h"], sp["kappa"], eps)
    assert g.A_solver() == (eps, nstar)
    ref = np.stack([ax, ay])
    got = A.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref)), np.max(np.abs(got - ref))
    b = fields.curl(ax, ay, sp["h"])
    assert np.max(np.abs(B.cpu().numpy() - b)) <= 1e-10 * np.max(np.abs(b))
    g.set_A_solver(0.0)
    assert g.A_solver() == (0.0, 0)
    A2, _ = g.solve_A(j)
    ex, ey = fields.solve_A(jj[0], jj[1], og.mask, sp["h"], sp["kappa"], method="direct")
    assert _close(A2.cpu().numpy(), np.stack([ex, ey]), FP64_TOL)
    g.close()


def test_eigen_A_solve_full_size_and_magnetic_moment():
    """The 400x400 [110] square: the eigen-truncated A-solve at the paper's
    default tolerance (1e-6) against the oracle's (1e-10) and within the
    truncation bound of the exact solve; the magnetic moment of the current
    (Sec. V.A) against the oracle's sum (1e-12)."""
    qs = _qs()
    name = "d110_square_400"
    sp = wl.spec(name)
    _note("case %s: eigen-truncated A-solve and magnetic moment" % name)
    g = qs.Grain(sp, "fp64")
    og_mask = qs.Plan(dict(sp, n_theta=4)).mask()
    _, j, _ = g.sweep(_dev(wl.initial_delta(name, sp), torch.complex128), _dev(wl.initial_A(name, sp), torch.float64))
    jj = j.cpu().numpy()
    exact, _ = g.solve_A(j, B=False)
    g.set_A_solver(1e-6)
    A, _ = g.solve_A(j, B=False)
    ax, ay, nstar = fields.solve_A_eigen(jj[0], jj[1], og_mask, sp["h"], sp["kappa"], 1e-6)
    assert g.A_solver()[1] == nstar
    ref = np.stack([ax, ay])
    assert np.max(np.abs(A.cpu().numpy() - ref)) <= 1e-10 * np.max(np.abs(ref))
    lam, V = fields.green_eigen(sp["nx"], sp["h"], 1e-6)
    G = fields.green_matrix(sp["nx"], sp["h"])
    dK = np.linalg.norm(G - (V * lam) @ V.T)
    for c in range(2):
        jp = np.where(og_mask, jj[c] - jj[c][og_mask].mean(), 0.0)
        bound = 2.0 / sp["kappa"] ** 2 * dK * np.linalg.norm(jp)
        assert np.max(np.abs(A.cpu().numpy()[c] - exact.cpu().numpy()[c])) <= bound
    X, Y = wl.centres(sp)
    m = g.magnetic_moment(j)
    mref = fields.magnetic_moment(jj[0], jj[1], og_mask, X, Y, 0.0, 0.0)
    assert abs(m - mref) <= 1e-12 * max(abs(mref), 1e-300) + 1e-15
    g.close()


def test_ldos_converge_matches_oracle():
    """The LDOS post-process run to convergence (Sec. IV, App. B): the
    boundary iteration stops once the LDOS changes by less than tol; with
    one energy block the result is qc_ldos with bc_iters = sweeps - 1, and
    matches the oracle's LDOS with that burn-in (FP64 1e-10)."""
    qs = _qs()
    name = "small_d110_field"
    sp = wl.spec(name)
    _note("case %s: LDOS to convergence" % name)
    g = qs.Grain(sp, "fp64")
    og = oracle_grain(sp)
    d0 = wl.initial_delta(name, sp)
    a0 = wl.initial_A(name, sp)
    dd, ad = _dev(d0, torch.complex128), _dev(a0, torch.float64)
    en = np.linspace(-0.3, 0.3, 5)
    out, iters = g.ldos_converge(dd, ad, en, 0.02, 1e-6, 60, energies_per_block=len(en))
    assert 2 <= iters < 60
    same = g.ldos(dd, ad, en, 0.02, iters - 1).cpu().numpy()
    got = out.cpu().numpy()
    assert np.max(np.abs(got - same)) <= 1e-12 * np.max(np.abs(same))
    ref = og.ldos(d0, a0, en, 0.02, iters - 1)
    assert _close(got, ref, FP64_TOL), rel_err(got, ref)
    # blocks of two energies converge on their own, each within the tolerance
    out2, it2 = g.ldos_converge(dd, ad, en, 0.02, 1e-6, 60, energies_per_block=2)
    assert it2 <= iters + 1
    assert np.max(np.abs(out2.cpu().numpy() - got)) <= 1e-4 * np.max(np.abs(got))
    g.close()


def test_resume_from_saved_state_and_burn_in():
    """Save and resume (App. B): Delta, A and the boundary store saved after
    8 Picard iterations and loaded into a fresh grain continue exactly as the
    uninterrupted run (FP64, bitwise).  Loading only Delta and A, burn-in
    iterations update the boundary store with the fields held fixed (the
    residuals read 0), and bring the next map closer to the resumed one
    than a restart from bulk start values."""
    qs = _qs()
    name = "small_d110_field"
    sp = wl.spec(name)
    _note("case %s: save, resume, burn-in" % name)
    d0 = _dev(wl.initial_delta(name, sp), torch.complex128)
    a0 = _dev(wl.initial_A(name, sp), torch.float64)
    g1 = qs.Grain(sp, "fp64")
    d, a = d0.clone(), a0.clone()
    g1.scf(d, a, 8, alpha=0.7)
    d8, a8, st = d.clone(), a.clone(), g1.get_state().clone()
    g1.scf(d, a, 4, alpha=0.7)
    g2 = qs.Grain(sp, "fp64")
    g2.set_state(st)
    dr, ar = d8.clone(), a8.clone()
    g2.scf(dr, ar, 4, alpha=0.7)
    assert torch.equal(dr, d) and torch.equal(ar, a)
    # fields only: restart from bulk starts, with and without burn-in
    g3 = qs.Grain(sp, "fp64")
    db, ab = d8.clone(), a8.clone()
    it, res, _ = g3.scf(db, ab, 6, burnin=6, alpha=0.7)
    assert torch.equal(db, d8) and torch.equal(ab, a8)
    assert np.all(res[:, :4] == 0.0)
    g4 = qs.Grain(sp, "fp64")
    g4.set_state(st)
    dn_resumed = g4.sweep(d8, a8)[0]
    dn_burnt = g3.sweep(d8, a8)[0]
    g5 = qs.Grain(sp, "fp64")
    dn_cold = g5.sweep(d8, a8)[0]
    e_burnt = float((dn_burnt - dn_resumed).abs().max())
    e_cold = float((dn_cold - dn_resumed).abs().max())
    assert e_burnt < e_cold, (e_burnt, e_cold)
    for g in (g1, g2, g3, g4, g5):
        g.close()
