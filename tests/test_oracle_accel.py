"""Pins of the oracle's Polyak accelerator (App. E) against what the
mathematics fixes: a closed form on a linear map, and the reduction to
Picard at full drag."""
import numpy as np
import pytest

from oracle import scf
from tests.test_oracle_sweep import _cfg1_like


@pytest.mark.parametrize("lam,alpha,beta", [(0.9, 2.0, 0.5), (0.5, 1.0, 0.3), (-0.4, 0.7, 0.8), (0.95, 3.0, 0.2)])
def test_heavy_ball_on_a_linear_map_follows_its_recurrence_closed_form(lam, alpha, beta):
    # g(x) = lam x + b has the fixed point x* = b / (1 - lam); with v_0 = 0
    # the error e_i = x_i - x* obeys e_1 = (1 + alpha (lam - 1)) e_0 and
    # e_{i+1} = (2 - beta + alpha (lam - 1)) e_i - (1 - beta) e_{i-1},
    # solved by c1 r1^i + c2 r2^i with r1, r2 the roots of its
    # characteristic polynomial (complex when the iteration oscillates)
    b = 0.3
    xs = b / (1.0 - lam)
    x0 = np.array([1.7, -0.2])
    e0 = x0 - xs
    e1 = (1.0 + alpha * (lam - 1.0)) * e0
    r1, r2 = np.roots([1.0, -(2.0 - beta + alpha * (lam - 1.0)), 1.0 - beta]).astype(complex)
    c2 = (e1 - r1 * e0) / (r2 - r1)
    c1 = e0 - c2
    x, v = x0.copy(), np.zeros_like(x0)
    for i in range(1, 41):
        x, v = scf.polyak_step(x, v, lam * x + b, alpha, beta)
        want = (c1 * r1 ** i + c2 * r2 ** i).real + xs
        assert np.allclose(x, want, rtol=1e-11, atol=1e-12 * max(1.0, abs(xs)))


def test_polyak_at_full_drag_is_picard():
    gr = _cfg1_like()
    rng = np.random.default_rng(3)
    d0 = 0.28 * (1.0 + rng.uniform(-0.05, 0.05, (32, 32)))
    delta = np.where(gr.mask, d0, 0)[None].astype(complex)
    A0 = np.zeros((2, 32, 32))
    dp, ap, hp, _ = scf.scf(gr, delta, A0, 3, alpha=1.3)
    dk, ak, hk, _ = scf.scf(gr, delta, A0, 3, alpha=1.3, accelerator="polyak", beta=1.0)
    assert np.array_equal(dp, dk) and np.array_equal(ap, ak)
    assert hp == hk


def test_polyak_keeps_the_bcs_fixed_point():
    # the uniform BCS gap is a fixed point of the map; with d = 0 the
    # velocity stays zero and the state stays put
    from oracle import bulk
    gr = _cfg1_like()
    dbulk = bulk.bulk_gap(0.5, 16)
    delta = np.where(gr.mask, dbulk, 0)[None].astype(complex)
    # one plain iteration first, so the boundary store is the bulk one
    d1, a1, _, _ = scf.scf(gr, delta, np.zeros((2, 32, 32)), 3, accelerator="polyak", alpha=2.0, beta=0.5)
    assert np.max(np.abs(d1[0][gr.mask] - dbulk)) < 1e-12
    assert np.max(np.abs(a1)) < 1e-15


def _bb_run(lam, b, x0, alpha0, n):
    x = np.array(x0, dtype=np.float64)
    a, d_prev, xs = alpha0, None, []
    for i in range(n):
        d = lam * x + b - x
        a = scf.bb_step_size(a, d, d_prev, i)
        d_prev = d
        x = x + a * d
        xs.append((x.copy(), a))
    return xs


@pytest.mark.parametrize("lam", [0.9, 0.5, -0.3, 0.99])
def test_bb_lands_on_the_fixed_point_of_a_uniform_linear_map(lam):
    # on g(x) = lam x + b, d_i - d_{i-1} = (lam - 1) alpha_i d_{i-1}, so the
    # BB1 step of iteration 1 is alpha_1 / (alpha_1 |lam - 1|) = 1 / (1 - lam):
    # the exact fixed point x* = b / (1 - lam) after two iterations; there d
    # vanishes and the next (BB2) step keeps its size
    b = 0.4
    xs = b / (1.0 - lam)
    run = _bb_run(lam, b, [2.0, -1.0, 0.5], 0.3, 3)
    assert np.allclose(run[0][0], [2.0, -1.0, 0.5] + 0.3 * ((lam - 1.0) * np.array([2.0, -1.0, 0.5]) + b))
    assert abs(run[1][1] - 1.0 / (1.0 - lam)) < 1e-12 / (1.0 - lam)
    assert np.allclose(run[1][0], xs, rtol=1e-12, atol=1e-13)
    assert np.allclose(run[2][0], xs, rtol=1e-12, atol=1e-13)


def test_bb_step_is_clamped_and_alternates():
    # lam = 0.999: the exact step 1000 is clamped to the upper bound 100
    run = _bb_run(0.999, 0.1, [1.0, 2.0], 1.0, 2)
    assert run[1][1] == scf.BB_STEP_MAX
    # two components relaxing at different rates: BB1 for odd i, BB2 for even
    # i, each the ratio of the dot products of App. E
    lam = np.array([0.2, 0.9])
    x = np.array([1.0, 1.0])
    d0 = lam * x - x
    x1 = x + 0.5 * d0
    d1 = lam * x1 - x1
    a1 = scf.bb_step_size(0.5, d1, d0, 1)
    assert abs(a1 - 0.5 * np.dot(d0, d0) / abs(np.dot(d0, d1 - d0))) < 1e-15
    a2 = scf.bb_step_size(a1, d1, d0, 2)
    assert abs(a2 - a1 * abs(np.dot(d0, d1 - d0)) / np.dot(d1 - d0, d1 - d0)) < 1e-15


def test_bb_on_the_bcs_fixed_point_stays_put():
    from oracle import bulk
    gr = _cfg1_like()
    dbulk = bulk.bulk_gap(0.5, 16)
    delta = np.where(gr.mask, dbulk, 0)[None].astype(complex)
    d1, a1, _, _ = scf.scf(gr, delta, np.zeros((2, 32, 32)), 3, accelerator="bb", alpha=1.0)
    assert np.max(np.abs(d1[0][gr.mask] - dbulk)) < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_similarity_weight_solves_its_quadratic(seed):
    # S_C(w m + (1 - w) d, d) = smin squared is a quadratic in w:
    # (w md + (1-w) dd)^2 = smin^2 dd (w^2 mm + 2 w (1-w) md + (1-w)^2 dd);
    # its root in [0, 1] with a positive left side is the weight
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(7)
    m = -d + 0.6 * rng.standard_normal(7)  # pointing away from d
    mm, md, dd = m @ m, m @ d, d @ d
    smin = scf.CONG_SMIN
    a, b = md - dd, dd  # numerator = a w + b
    q2 = a * a - smin ** 2 * dd * (mm - 2 * md + dd)
    q1 = 2 * a * b - smin ** 2 * dd * (2 * md - 2 * dd)
    q0 = b * b - smin ** 2 * dd * dd
    roots = [r.real for r in np.roots([q2, q1, q0]) if abs(r.imag) < 1e-12 and 0 <= r.real <= 1
             and a * r.real + b > 0]
    assert len(roots) == 1
    w = scf.similarity_weight(mm, md, dd, smin)
    assert abs(w - roots[0]) < 1e-12
    u = w * m + (1 - w) * d
    assert abs(u @ d / np.sqrt((u @ u) * dd) - smin) < 1e-12


def test_congacc_component_scales_the_step_by_the_similarity():
    d = np.array([1.0, -2.0, 0.5])
    m0, a0, w0 = scf.congacc_component(None, d, 0.5, 0.3, True)
    assert np.array_equal(m0, d) and a0 == 0.5 and w0 == 0.0
    # aligned: s = 1, alpha grows by k, the weight is kept
    m1, a1, w1 = scf.congacc_component(2.0 * d, d, 0.5, 0.25, False)
    assert abs(a1 - 0.5 * scf.CONG_K) < 1e-15 and w1 == 0.25
    assert np.allclose(m1, 0.25 * 2.0 * d + 0.75 * d, rtol=1e-15)
    # pointing away: alpha shrinks by k^s (s < 0), and the weight makes the
    # new average exactly smin-similar to d
    e = np.array([2.0, 1.0, 0.0])  # orthogonal to d
    m = -d + 0.5 * e
    s = m @ d / np.sqrt((m @ m) * (d @ d))
    m2, a2, w2 = scf.congacc_component(m, d, 0.5, 0.25, False)
    assert s < 0 and abs(a2 - 0.5 * scf.CONG_K ** s) < 1e-15 and 0.0 < w2 < 1.0
    assert abs(m2 @ d / np.sqrt((m2 @ m2) * (d @ d)) - scf.CONG_SMIN) < 1e-12


def test_congacc_on_the_bcs_fixed_point_stays_put():
    from oracle import bulk
    gr = _cfg1_like()
    dbulk = bulk.bulk_gap(0.5, 16)
    delta = np.where(gr.mask, dbulk, 0)[None].astype(complex)
    d1, a1, _, _ = scf.scf(gr, delta, np.zeros((2, 32, 32)), 3, accelerator="congacc", alpha=0.5)
    assert np.max(np.abs(d1[0][gr.mask] - dbulk)) < 1e-12


def test_congacc_anti_parallel_average_restarts_from_d():
    """m exactly opposite to d: the blend w m + (1 - w) d is (1 - w(1 + c)) d
    for m = -c d, so its similarity with d is +1 below w = 1/(1 + c) and -1
    above, and no weight gives s_min.  A bisection on the similarity stops
    where the blend vanishes (its norm falls to rounding level, which froze
    the component in the earlier rule); the rule takes w = 0 instead, so the
    average restarts from d and the step shrinks by k^-1."""
    d = np.array([0.3, -1.1, 0.7, 2.0])
    m = -0.4 * d
    mm, md, dd = m @ m, m @ d, d @ d
    w_bis = scf.similarity_weight(mm, md, dd, scf.CONG_SMIN)
    blend = w_bis * m + (1 - w_bis) * d
    assert np.linalg.norm(blend) < 1e-6 * np.linalg.norm(d)   # the collapse the rule avoids
    st = {}
    m1, a1, w1 = scf.congacc_component(m, d, 0.8, 0.35, False, stats=st)
    assert w1 == 0.0 and np.array_equal(m1, d)
    assert abs(a1 - 0.8 / scf.CONG_K) < 1e-15
    assert st == {"anti": 1}
    # nearly but not exactly opposite: the equation has its root again and
    # the bisection sets the weight
    e = np.array([1.0, 0.5, 0.2, -0.1])
    e -= (e @ d) / dd * d
    mb = -0.4 * d + 1e-3 * e
    st = {}
    m2, a2, w2 = scf.congacc_component(mb, d, 0.8, 0.35, False, stats=st)
    assert st == {"bisect": 1} and 0.0 < w2 < 1.0
    assert abs(m2 @ d / np.sqrt((m2 @ m2) * dd) - scf.CONG_SMIN) < 1e-9


def test_congacc_collinear_component_converges_to_its_fixed_point():
    """A component whose map is g(x) = 0 (every d, m and x are multiples of
    one vector): with alpha growing by k per iteration the steps overshoot,
    m turns exactly opposite to d, and the earlier bisection rule froze x at
    a nonzero value with a step of rounding size.  With the anti-parallel
    rule x keeps shrinking toward the fixed point 0."""
    x0 = np.array([0.2, -0.5, 0.1])
    x = x0.copy()
    m, a, w, first = None, 0.5, 0.0, True
    st = {}
    for _ in range(40):
        d = -x
        m, a, w = scf.congacc_component(m, d, a, w, first, stats=st)
        first = False
        x = x + a * m
    assert st.get("anti", 0) >= 1
    assert np.linalg.norm(x) < 1e-6 * np.linalg.norm(x0)


def test_scf_residual_is_checked_before_the_step():
    """Alg. 1 checks Eq. global_error after the A-solve and before the
    accelerator: eps_Delta = ||g(x) - x|| / ||x||, whatever step is then
    taken.  A Picard run with alpha = 0.3 reports the same first eps_Delta
    as one with alpha = 1 (both start from the same x)."""
    gr = _cfg1_like()
    rng = np.random.default_rng(3)
    delta = np.where(gr.mask, 0.25 * (1 + 0.05 * rng.uniform(-1, 1, gr.mask.shape)), 0)[None].astype(complex)
    _, _, h1, _ = scf.scf(gr, delta, np.zeros((2, 32, 32)), 1, alpha=1.0)
    _, _, h3, _ = scf.scf(gr, delta, np.zeros((2, 32, 32)), 1, alpha=0.3)
    out = gr.iterate(delta, np.zeros((2, 32, 32)))
    m = gr.mask
    ref = np.linalg.norm(out["delta_new"][:, m] - delta[:, m]) / np.linalg.norm(delta[:, m])
    assert abs(h1[0][0] - ref) < 1e-14 and abs(h3[0][0] - ref) < 1e-14


def test_scf_without_screening_holds_A_at_zero():
    """kappa <= 0: no induced vector potential; a nonzero A given to the
    SCF is dropped before the first sweep."""
    gr = _cfg1_like()
    delta = np.where(gr.mask, 0.25, 0)[None].astype(complex)
    A0 = 0.01 * np.ones((2, 32, 32))
    d1, a1, h, _ = scf.scf(gr, delta, A0, 2, accelerator="congacc", alpha=0.5)
    d2, _, _, _ = scf.scf(gr, delta, np.zeros((2, 32, 32)), 2, accelerator="congacc", alpha=0.5)
    assert np.array_equal(a1, np.zeros((2, 32, 32))) and all(r[2] == 0.0 for r in h)
    assert np.array_equal(d1, d2)
