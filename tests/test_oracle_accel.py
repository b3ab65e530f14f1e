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
