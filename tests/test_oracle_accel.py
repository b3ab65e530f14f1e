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
