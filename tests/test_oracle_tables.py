"""Pins of the oracle's tables against what mathematics fixes."""
import math
import os

import numpy as np
import pytest
from scipy.integrate import dblquad

from oracle import tables, fields


@pytest.mark.parametrize("n", [1, 4, 16, 64])
def test_ozaki_reproduces_fermi_function(n):
    # 1/(1+e^x) = 1/2 - sum_p 2 R_p x/(x^2+z_p^2); the error falls fast with n
    z, r = tables.ozaki_poles(n)
    x = np.linspace(-30, 30, 601)
    exact = 0.5 * (1.0 - np.tanh(0.5 * x))
    err = np.max(np.abs(tables.fermi_from_poles(x, z, r) - exact))
    bound = {1: 0.5, 4: 2e-2, 16: 1e-14, 64: 1e-14}[n]
    assert err < bound


def test_ozaki_low_poles_are_matsubara():
    # the lowest Ozaki poles converge to (2n+1) pi with unit residue
    z, r = tables.ozaki_poles(16)
    assert np.allclose(z[:6], np.pi * (2 * np.arange(6) + 1), rtol=1e-6)
    assert np.allclose(r[:6], 1.0, atol=1e-6)
    assert np.all(np.diff(z) > 0) and np.all(r > 0)


def test_ozaki_sum_matches_brute_force_matsubara():
    # T sum_n F(i e_n) for F = 1/(e^2 + a^2) equals tanh(a/2T)/(2a) in
    # closed form; the Ozaki pole sum reproduces it
    a, T = 0.7, 0.3
    z, r = tables.ozaki_poles(32)
    ozaki = T * np.sum(r * 2.0 / (a * a - (z * T) ** 2 * -1.0))
    exact = math.tanh(a / (2 * T)) / (2 * a)
    n = np.arange(-10 ** 6, 10 ** 6)
    en = np.pi * T * (2 * n + 1)
    brute = T * np.sum(1.0 / (en * en + a * a))
    assert abs(ozaki - exact) < 1e-12
    assert abs(brute - exact) < 1e-6


@pytest.mark.parametrize("n", [32, 33, 34, 35, 64])
def test_weights_normalised_and_exact_on_low_harmonics(n):
    w = tables.fs_weights(n)
    phi = tables.fs_angles(n)
    assert abs(w.sum() - 1.0) < 1e-15
    for m in range(1, 4):
        assert abs(np.sum(w * np.cos(m * phi))) < 1e-14
        assert abs(np.sum(w * np.sin(m * phi))) < 1e-14


def test_boole_pattern():
    w = tables.fs_weights(8) * 90.0 * 2  # two Boole panels
    assert np.allclose(w / w[1] * 32, [14, 32, 12, 32, 14, 32, 12, 32])


@pytest.mark.parametrize("n", [32, 64])
def test_basis_orthonormal(n):
    phi = tables.fs_angles(n)
    w = tables.fs_weights(n)
    B = np.array([tables.basis(b, phi) for b in ("s", "dx2y2", "dxy")])
    gram = np.einsum("k,ak,bk->ab", w, np.conj(B), B)
    assert np.allclose(gram, np.eye(3), atol=1e-14)


def test_basis_rotation_in_turns():
    phi = tables.fs_angles(64)
    a = tables.basis("dx2y2", phi, crystal_rotation=1.0 / 8.0)
    b = tables.basis("dxy", phi)
    assert np.allclose(a, b, atol=1e-14)

def _golden_basis_rows():
    rows = []
    path = os.path.join(os.path.dirname(__file__), "golden", "basis_functions.txt")
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _eval_expr(expr, **names):
    env = {"__builtins__": {}, "sqrt": np.sqrt, "sin": np.sin, "cos": np.cos}
    env.update(names)
    return np.broadcast_to(np.asarray(eval(expr, env), dtype=np.float64), names["phi"].shape)


@pytest.mark.parametrize("row", _golden_basis_rows(), ids=lambda r: r[0])
def test_basis_matches_the_tabulated_polynomials(row):
    # both columns of the table: Delta(k) normalised to unit Fermi-surface
    # mean square gives eta(phi) with a positive factor, and the oracle's
    # basis is that eta
    _, name, poly, eta = row
    phi = tables.fs_angles(64)
    w = tables.fs_weights(64)
    pk = _eval_expr(poly, kx=np.cos(phi), ky=np.sin(phi), phi=phi)
    et = _eval_expr(eta, phi=phi)
    assert np.allclose(pk / math.sqrt(np.sum(w * pk * pk)), et, atol=1e-14)
    ob = tables.basis(name, phi)
    assert np.max(np.abs(ob.imag)) == 0.0
    assert np.allclose(ob.real, et, atol=1e-14)


@pytest.mark.parametrize("m,n,h", [(0, 0, 1.0), (1, 0, 1.0), (2, 3, 1.0), (5, 1, 1.0), (3, 2, 0.25), (0, 4, 0.1)])
def test_green_kernel_closed_form_matches_quadrature(m, n, h):
    # App. D: G_{m,n} = (1/4pi) int over one cell of ln(((x'+hm)^2+(y'+hn)^2))
    f = lambda y, x: math.log((x + h * m) ** 2 + (y + h * n) ** 2)
    if m == 0 and n == 0:
        # split at the log singularity
        val = 0.0
        for (xa, xb) in ((-h / 2, 0), (0, h / 2)):
            for (ya, yb) in ((-h / 2, 0), (0, h / 2)):
                val += dblquad(f, xa, xb, ya, yb, epsabs=1e-14, epsrel=1e-13)[0]
    else:
        val = dblquad(f, -h / 2, h / 2, -h / 2, h / 2, epsabs=1e-14, epsrel=1e-13)[0]
    assert abs(fields.green_kernel(m, n, h) - val / (4 * math.pi)) < 1e-12 * max(1.0, h * h)


def test_green_kernel_symmetric():
    assert abs(fields.green_kernel(2, 5, 0.3) - fields.green_kernel(5, 2, 0.3)) < 1e-15
