"""Closed forms of the homogeneous (bulk) state, used to pin the oracle.

Oracle (test infrastructure only).  Units of App. F: energies in 2 pi k_B Tc,
t = T/Tc, t~ = t/(2 pi); eps~_p = z_p t~ for Ozaki pole z_p.
"""
import math
import numpy as np
from scipy.optimize import brentq

from . import tables

DELTA0 = math.pi * math.exp(-np.euler_gamma) / (2.0 * math.pi)  # BCS gap at T=0 in 2 pi k_B Tc


def gap_residual(d, t, n_poles, eta2=None, weights=None):
    """Regularised gap equation (Eq. gapeq_regularized) for a homogeneous
    state Delta(phi) = d eta(phi): f = pi Delta/Omega_p at the poles gives
    ln t = 2 pi sum_p R_p < |eta|^2 (1/sqrt(eps~_p^2 + d^2 |eta|^2) - 1/eps~_p) >.
    eta2: |eta(phi_k)|^2 samples, weights: Fermi-surface weights."""
    z, res = tables.ozaki_poles(n_poles)
    tt = t / (2.0 * math.pi)
    ep = z * tt
    if eta2 is None:
        eta2 = np.array([1.0])
        weights = np.array([1.0])
    tot = 0.0
    for e2, w in zip(eta2, weights):
        tot += w * e2 * np.sum(res * (1.0 / np.sqrt(ep * ep + d * d * e2) - 1.0 / ep))
    # pi T sum over both signs of e_n = 2 pi t~ sum over the positive poles
    return math.log(t) - 2.0 * math.pi * tt * tot


def bulk_gap(t, n_poles, eta2=None, weights=None):
    """Root of the homogeneous gap equation (0 above the transition)."""
    f = lambda d: gap_residual(d, t, n_poles, eta2, weights)
    if f(1e-12) >= 0.0:
        return 0.0
    return brentq(f, 1e-12, 2.0, xtol=1e-15, rtol=1e-15, maxiter=200)


def bulk_free_energy(d, t, n_poles, eta2=None, weights=None):
    """Bulk free-energy density (Sec. V, Eq. FEbulk, per N_F):
      |D|^2 ln t + pi T sum_n |D|^4 / (|e_n| (Omega_n + |e_n|)^2),
    with the Matsubara sum replaced by the Ozaki poles (both signs)."""
    z, res = tables.ozaki_poles(n_poles)
    tt = t / (2.0 * math.pi)
    ep = z * tt
    if eta2 is None:
        eta2 = np.array([1.0])
        weights = np.array([1.0])
    tot = d * d * math.log(t)
    for e2, w in zip(eta2, weights):
        a2 = d * d * e2
        om = np.sqrt(ep * ep + a2)
        tot += w * 2.0 * math.pi * tt * np.sum(res * a2 * a2 / (ep * (om + ep) ** 2))
    return tot


def yoshida(d, t, n_poles):
    """Angle-resolved Yoshida function of Sec. V.A for |Delta(p)| = d,
    Y = pi T sum_n |D|^2 / Lambda_n^3 (sum over both signs of e_n),
    i.e. 2 pi t~ sum_p R_p d^2 / Lambda_p^3 over the positive poles."""
    z, res = tables.ozaki_poles(n_poles)
    tt = t / (2.0 * math.pi)
    ep = z * tt
    om = np.sqrt(ep * ep + d * d)
    return 2.0 * math.pi * tt * np.sum(res * d * d / om ** 3)
