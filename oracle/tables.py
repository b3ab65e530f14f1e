"""Small tables of the method: Ozaki poles, Fermi-surface weights, basis.

Oracle (test infrastructure only).
"""
import math
import numpy as np


def ozaki_poles(n_poles):
    """Poles z_p > 0 and residues R_p of the Ozaki continued-fraction
    expansion of the Fermi function (Sec. III.A cites Ozaki 2007 for the
    energy sums; the construction is not printed in the paper).

    Reading: the 2N x 2N real symmetric tridiagonal matrix with zero
    diagonal and off-diagonal b_m = 1 / (2 sqrt((2m-1)(2m+1))), m=1..2N-1.
    For each of its N positive eigenvalues lam_p with normalised
    eigenvector v_p: z_p = 1/lam_p and R_p = v_p[0]^2 / (4 lam_p^2), so that
        1/(1+e^x) = 1/2 - sum_p 2 R_p x / (x^2 + z_p^2).
    Returned in increasing z_p.  The Matsubara sum is the special case
    z = (2n+1) pi, R = 1.
    """
    if n_poles < 1:
        raise ValueError("n_poles must be >= 1")
    n = 2 * n_poles
    m = np.arange(1, n, dtype=np.float64)
    b = 1.0 / (2.0 * np.sqrt((2.0 * m - 1.0) * (2.0 * m + 1.0)))
    mat = np.diag(b, 1) + np.diag(b, -1)
    lam, vec = np.linalg.eigh(mat)
    keep = lam > 0.0
    lam = lam[keep]
    v0 = vec[0, keep]
    order = np.argsort(-lam)
    lam = lam[order]
    v0 = v0[order]
    z = 1.0 / lam
    res = v0 * v0 / (4.0 * lam * lam)
    return z, res


def fermi_from_poles(x, z, res):
    """The Fermi function rebuilt from poles and residues (Ozaki form)."""
    x = np.asarray(x, dtype=np.float64)[..., None]
    return 0.5 - np.sum(2.0 * res * x / (x * x + z * z), axis=-1)


def fs_angles(n_theta):
    """Discrete Fermi-surface angles phi_k = 2 pi k / N (Sec. III.A)."""
    return np.array([2.0 * math.pi * k / n_theta for k in range(n_theta)])


def fs_weights(n_theta):
    """Normalised Fermi-surface quadrature weights (Sec. III.A).

    The paper picks Boole's rule, Simpson's 3/8, Simpson's 1/3 or the
    trapezoidal rule when the number of angles is divisible by 4, 3, 2, or
    otherwise.  Reading: the composite rule applied periodically around the
    circle, so that the shared end points of adjacent panels add up:
    Boole (14,32,12,32), Simpson 3/8 (2,3,3), Simpson 1/3 (2,4), trapezoid
    (1); scaled so that the weights sum to one (the Fermi-surface average).
    """
    if n_theta < 1:
        raise ValueError("n_theta must be >= 1")
    if n_theta % 4 == 0:
        pattern = [14.0, 32.0, 12.0, 32.0]
    elif n_theta % 3 == 0:
        pattern = [2.0, 3.0, 3.0]
    elif n_theta % 2 == 0:
        pattern = [2.0, 4.0]
    else:
        pattern = [1.0]
    w = np.array([pattern[k % len(pattern)] for k in range(n_theta)])
    return w / w.sum()


BASIS_NAMES = ("s", "dx2y2", "dxy", "g")


def basis(name, phi, crystal_rotation=0.0):
    """Order-parameter basis functions for a circular Fermi surface
    (App. F, basis-function table): s = 1, d_{x2-y2} = sqrt2 cos 2phi,
    d_xy = sqrt2 sin 2phi, g = sqrt2 sin 4phi, evaluated at
    phi - 2 pi theta_c with the crystal-axes rotation theta_c given in
    full turns (App. B)."""
    p = np.asarray(phi, dtype=np.float64) - 2.0 * math.pi * crystal_rotation
    if name == "s":
        v = np.ones_like(p)
    elif name == "dx2y2":
        v = math.sqrt(2.0) * np.cos(2.0 * p)
    elif name == "dxy":
        v = math.sqrt(2.0) * np.sin(2.0 * p)
    elif name == "g":
        v = math.sqrt(2.0) * np.sin(4.0 * p)
    else:
        raise ValueError("unknown basis function %r" % (name,))
    return v.astype(np.complex128)
