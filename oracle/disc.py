"""Superflow free energy of a thin s-wave disc without screening.

Oracle (test infrastructure only).  Follows Sec. V.B: with the penetration
depth the largest scale, the superfluid momentum of a disc of radius R in
the applied field (alpha flux quanta through its area, symmetric gauge) with
a phase winding n around its centre is p_s = (hbar / 2)(n / r + alpha r / R^2)
along phi-hat, and the linear-response kinetic free energy (Eq. lFEkin)
gives (Eqs. 0vor, 1vor, lFKinfty)
  n = 0:   (Omega(alpha) - Omega_bulk) / A = dw alpha^2,
  n = -1:  (Omega(alpha) - Omega_bulk) / A = dw (eps_core - 4 alpha + alpha^2),
  dw = (xi0 / R)^2 Y / 16,
with Y the superfluid fraction at the temperature and eps_core the vortex
core term, which the London theory leaves open.  Units (App. F): lengths in
xi0, free-energy densities in N_F (2 pi k_B T_c)^2.
"""


def kinetic_coefficient(R, Y):
    """dw = Y / (16 R^2) (Eq. lFKinfty)."""
    return Y / (16.0 * R * R)


def free_energy_shift(R, Y, alpha, n, eps_core=0.0):
    """(Omega(alpha) - Omega_bulk) / A for n = 0 or n = -1 (Eqs. 0vor, 1vor)."""
    dw = kinetic_coefficient(R, Y)
    if n == 0:
        return dw * alpha * alpha
    if n == -1:
        return dw * (eps_core - 4.0 * alpha + alpha * alpha)
    raise ValueError("the closed forms cover n = 0 and n = -1")
