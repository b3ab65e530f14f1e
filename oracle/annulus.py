"""London-Maxwell closed forms of a screened s-wave annulus.

Oracle (test infrastructure only).  Follows Sec. V.A: the London-Maxwell
equation of an annulus with a phase winding n (Eq. LMeqRing), its
cylindrically symmetric solution in modified Bessel functions (Eqs. Aring,
Bring) and the magnetic moment it implies (Eq. magneticannulus).  These are
the linear-response predictions that a self-consistent solve of an s-wave
annulus must reproduce; nothing here runs the method itself.

Units (App. F): lengths in xi0, the vector potential in A0 = Phi0/(pi xi0),
so the flux quantum is Phi0 = pi, fields in B0 = Phi0/(pi xi0^2), currents
in j0 and moments in m0 = j0 xi0 V.  The annulus has outer and inner radii
Ro > Ri, area A = pi (Ro^2 - Ri^2) and hole area Ah = pi Ri^2; the applied
field is alpha flux quanta through A, B_ext = alpha Phi0 / A.  The
penetration depth at temperature T is lam = lam0 / sqrt(Y) with Y the
superfluid fraction (Sec. V.A), lam0 = kappa in units of xi0.
"""
import math

from scipy.special import iv, kv

PHI0 = math.pi


def _coefficients(Ro, Ri, lam, alpha, n):
    """(a, b, beta, M) of Eq. Aring: A bounded in the hole and continuous at
    Ri, B continuous at Ro (Sec. V.A)."""
    A = math.pi * (Ro * Ro - Ri * Ri)
    Ah = math.pi * Ri * Ri
    I0o, I0i, I2o, I2i = iv(0, Ro / lam), iv(0, Ri / lam), iv(2, Ro / lam), iv(2, Ri / lam)
    K0o, K0i, K2i = kv(0, Ro / lam), kv(0, Ri / lam), kv(2, Ri / lam)
    M = I0o * K2i - I2i * K0o
    a = (K2i / A * alpha + K0o / Ah * n) / M
    b = (I2i / A * alpha + I0o / Ah * n) / M
    beta = (2.0 * math.pi * lam * lam / A * alpha - (I0o * K0i - I0i * K0o) * n) / M
    return a, b, beta, M


def field(R, Ro, Ri, lam, alpha, n):
    """Azimuthal vector potential A(R) and field B(R) (Eqs. Aring, Bring) at
    radii 0 < R <= Ro; the hole (R < Ri) carries the uniform field
    beta Phi0 / Ah."""
    a, b, beta, _ = _coefficients(Ro, Ri, lam, alpha, n)
    Ah = math.pi * Ri * Ri
    if R < Ri:
        return beta * PHI0 / Ah * R / 2.0, beta * PHI0 / Ah
    x = R / lam
    A_R = PHI0 * lam * (a * iv(1, x) + b * kv(1, x)) - n * PHI0 / (2.0 * math.pi * R)
    B_R = PHI0 * (a * iv(0, x) - b * kv(0, x))
    return A_R, B_R


def current(R, Ro, Ri, lam0, Y, alpha, n):
    """Linear-response supercurrent along phi in the annulus (Eq. LMeqRing
    with Ampere's law): j = -(lam0^2 / lam^2) (A + n Phi0 / (2 pi R))
    in units of j0, i.e. -Y times the gauge-invariant superfluid momentum."""
    lam = lam0 / math.sqrt(Y)
    A_R, _ = field(R, Ro, Ri, lam, alpha, n)
    return -Y * (A_R + n * PHI0 / (2.0 * math.pi * R))


def moment(Ro, Ri, lam0, Y, alpha, n):
    """m_z / m0 = d_alpha alpha + d_n n (Eq. magneticannulus) with
      d_alpha = (pi lam0^2 / A) (A + Ah) / (M A) (I2(Ri) K2(Ro) - I2(Ro) K2(Ri)),
      d_n     = (pi lam0^2 / A) (2 pi lam^2 / (M Ah) - 1),
    the Bessel functions at R / lam.  Returns (m, d_alpha, d_n)."""
    lam = lam0 / math.sqrt(Y)
    A = math.pi * (Ro * Ro - Ri * Ri)
    Ah = math.pi * Ri * Ri
    _, _, _, M = _coefficients(Ro, Ri, lam, alpha, n)
    pre = math.pi * lam0 * lam0 / A
    d_alpha = pre * (A + Ah) / (M * A) * (iv(2, Ri / lam) * kv(2, Ro / lam) - iv(2, Ro / lam) * kv(2, Ri / lam))
    d_n = pre * (2.0 * math.pi * lam * lam / (M * Ah) - 1.0)
    return d_alpha * alpha + d_n * n, d_alpha, d_n


def free_energy_shift(Ro, Ri, lam0, Y, alpha, n, kappa):
    """Omega(alpha, n) - Omega_bulk of the screened annulus in linear response
    (Sec. V.A, Eqs. FEsuperflow, lFEkin, lFEmag) with the London fields of
    Eqs. Aring, Bring, in units of N_F (2 pi k_B T_c)^2 xi0^2:
      kinetic  int over the annulus of (Y / 2) (A + n Phi0 / (2 pi R))^2
               (the density Y q^2 / 8 of Eq. lFEkin with q = 2 (A + n / (2R)),
               q the phase gradient plus the vector potential in 1/xi0),
      magnetic int of (kappa^2 / 2) (B - B_ext)^2 over the annulus and the
               hole (outside the annulus B = B_ext; kappa^2 / 2 is 1 / (8 pi)
               in these units).
    Returns (total, kinetic, magnetic)."""
    from scipy.integrate import quad
    lam = lam0 / math.sqrt(Y)
    A = math.pi * (Ro * Ro - Ri * Ri)
    Ah = math.pi * Ri * Ri
    b_ext = alpha * PHI0 / A
    kin = quad(lambda R: 0.5 * Y * (field(R, Ro, Ri, lam, alpha, n)[0] + n * PHI0 / (2 * math.pi * R)) ** 2
               * 2 * math.pi * R, Ri, Ro, limit=200)[0]
    mag = quad(lambda R: 0.5 * kappa * kappa * (field(R, Ro, Ri, lam, alpha, n)[1] - b_ext) ** 2 * 2 * math.pi * R,
               Ri, Ro, limit=200)[0]
    mag += 0.5 * kappa * kappa * (field(0.5 * Ri, Ro, Ri, lam, alpha, n)[1] - b_ext) ** 2 * Ah
    return kin + mag, kin, mag
