"""Vector potential: external gauges and the induced A from Ampere's law.

Oracle (test infrastructure only).  Follows Sec. II (Ampere's law and units,
App. F unit table), App. D (cell-averaged 2D Laplacian Green's function,
mean-current subtraction) and App. B (gauge choice, charge sign).
"""
import math
import numpy as np

GAUGES = ("symmetric", "landau", "solenoid")


def external_A(gauge, flux_quanta, area, cx, cy, x, y):
    """External vector potential in units of A0 = Phi0/(pi xi0) (App. F).

    symmetric: B/2 (-(y-cy), x-cx) with B = pi alpha / area (alpha flux
      quanta through the grain area, App. F), in units of B0;
    solenoid: alpha / (2 r) along the azimuthal unit vector (flux alpha
      through a thin solenoid at the centre, App. F);
    landau (formula not printed; reading): (-B (y-cy), 0) with the same B.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    dx = x - cx
    dy = y - cy
    if flux_quanta == 0.0:
        return np.zeros_like(dx), np.zeros_like(dy)
    if gauge == "symmetric":
        b = math.pi * flux_quanta / area
        return -0.5 * b * dy, 0.5 * b * dx
    if gauge == "landau":
        b = math.pi * flux_quanta / area
        return -b * dy, np.zeros_like(dx)
    if gauge == "solenoid":
        r2 = dx * dx + dy * dy
        r2 = np.where(r2 > 0.0, r2, np.inf)
        return -0.5 * flux_quanta * dy / r2, 0.5 * flux_quanta * dx / r2
    raise ValueError("unknown gauge %r" % (gauge,))


def green_kernel(m, n, h):
    """Cell-averaged Green's function of the 2D Laplacian, G_{m,n} of
    App. D in closed form (h in units of xi0):
      G = h^2/(4 pi) (2 ln h - ln 2 - 3 + 1/4 sum_{a,b=+-} Gamma(a m, b n)),
      Gamma(m,n) = alpha(m,n) + beta(m,n) + beta(n,m),
      alpha(m,n) = (1+2m)(1+2n) ln((1+2m)^2/2 + (1+2n)^2/2),
      beta(m,n) = (-2m^2 + 2n^2 + 4n + 1) atan((1+2m)/(1+2n))."""
    m = np.asarray(m, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)

    def alpha(a, b):
        return (1 + 2 * a) * (1 + 2 * b) * np.log(0.5 * (1 + 2 * a) ** 2 + 0.5 * (1 + 2 * b) ** 2)

    def beta(a, b):
        return (-2 * a * a + 2 * b * b + 4 * b + 1) * np.arctan((1 + 2 * a) / (1 + 2 * b))

    tot = 0.0
    for sa in (1.0, -1.0):
        for sb in (1.0, -1.0):
            a = sa * m
            b = sb * n
            tot = tot + alpha(a, b) + beta(a, b) + beta(b, a)
    return h * h / (4.0 * math.pi) * (2.0 * math.log(h) - math.log(2.0) - 3.0 + 0.25 * tot)


def solve_A(jx, jy, mask, h, kappa, method="auto"):
    """Induced vector potential (App. D):
      A_ind[m,n] = -kappa^-2 sum_{m',n'} G_{|m'-m|,|n'-n|} j'[m',n'],
    with j' = (j - mean of j over the grain cells) on grain cells and zero
    elsewhere (reading of the mean-current subtraction).  kappa <= 0 means
    an infinite penetration depth: A_ind = 0.  The correlation is done as a
    direct double sum for small grids and by zero-padded FFT otherwise
    (identical up to rounding)."""
    ny, nx = jx.shape
    if kappa <= 0.0:
        return np.zeros((ny, nx)), np.zeros((ny, nx))
    msk = mask.astype(bool)
    jpx = np.where(msk, jx - jx[msk].mean(), 0.0)
    jpy = np.where(msk, jy - jy[msk].mean(), 0.0)
    if method == "auto":
        method = "direct" if nx * ny <= 64 * 64 else "fft"
    if method == "direct":
        I, J = np.meshgrid(np.arange(nx), np.arange(ny))
        ax = np.zeros((ny, nx))
        ay = np.zeros((ny, nx))
        for r in range(ny):
            for c in range(nx):
                G = green_kernel(np.abs(I - c), np.abs(J - r), h)
                ax[r, c] = np.sum(G * jpx)
                ay[r, c] = np.sum(G * jpy)
    else:
        py, px = 2 * ny, 2 * nx
        dm = np.minimum(np.arange(px), px - np.arange(px))
        dn = np.minimum(np.arange(py), py - np.arange(py))
        Gp = green_kernel(dm[None, :], dn[:, None], h)
        Gh = np.fft.fft2(Gp)
        jc = np.zeros((py, px), dtype=np.complex128)
        jc[:ny, :nx] = jpx + 1j * jpy
        conv = np.fft.ifft2(np.fft.fft2(jc) * Gh)[:ny, :nx]
        ax, ay = conv.real, conv.imag
    s = -1.0 / (kappa * kappa)
    return s * ax, s * ay


def green_matrix(n, h):
    """The N x N matrix G_{m,n}, 0 <= m, n < N, of App. D (symmetric)."""
    m = np.arange(n)
    return green_kernel(m[:, None], m[None, :], h)


def truncation_rank(lams, eps):
    """N* of App. D: with the eigenvalues sorted by decreasing magnitude,
    the smallest integer with sqrt(1 - sum_{n<N*} lam_n^2 / sum_n lam_n^2)
    < eps (eps > 0).  The left side is evaluated as
    sqrt(sum_{n>=N*} lam_n^2 / sum_n lam_n^2), equal in exact arithmetic,
    so that tolerances below 1e-8 are not lost to the cancellation in
    1 - (kept / total)."""
    l2 = np.sort(np.abs(np.asarray(lams, dtype=np.float64)))[::-1] ** 2
    tot = float(np.sum(l2))
    # tail[k] = sum_{n >= k} lam_n^2, summed from the smallest
    tail = np.concatenate([np.cumsum(l2[::-1])[::-1], [0.0]])
    for k in range(len(l2) + 1):
        if math.sqrt(tail[k] / tot) < eps:
            return k
    return len(l2)


def green_eigen(n, h, eps):
    """Eigen-decomposition of G (App. D), G = V Lambda V^T, truncated to the
    N* eigenpairs of largest |lambda| (truncation_rank).  Returns (lam[N*],
    V[N, N*]) with the eigenvectors as columns."""
    lam, vec = np.linalg.eigh(green_matrix(n, h))
    order = np.argsort(-np.abs(lam), kind="stable")
    lam, vec = lam[order], vec[:, order]
    k = truncation_rank(lam, eps)
    return lam[:k], vec[:, :k]


def solve_A_eigen(jx, jy, mask, h, kappa, eps):
    """Induced vector potential with the separable, eigen-truncated kernel of
    App. D on an N x N grid: with G_{a,b} = sum_k lam_k V_a^(k) V_b^(k),
      A[r,c] = -kappa^-2 sum_{k<N*} lam_k sum_{r',c'} V^(k)_{|r'-r|} V^(k)_{|c'-c|} j'[r',c'],
    i.e. A = -kappa^-2 sum_k lam_k T_k J' T_k with the symmetric Toeplitz
    matrices T_k[a,b] = V^(k)_{|a-b|}; j' is the current minus its grain
    mean on grain cells, zero elsewhere (as in solve_A).  eps = 0: no
    decomposition, the full kernel (solve_A).  Returns (A_x, A_y, N*)."""
    ny, nx = jx.shape
    if ny != nx:
        raise ValueError("the eigen-truncated kernel needs a square grid")
    if kappa <= 0.0:
        return np.zeros((ny, nx)), np.zeros((ny, nx)), 0
    if eps <= 0.0:
        ax, ay = solve_A(jx, jy, mask, h, kappa)
        return ax, ay, nx
    msk = mask.astype(bool)
    jpx = np.where(msk, jx - jx[msk].mean(), 0.0)
    jpy = np.where(msk, jy - jy[msk].mean(), 0.0)
    lam, V = green_eigen(nx, h, eps)
    idx = np.abs(np.arange(nx)[:, None] - np.arange(nx)[None, :])
    ax = np.zeros((ny, nx))
    ay = np.zeros((ny, nx))
    for k in range(len(lam)):
        T = V[idx, k]
        ax += lam[k] * (T @ jpx @ T)
        ay += lam[k] * (T @ jpy @ T)
    s = -1.0 / (kappa * kappa)
    return s * ax, s * ay, len(lam)


def magnetic_moment(jx, jy, mask, X, Y, cx, cy):
    """Magnetic moment of the in-plane current (Sec. V.A,
    Eq. magnetic_moment_def), m = (N_l d / 2) int R x j dR, along z, in the
    unit m0 = j0 xi0 V with V = N_l d A (A the grain area h^2 x grain
    cells): m_z / m0 = (1 / (2 A)) h^2 sum over grain cells of
    ((x - cx) j_y - (y - cy) j_x) at the cell centres X, Y, about the
    origin (cx, cy) (reading: the grid centre).  The h^2 cancels."""
    msk = np.asarray(mask, dtype=bool)
    tq = (X - cx) * jy - (Y - cy) * jx
    return float(np.sum(tq[msk])) / (2.0 * float(np.count_nonzero(msk)))


def curl(ax, ay, h):
    """B = d_x A_y - d_y A_x with central differences inside and one-sided
    differences at the array edge (reading)."""
    def ddx(f):
        d = np.empty_like(f)
        d[:, 1:-1] = (f[:, 2:] - f[:, :-2]) / (2 * h)
        d[:, 0] = (f[:, 1] - f[:, 0]) / h
        d[:, -1] = (f[:, -1] - f[:, -2]) / h
        return d

    def ddy(f):
        return ddx(f.T).T

    return ddx(ay) - ddy(ax)
