"""Independent mathematics used to pin the oracle.

Nothing here calls the oracle or the GPU library.  Each helper is a textbook
fact about periodic cubic splines, written in a different form from the
oracle's (dense matrices, the centred B-spline, the circulant inverse in closed
form, Fourier multipliers), so that a mistake in the oracle does not repeat
itself here.
"""
import numpy as np

Z1 = np.sqrt(3.0) - 2.0  # pole of the cubic B-spline interpolation filter


def circulant_141(n):
    """Dense periodic matrix of (S[m-1] + 4 S[m] + S[m+1]) / 6."""
    a = np.zeros((n, n))
    for m in range(n):
        a[m, m] = 4.0 / 6.0
        a[m, (m - 1) % n] += 1.0 / 6.0
        a[m, (m + 1) % n] += 1.0 / 6.0
    return a


def circulant_141_inverse_closed_form(n):
    """(A^-1)[m, q] = sqrt(3) (z1^d + z1^(n-d)) / (1 - z1^n), d = (m - q) mod n,
    z1 = sqrt(3) - 2: the periodic sum of the two-sided geometric kernel
    sqrt(3) z1^|j| that inverts the 1-4-1/6 stencil on the infinite line."""
    d = (np.arange(n)[:, None] - np.arange(n)[None, :]) % n
    return np.sqrt(3.0) * (Z1 ** d + Z1 ** (n - d)) / (1.0 - Z1 ** n)


def fourier_multiplier(kappa_h):
    """Spline coefficients of the samples exp(i kappa m h) are
    3 / (2 + cos(kappa h)) times the samples."""
    return 3.0 / (2.0 + np.cos(kappa_h))


def beta3(u):
    """Centred cubic B-spline: 2/3 - u^2 + |u|^3/2 on |u| < 1,
    (2 - |u|)^3 / 6 on 1 <= |u| < 2, zero outside."""
    a = np.abs(u)
    return np.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3,
                    np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))


def dbeta3(u):
    """Derivative of beta3."""
    a = np.abs(u)
    s = np.sign(u)
    return np.where(a < 1.0, -2.0 * u + 1.5 * s * a * a,
                    np.where(a < 2.0, -0.5 * s * (2.0 - a) ** 2, 0.0))


def shadow_grid_units(x, n, L):
    """Position in grid units folded into [0, n) with numpy's remainder."""
    return np.mod(np.asarray(x) * (n / L), n)


def dense_spline_3d(field):
    """Unpadded spline coefficients of a [nz][ny][nx] grid by solving each
    axis with the dense matrix (numpy.linalg.solve)."""
    nz, ny, nx = field.shape
    s = np.linalg.solve(circulant_141(nx), field.reshape(-1, nx).T).T.reshape(field.shape)
    s = np.moveaxis(s, 1, 2)  # [nz][nx][ny]
    s = np.linalg.solve(circulant_141(ny), s.reshape(-1, ny).T).T.reshape(nz, nx, ny)
    s = np.moveaxis(s, 2, 1)
    s = np.moveaxis(s, 0, 2)  # [ny][nx][nz]
    s = np.linalg.solve(circulant_141(nz), s.reshape(-1, nz).T).T.reshape(ny, nx, nz)
    return np.moveaxis(s, 2, 0)


def brute_force_spline(S, pos, L):
    """sum over ALL coefficients S[r][q][p] (and their periodic images) of
    S * beta3(u_x - p) beta3(u_y - q) beta3(u_z - r), u = shadow position in
    grid units.  No cells, no padding, no truncated stencil."""
    nz, ny, nx = S.shape
    n = (nx, ny, nz)
    out = np.zeros(pos.shape[1])
    w = []
    for d in range(3):
        u = shadow_grid_units(pos[d], n[d], L[d])
        p = np.arange(n[d])
        wd = np.zeros((pos.shape[1], n[d]))
        for img in (-1, 0, 1):
            wd += beta3(u[:, None] - (p[None, :] + img * n[d]))
        w.append(wd)
    out = np.einsum("ar,aq,ap,rqp->a", w[2], w[1], w[0], S)
    return out


def spline_of_modes_1d(kappa, u, n):
    """Spline interpolant of exp(i kappa h m) (h = L/n, kappa in units of 1/h
    so kappa*h is passed as kappa) at grid-unit positions u: the coefficients
    are fourier_multiplier(kappa) * exp(i kappa p); returns
    sum_p coeff_p beta3(u - p) over the four p that touch u."""
    base = np.floor(u)
    out = np.zeros(np.broadcast(u, kappa).shape, dtype=np.complex128)
    for off in (-1, 0, 1, 2):
        p = base + off
        out = out + np.exp(1j * kappa * p) * beta3(u - p)
    return out * fourier_multiplier(kappa)
