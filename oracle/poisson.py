"""Eigenfunction-expansion Poisson solver (Sec. 2.2 after Eq. p_update_imp1d: Fourier
transforms in the periodic directions, the Thomas algorithm along the non-uniform one;
Eq. poi).  Test infrastructure only.

Solves D(G phi) = f for phi at cell centres, where D and G are the staggered divergence
and gradient of ops.py with G.n = 0 on walls (Neumann) or periodic z.  The discrete
eigenvalues of the periodic second difference are
    lambda_x(l) = -(4/dx^2) sin^2(pi l / nx),  lambda_y(m) likewise.
Normalisation (R20): forward transform unscaled, inverse scaled by 1/N (numpy.fft).

With walls in y (square duct, Sec. 4.4) y is a Neumann direction like wall-bounded z: the
eigenvectors of its second difference with zero flux through both walls are the cosines
cos(pi m (j + 1/2) / ny), m = 0..ny-1, with eigenvalues -(4/dy^2) sin^2(pi m / (2 ny)); the
expansion is written out with that matrix (R37).
"""
import numpy as np


def eigenvalues(n, h):
    return np.array([-(4.0 / h ** 2) * np.sin(np.pi * l / n) ** 2 for l in range(n)])


def neumann_eigenvalues(n, h):
    """Eigenvalues of the cell-centred second difference with zero flux at both ends."""
    return np.array([-(4.0 / h ** 2) * np.sin(np.pi * m / (2.0 * n)) ** 2 for m in range(n)])


def cosine_basis(n):
    """C[m, j] = cos(pi m (j + 1/2) / n): the eigenvectors of the Neumann second difference
    (orthogonal; squared norms n for m = 0 and n / 2 otherwise)."""
    return np.array([[np.cos(np.pi * m * (j + 0.5) / n) for j in range(n)] for m in range(n)])


def z_coefficients(g):
    """Tridiagonal rows of the z part of D G for interior planes k = 1..nz:
    a_k phi_{k-1} + b_k phi_k + c_k phi_{k+1} with a_k = 1/(dzc_{k-1} dzf_k),
    c_k = 1/(dzc_k dzf_k), b_k = -(a_k + c_k); at the walls the flux through the wall
    vanishes, so a_1 and c_nz are dropped (zero Neumann)."""
    n = g.nz
    a = np.zeros(n)
    c = np.zeros(n)
    for k in range(1, n + 1):
        a[k - 1] = 1.0 / (g.dzc[k - 1] * g.dzf[k])
        c[k - 1] = 1.0 / (g.dzc[k] * g.dzf[k])
    if not g.periodic_z:
        a[0] = 0.0
        c[n - 1] = 0.0
    b = -(a + c)
    return a, b, c


def thomas(a, b, c, d):
    """Plain Thomas algorithm for one tridiagonal system (complex right-hand side)."""
    n = len(d)
    cp = np.zeros(n, dtype=np.complex128)
    dp = np.zeros(n, dtype=np.complex128)
    cp[0] = c[0] / b[0]
    dp[0] = d[0] / b[0]
    for k in range(1, n):
        m = b[k] - a[k] * cp[k - 1]
        cp[k] = c[k] / m
        dp[k] = (d[k] - a[k] * dp[k - 1]) / m
    x = np.zeros(n, dtype=np.complex128)
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def thomas_columns(a, b, c, lam, d):
    """Thomas algorithm applied independently to every column (m, l) of d[k, m, l], the
    diagonal of column (m, l) being b_k + lam[m, l]; the same steps as thomas().  The
    (0, 0) column is left to the caller (its system is singular)."""
    n = d.shape[0]
    cp = np.zeros(d.shape)
    dp = np.zeros(d.shape, dtype=np.complex128)
    bb = b[0] + lam
    bb = np.where(bb == 0.0, 1.0, bb)
    cp[0] = c[0] / bb
    dp[0] = d[0] / bb
    for k in range(1, n):
        m = b[k] + lam - a[k] * cp[k - 1]
        m = np.where(m == 0.0, 1.0, m)
        cp[k] = c[k] / m
        dp[k] = (d[k] - a[k] * dp[k - 1]) / m
    x = np.zeros(d.shape, dtype=np.complex128)
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def solve(g, f):
    """phi with D(G phi) = f.  f and the result have shape (nz, ny, nx) (interior planes).

    Wall-bounded z: 2-D FFT over (y, x), then for every wavenumber pair (l, m) the
    tridiagonal system (A_z + lambda_x(l) + lambda_y(m)) phi_hat = f_hat by Thomas.
    The (0, 0) system is singular (constant null space); R19: its last unknown is pinned
    to zero, the first nz - 1 rows are solved (the last row holds automatically when
    sum_k f_hat dzf_k = 0), and the dzf-weighted mean of phi is then removed.
    Periodic z: 3-D FFT and division by lambda_x + lambda_y + lambda_z, with the
    (0, 0, 0) mode set to zero."""
    if getattr(g, "ywalls", False):
        return _solve_duct(g, f)
    nz, ny, nx = f.shape
    lx = eigenvalues(nx, g.dx)
    ly = eigenvalues(ny, g.dy)
    if g.periodic_z:
        lz = eigenvalues(nz, g.dzf[1])
        fh = np.fft.fftn(f)
        den = lz[:, None, None] + ly[None, :, None] + lx[None, None, :]
        den[0, 0, 0] = 1.0
        ph = fh / den
        ph[0, 0, 0] = 0.0
        return np.real(np.fft.ifftn(ph))
    a, b, c = z_coefficients(g)
    fh = np.fft.fft2(f, axes=(1, 2))
    lam = ly[:, None] + lx[None, :]                 # (ny, nx): lambda_x(l) + lambda_y(m)
    ph = thomas_columns(a, b, c, lam, fh)
    x = np.zeros(nz, dtype=np.complex128)
    x[:nz - 1] = thomas(a[:nz - 1], b[:nz - 1], c[:nz - 1], fh[:nz - 1, 0, 0])
    ph[:, 0, 0] = x
    phi = np.real(np.fft.ifft2(ph, axes=(1, 2)))
    dzf = g.dzf[1:nz + 1]
    mean = np.sum(phi * dzf[:, None, None]) / (np.sum(dzf) * nx * ny)
    return phi - mean


def _solve_duct(g, f):
    """Walls in y and z (R37): FFT in x, cosine expansion in y, then for every pair (l, m)
    the z system (A_z + lambda_x(l) + lambda_y(m)) phi_hat = f_hat by Thomas, the singular
    (0, 0) system pinned as in solve(), the dzf-weighted mean removed.  f has the stored
    rows (nz, ny + 2, nx); only rows 0..ny-1 are read, and the result's ghost rows are 0."""
    nz, nx, ny = g.nz, g.nx, g.ny
    fi = f[:, :ny, :]
    C = cosine_basis(ny)
    norm = np.array([1.0 / ny] + [2.0 / ny] * (ny - 1))       # inverse of the squared norms
    fx = np.fft.fft(fi, axis=2)
    fh = np.einsum("mj,kjl->kml", C, fx)
    lam = neumann_eigenvalues(ny, g.dy)[:, None] + eigenvalues(nx, g.dx)[None, :]
    a, b, c = z_coefficients(g)
    ph = thomas_columns(a, b, c, lam, fh)
    x = np.zeros(nz, dtype=np.complex128)
    x[:nz - 1] = thomas(a[:nz - 1], b[:nz - 1], c[:nz - 1], fh[:nz - 1, 0, 0])
    ph[:, 0, 0] = x
    py = np.einsum("mj,kml->kjl", C * norm[:, None], ph)
    phi_i = np.real(np.fft.ifft(py, axis=2))
    dzf = g.dzf[1:nz + 1]
    mean = np.sum(phi_i * dzf[:, None, None]) / (np.sum(dzf) * nx * ny)
    out = np.zeros((nz, g.nys, nx))
    out[:, :ny] = phi_i - mean
    return out
