"""Pins of the oracle's grid and staggered operators against closed forms."""
import numpy as np
import pytest

from oracle import Case, Grid, ops, bc, poisson
from oracle.case import ZBC_PERIODIC, ZBC_NOSLIP
from oracle.grid import tanh_faces


def test_tanh_faces_endpoints_and_mirror():
    for nz, beta in ((96, 1.5), (17, 2.0), (8, 0.7)):
        zf = tanh_faces(nz, 2.0, beta)
        assert zf[0] == 0.0 and zf[nz] == 2.0
        for k in range(nz + 1):
            assert zf[nz - k] == 2.0 - zf[k]          # bitwise mirror symmetry
        assert np.all(np.diff(zf) > 0)
        d = np.diff(zf)
        assert d[0] < d[nz // 2]                      # clustered at the walls


def test_grid_metrics_consistency():
    g = Grid(Case(8, 6, 12, 2 * np.pi, np.pi, 2.0, zbc=ZBC_NOSLIP, beta=1.5))
    n = g.nz
    assert np.isclose(g.dzf[1:n + 1].sum(), 2.0, rtol=0, atol=1e-15)
    assert g.zc[0] == -g.zc[1]
    for k in range(1, n + 1):
        assert g.zf[k - 1] < g.zc[k] < g.zf[k]
    assert np.allclose(g.dzc[1:n], 0.5 * (g.dzf[1:n] + g.dzf[2:n + 1]), rtol=1e-14)


def _fields(g, fu, fv, fw):
    n = g.nz
    shape = (n + 2, g.ny, g.nx)
    xf = (np.arange(g.nx) + 1.0) * g.dx
    xc = (np.arange(g.nx) + 0.5) * g.dx
    yf = (np.arange(g.ny) + 1.0) * g.dy
    yc = (np.arange(g.ny) + 0.5) * g.dy
    Z, Y, X = np.meshgrid(g.zc, yc, xf, indexing="ij")
    u = fu(X, Y, Z)
    Z, Y, X = np.meshgrid(g.zc, yf, xc, indexing="ij")
    v = fv(X, Y, Z)
    Z, Y, X = np.meshgrid(np.concatenate([g.zf, [g.zf[-1] + g.dzf[-1]]]), yc, xc, indexing="ij")
    w = fw(X, Y, Z)
    assert u.shape == v.shape == w.shape == shape
    return u, v, w


def test_divergence_of_linear_w_is_one_on_stretched_grid():
    g = Grid(Case(4, 4, 10, 1.0, 1.0, 2.0, zbc=ZBC_NOSLIP, beta=1.8))
    zero = lambda X, Y, Z: 0.0 * X
    u, v, w = _fields(g, zero, zero, lambda X, Y, Z: Z.copy())
    d = ops.divergence(g, u, v, w)
    assert np.allclose(d, 1.0, rtol=0, atol=1e-13)


@pytest.mark.parametrize("l,m", [(1, 0), (3, 2), (4, 3)])
def test_dg_fourier_eigenvalues(l, m):
    """D(G phi) of a Fourier mode is lambda_x(l) + lambda_y(m) times the mode, with
    lambda = -(4/h^2) sin^2(pi l / n) (closed form of the periodic second difference)."""
    nx, ny, nz = 8, 6, 4
    case = Case(nx, ny, nz, 2.0, 1.5, 1.0, zbc=ZBC_PERIODIC)
    g = Grid(case)
    xc = (np.arange(nx) + 0.5) * g.dx
    yc = (np.arange(ny) + 0.5) * g.dy
    phi = np.zeros((nz + 2, ny, nx))
    phi[:] = np.cos(2 * np.pi * l * xc / g.lx)[None, None, :] * np.cos(2 * np.pi * m * yc / g.ly)[None, :, None]
    gx, gy, gz = ops.gradient(g, phi)
    u, v, w = np.zeros_like(phi), np.zeros_like(phi), np.zeros_like(phi)
    u[1:nz + 1], v[1:nz + 1], w[1:nz + 1] = gx, gy, gz
    bc.fill_velocity(case, g, u, v, w)
    d = ops.divergence(g, u, v, w)
    lam = -(4 / g.dx ** 2) * np.sin(np.pi * l / nx) ** 2 - (4 / g.dy ** 2) * np.sin(np.pi * m / ny) ** 2
    assert np.allclose(d, lam * phi[1:nz + 1], rtol=0, atol=1e-12 * abs(lam))


@pytest.mark.parametrize("q", [1, 2, 5])
def test_dg_neumann_cosine_eigenvalues(q):
    """Uniform walls: cos(pi q (k - 1/2)/nz) is an eigenvector of the zero-flux second
    difference with eigenvalue -(4/dz^2) sin^2(pi q / (2 nz))."""
    nz = 8
    case = Case(2, 2, nz, 1.0, 1.0, 2.0, zbc=ZBC_NOSLIP)
    g = Grid(case)
    k = np.arange(1, nz + 1)
    phi = np.zeros((nz + 2, 2, 2))
    phi[1:nz + 1] = np.cos(np.pi * q * (k - 0.5) / nz)[:, None, None]
    bc.fill_scalar(case, g, phi)
    lap = ops.lap_z_centre(g, phi)
    dz = g.dzf[1]
    lam = -(4 / dz ** 2) * np.sin(np.pi * q / (2 * nz)) ** 2
    assert np.allclose(lap, lam * phi[1:nz + 1], rtol=0, atol=1e-12 * abs(lam))
    # the Poisson rows used by the solver are the same operator
    a, b, c = poisson.z_coefficients(g)
    x = phi[1:nz + 1, 0, 0]
    y = b * x + c * np.append(x[1:], 0.0) + a * np.insert(x[:-1], 0, 0.0)
    assert np.allclose(y, lam * x, rtol=0, atol=1e-12 * abs(lam))


def test_gradient_of_quadratic_on_stretched_grid():
    """G p for p = z^2 at the w faces equals (zc_{k+1}^2 - zc_k^2)/dzc_k = zc_{k+1} + zc_k."""
    g = Grid(Case(3, 3, 9, 1.0, 1.0, 2.0, zbc=ZBC_NOSLIP, beta=1.2))
    p = np.zeros((g.nz + 2, 3, 3)) + (g.zc ** 2)[:, None, None]
    _, _, gz = ops.gradient(g, p)
    expect = (g.zc[2:g.nz + 2] + g.zc[1:g.nz + 1])[:, None, None]
    assert np.allclose(gz, expect, rtol=1e-13, atol=0)


def test_laplacian_of_quadratic_is_exact():
    """L_zz of z^2 at centres: each flux (zc_{k+1}^2 - zc_k^2)/dzc_k = zc_{k+1} + zc_k, so the
    operator gives (zc_{k+1} - zc_{k-1})/dzf_k, which is 2 on a uniform grid."""
    g = Grid(Case(2, 2, 7, 1.0, 1.0, 2.0, zbc=ZBC_NOSLIP, beta=1.0))
    a = np.zeros((g.nz + 2, 2, 2)) + (g.zc ** 2)[:, None, None]
    lap = ops.lap_z_centre(g, a)[:, 0, 0]
    n = g.nz
    # (zc_{k+1} + zc_k) - (zc_k + zc_{k-1}) over dzf_k
    expect = (g.zc[2:n + 2] - g.zc[0:n]) / g.dzf[1:n + 1]
    assert np.allclose(lap, expect, rtol=1e-13)


def test_uniform_translation_has_no_strain_or_advection():
    """A uniform velocity has zero strain and, with zero divergence, zero advection."""
    nx = ny = 8
    case = Case(nx, ny, 4, 2 * np.pi, 2 * np.pi, 1.0, zbc=ZBC_PERIODIC)
    g = Grid(case)
    zero = lambda X, Y, Z: 0.0 * X
    u, v, w = _fields(g, lambda X, Y, Z: 0.0 * X + 3.0, lambda X, Y, Z: 0.0 * X - 1.0, zero)
    s = ops.centre_strain(g, u, v, w)
    for comp in s:
        assert np.all(np.abs(comp) < 1e-14)
    adv = ops.advection(g, u, v, w)
    for a in adv:
        assert np.all(np.abs(a) < 1e-13)
