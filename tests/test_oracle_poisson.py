"""Pins of the oracle's Poisson solver: manufactured solutions (exact discrete operator)
and a dense brute-force least-squares solve on tiny grids."""
import numpy as np
import pytest

from oracle import Case, Grid, ops, bc, poisson
from oracle.case import ZBC_PERIODIC, ZBC_NOSLIP


def _dg(case, g, phi_int):
    """Apply D(G .) with the solver's boundary conditions to interior values."""
    n = g.nz
    phi = np.zeros((n + 2, g.ny, g.nx))
    phi[1:n + 1] = phi_int
    bc.fill_scalar(case, g, phi)
    gx, gy, gz = ops.gradient(g, phi)
    u, v, w = np.zeros_like(phi), np.zeros_like(phi), np.zeros_like(phi)
    u[1:n + 1], v[1:n + 1], w[1:n + 1] = gx, gy, gz
    if case.zperiodic:
        bc.fill_velocity(case, g, u, v, w)
    else:
        w[0] = w[n] = 0.0
    return ops.divergence(g, u, v, w)


def _weighted_mean(g, phi):
    dzf = g.dzf[1:g.nz + 1]
    return np.sum(phi * dzf[:, None, None]) / (np.sum(dzf) * g.nx * g.ny)


CASES = [
    Case(16, 12, 10, 2 * np.pi, np.pi, 2.0, zbc=ZBC_NOSLIP, beta=1.5),
    Case(8, 6, 7, 1.0, 2.0, 2.0, zbc=ZBC_NOSLIP, beta=0.0),
    Case(8, 8, 8, 2 * np.pi, 2 * np.pi, 2 * np.pi, zbc=ZBC_PERIODIC),
    Case(12, 6, 10, 3.0, 1.0, 2.0, zbc=ZBC_PERIODIC),
]


@pytest.mark.parametrize("case", CASES)
def test_manufactured_solution(case):
    g = Grid(case)
    rng = np.random.Generator(np.random.PCG64(7))
    phi = rng.standard_normal((g.nz, g.ny, g.nx))
    phi -= _weighted_mean(g, phi)
    f = _dg(case, g, phi)
    sol = poisson.solve(g, f)
    assert np.max(np.abs(sol - phi)) <= 1e-12 * np.max(np.abs(phi)) * 10
    # residual of the discrete equation
    res = _dg(case, g, sol) - f
    assert np.max(np.abs(res)) <= 1e-11 * np.max(np.abs(f))


@pytest.mark.parametrize("case", [Case(6, 4, 5, 1.0, 1.0, 2.0, zbc=ZBC_NOSLIP, beta=1.3),
                                  Case(4, 4, 4, 1.0, 1.0, 1.0, zbc=ZBC_PERIODIC)])
def test_dense_bruteforce(case):
    """Assemble D(G .) column by column from unit vectors and solve with lstsq; the
    minimum-norm solution, shifted to zero weighted mean, must equal the FFT/Thomas one."""
    g = Grid(case)
    N = g.nz * g.ny * g.nx
    A = np.zeros((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        A[:, c] = _dg(case, g, e.reshape(g.nz, g.ny, g.nx)).ravel()
    rng = np.random.Generator(np.random.PCG64(3))
    phi = rng.standard_normal(N)
    f = A @ phi                                     # compatible right-hand side
    x = np.linalg.lstsq(A, f, rcond=None)[0].reshape(g.nz, g.ny, g.nx)
    x -= _weighted_mean(g, x)
    sol = poisson.solve(g, f.reshape(g.nz, g.ny, g.nx))
    assert np.max(np.abs(sol - x)) <= 1e-11 * np.max(np.abs(x))


def test_zero_mode_mean_removed():
    case = CASES[0]
    g = Grid(case)
    rng = np.random.Generator(np.random.PCG64(11))
    phi = rng.standard_normal((g.nz, g.ny, g.nx)) + 5.0
    sol = poisson.solve(g, _dg(case, g, phi))
    assert abs(_weighted_mean(g, sol)) < 1e-13
    assert np.max(np.abs(sol - (phi - _weighted_mean(g, phi)))) < 1e-11


def test_thomas_matches_dense_solve():
    rng = np.random.Generator(np.random.PCG64(5))
    n = 9
    a = rng.uniform(0.5, 1, n)
    c = rng.uniform(0.5, 1, n)
    b = -(a + c) - rng.uniform(0.1, 1, n)
    d = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    M = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    assert np.allclose(poisson.thomas(a, b, c, d), np.linalg.solve(M, d), rtol=1e-13, atol=1e-14)
