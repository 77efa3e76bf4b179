"""Pins of the statistics oracle (Secs. 4.2 and 4.3 channel statistics, Eqs. eps_f and error):
closed forms for uniform and sinusoidal fields, the discrete laminar Poiseuille wall stress,
bulk velocity and skin friction on a uniform grid, exact batch-means cases, and the profile
error of a constant offset."""
import numpy as np
import pytest

from oracle import Case, Grid, stats as ST
from oracle.case import ZBC_NOSLIP, ZBC_PERIODIC
from oracle.substep import State


def _state(g, u, v, w):
    p = np.zeros_like(u)
    return State(u, v, w, p)


def test_uniform_state_means_and_zero_covariances():
    case = Case(8, 4, 6, 1.0, 1.0, 2.0, zbc=ZBC_NOSLIP)
    g = Grid(case)
    shape = (g.nz + 2, g.ny, g.nx)
    u = np.full(shape, 0.75)
    v = np.full(shape, -0.25)
    w = np.zeros(shape)
    acc = ST.Accumulator(g)
    for _ in range(3):
        acc.add(case, g, _state(g, u, v, w))
    prof, sc = ST.finalize(case, g, acc)
    assert np.all(prof["U"] == 0.75) and np.all(prof["V"] == -0.25) and np.all(prof["W"] == 0.0)
    for q in ("uu", "vv", "ww", "uv", "uw", "vw"):
        assert np.all(prof[q] == 0.0), q
    assert sc["samples"] == 3


def test_sinusoidal_fluctuations_closed_forms():
    """u' = a sin(2 pi x / Lx) on the u points, w' = b sin(2 pi x / Lx) on the w points,
    v' = c sin(2 pi y / Ly) on the v points: <u'u'> = a^2/2, <w'w'> = b^2/2, <v'v'> = c^2/2,
    <u'w'> on the (x, z) edge = a b cos(pi / nx) / 2 (the x-mean of w shrinks it), <u'v'> = 0,
    <v'w'> = 0."""
    nx, ny, nz = 12, 10, 8
    case = Case(nx, ny, nz, 1.0, 1.0, 1.0, zbc=ZBC_PERIODIC)
    g = Grid(case)
    a, b, c = 0.3, 0.2, 0.1
    xu = (np.arange(nx) + 1.0) / nx       # u at (i+1) dx
    xw = (np.arange(nx) + 0.5) / nx       # w at (i+1/2) dx
    yv = (np.arange(ny) + 1.0) / ny       # v at (j+1) dy
    shape = (nz + 2, ny, nx)
    U = 1.0 + 0.1 * np.arange(nz + 2)
    u = U[:, None, None] + a * np.sin(2 * np.pi * xu)[None, None, :] + np.zeros(shape)
    w = b * np.sin(2 * np.pi * xw)[None, None, :] + np.zeros(shape)
    v = c * np.sin(2 * np.pi * yv)[None, :, None] + np.zeros(shape)
    u[0], u[nz + 1] = u[nz], u[1]        # periodic ghosts
    v[0], v[nz + 1] = v[nz], v[1]
    w[0], w[nz + 1] = w[nz], w[1]
    acc = ST.Accumulator(g)
    acc.add(case, g, _state(g, u, v, w))
    prof, _ = ST.finalize(case, g, acc)
    assert np.allclose(prof["U"], U[1:nz + 1], rtol=0, atol=1e-14)
    assert np.allclose(prof["uu"], a * a / 2, rtol=0, atol=1e-14)
    assert np.allclose(prof["vv"], c * c / 2, rtol=0, atol=1e-14)
    assert np.allclose(prof["ww"], b * b / 2, rtol=0, atol=1e-14)
    assert np.allclose(prof["uw"], a * b * np.cos(np.pi / nx) / 2, rtol=0, atol=1e-14)
    assert np.allclose(prof["uv"], 0.0, rtol=0, atol=1e-14)
    assert np.allclose(prof["vw"], 0.0, rtol=0, atol=1e-14)


def test_poiseuille_wall_stress_bulk_velocity_and_skin_friction():
    """Discrete laminar profile u = 1.5 (1 - (z - 1)^2) at the centres of a uniform no-slip
    grid (dz = 2/nz): the ghost stress is 2 nu u_1 / dz = 3 nu (1 - dz/4), the midpoint-rule
    bulk velocity is 1 + dz^2/8, so C_f = 6 nu (1 - dz/4) / (1 + dz^2/8)^2 and
    Re_tau = sqrt(3 nu (1 - dz/4)) / nu (h = 1)."""
    nz, nu = 16, 1e-3
    case = Case(4, 4, nz, 1.0, 1.0, 2.0, zbc=ZBC_NOSLIP, nu=nu)
    g = Grid(case)
    dz = 2.0 / nz
    zc = g.zc
    u = np.zeros((nz + 2, 4, 4))
    u[1:nz + 1] = (1.5 * (1.0 - (zc[1:nz + 1] - 1.0) ** 2))[:, None, None]
    u[0], u[nz + 1] = -u[1], -u[nz]
    v = np.zeros_like(u)
    w = np.zeros_like(u)
    acc = ST.Accumulator(g)
    for _ in range(4):
        acc.add(case, g, _state(g, u, v, w))
    _, sc = ST.finalize(case, g, acc)
    tau = 3.0 * nu * (1.0 - dz / 4.0)
    ub = 1.0 + dz * dz / 8.0
    assert abs(sc["tau_w"] - tau) < 1e-15
    assert abs(sc["u_b"] - ub) < 1e-14
    assert abs(sc["c_f"] - 2.0 * tau / ub ** 2) < 1e-15
    assert abs(sc["re_tau"] - np.sqrt(tau) / nu) < 1e-10
    assert sc["c_f_sigma"] == 0.0 or np.isnan(sc["c_f_sigma"])


def test_batch_means_exact_cases():
    """Series constant within each of nb batches: sigma = std(batch values) / sqrt(nb);
    leading samples beyond nb * floor(n / nb) are dropped; a constant series gives 0."""
    vals = np.array([1.0, 3.0, 2.0, 6.0])
    x = np.repeat(vals, 5)
    assert abs(ST.batch_means_sigma(x, 4) - np.std(vals, ddof=1) / 2.0) < 1e-15
    x2 = np.concatenate([[100.0, -50.0], x])   # 22 samples, 4 batches of 5: first 2 dropped
    assert abs(ST.batch_means_sigma(x2, 4) - np.std(vals, ddof=1) / 2.0) < 1e-15
    assert ST.batch_means_sigma(np.full(40, 0.7), 8) == 0.0
    assert np.isnan(ST.batch_means_sigma(np.ones(3), 8))


@pytest.mark.parametrize("offset", [0.0, 0.05, -0.2])
def test_profile_error_constant_offset(offset):
    """Eq. error with phi = phi_ref + c and phi_ref = 1 on [0.1, 1]: sqrt(0.9 c^2) / 0.9,
    on any point set covering the interval (here a stretched one)."""
    z = np.sort(np.concatenate([[0.0, 1.3], np.random.default_rng(3).uniform(0.0, 1.3, 17)]))
    ref = np.ones_like(z)
    e = ST.eps_phi(z, ref + offset, ref, 0.1, 1.0)
    assert abs(e - np.sqrt(0.9 * offset ** 2) / 0.9) < 1e-14


def test_profile_error_linear_difference():
    """phi - phi_ref = z on [0.1, 1] with phi_ref = 2: integral of z^2 = (1 - 0.001)/3, of the
    reference = 1.8."""
    z = np.linspace(0.0, 1.0, 11)
    ref = np.full_like(z, 2.0)
    e = ST.eps_phi(z, ref + z, ref, 0.1, 1.0)
    assert abs(e - np.sqrt(0.999 / 3.0) / 1.8) < 1e-14


def test_eps_f():
    assert ST.eps_f(0.0060, 0.0050) == pytest.approx(0.2, abs=1e-15)


def test_duct_laminar_perimeter_stress_balances_the_driving_gradient():
    """R39: for the discrete laminar duct flow nu (L_yy + L_zz) u = -G (solved directly, no-slip)
    the wall fluxes telescope: the perimeter-mean wall stress times the perimeter equals
    G times the cross-section area, tau_w = G ly lz / (2 (ly + lz)), to roundoff; u_b is the
    area mean, so C_f = 2 tau_w / u_b^2."""
    from oracle.case import YBC_WALL
    from tests.test_oracle_duct import _laminar_duct
    G = 0.7
    case = Case(4, 8, 6, 1.0, 2.0, 1.5, zbc=ZBC_NOSLIP, ybc=YBC_WALL, beta=1.2, nu=0.05)
    g = Grid(case)
    prof = _laminar_duct(case, g, G)
    u = np.zeros((g.nz + 2, g.nys, g.nx))
    u[1:g.nz + 1, :g.ny] = prof[:, :, None]
    v, w = np.zeros_like(u), np.zeros_like(u)
    from oracle import bc
    bc.fill_velocity(case, g, u, v, w)
    acc = ST.Accumulator(g)
    for _ in range(3):
        acc.add(case, g, _state(g, u, v, w))
    prof_out, sc = ST.finalize(case, g, acc)
    tau = G * case.ly * case.lz / (2.0 * (case.ly + case.lz))
    assert abs(sc["tau_w"] - tau) < 1e-13 * tau
    dzf = g.dzf[1:g.nz + 1]
    ub = np.sum(prof * dzf[:, None]) / (g.ny * np.sum(dzf))
    assert abs(sc["u_b"] - ub) < 1e-14 * ub
    assert abs(sc["c_f"] - 2.0 * tau / ub ** 2) < 1e-13 * sc["c_f"]
    assert np.allclose(prof_out["U"], prof, rtol=0, atol=1e-14)
    for q in ("uu", "vv", "ww", "uv", "uw", "vw"):   # steady: no fluctuations (cancellation of U^2)
        assert np.max(np.abs(prof_out[q])) < 1e-14 * np.max(prof) ** 2, q


def test_duct_streamwise_fluctuation_closed_forms():
    """R39: u = U(k, j) + a sin(2 pi x / Lx), w = b sin(2 pi x / Lx) on their points:
    <u'u'> = a^2/2 and <w'w'> = b^2/2 on every line, <u'w'> = a b cos(pi / nx) / 2 on the
    interior (x, z) edges, and the cross-section means are the line means."""
    from oracle.case import YBC_WALL
    nx, ny, nz = 12, 6, 5
    case = Case(nx, ny, nz, 1.0, 2.0, 2.0, zbc=ZBC_NOSLIP, ybc=YBC_WALL)
    g = Grid(case)
    a, b = 0.3, 0.2
    xu = (np.arange(nx) + 1.0) / nx
    xw = (np.arange(nx) + 0.5) / nx
    rng = np.random.default_rng(4)
    Ucs = rng.uniform(0.5, 1.5, (nz, ny))
    u = np.zeros((nz + 2, g.nys, nx))
    w = np.zeros_like(u)
    u[1:nz + 1, :ny] = Ucs[:, :, None] + a * np.sin(2 * np.pi * xu)[None, None, :]
    w[1:nz, :ny] = b * np.sin(2 * np.pi * xw)[None, None, :]
    v = np.zeros_like(u)
    acc = ST.Accumulator(g)
    acc.add(case, g, _state(g, u, v, w))
    prof, _ = ST.finalize(case, g, acc)
    assert np.allclose(prof["U"], Ucs, rtol=0, atol=1e-14)
    assert np.allclose(prof["uu"], a * a / 2, rtol=0, atol=1e-14)
    assert np.allclose(prof["ww"][:nz - 1], b * b / 2, rtol=0, atol=1e-14)
    assert np.allclose(prof["ww"][nz - 1], 0.0, atol=1e-15)
    assert np.allclose(prof["uw"][:nz - 1], a * b * np.cos(np.pi / nx) / 2, rtol=0, atol=1e-14)
    assert np.allclose(prof["uv"], 0.0, atol=1e-15) and np.allclose(prof["vw"], 0.0, atol=1e-15)
