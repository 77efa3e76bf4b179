"""Pins of the oracle's log-law wall model (Eq. wm, Sec. 2.2)."""
import math

import numpy as np
import pytest

from oracle import Case, Grid, bc
from oracle.case import ZBC_WALLMODEL

KAPPA, B = 0.41, 5.2


def _bisect(U, h, nu, lo, hi):
    f = lambda x: x * (math.log(x * h / nu) / KAPPA + B) - U
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
        if hi - lo <= 1e-17 * hi:
            break
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("U,h,nu", [(1.0, 0.01, 5e-5), (0.3, 0.1, 1.6e-5), (2.0, 0.02, 1e-3),
                                    (1e-3, 0.05, 1e-3), (15.0, 0.1, 8e-6)])
def test_newton_equals_bisection(U, h, nu):
    """The root on the increasing branch is unique: bisection on [x_min, U + 1] (g(x_min) < 0
    and g(U + 1) > U) must agree with Newton to ~1e-15."""
    xmin = nu / h * math.exp(-KAPPA * B - 1.0)
    ref = _bisect(U, h, nu, xmin, U + 1.0 + 10 * nu / h)
    for guess in (0.0, ref * 0.5, ref * 1.3, ref * 10):
        x, it = bc.newton_utau(U, h, nu, KAPPA, B, guess)
        assert abs(x - ref) <= 4e-15 * ref, (guess, x, ref)


def test_zero_velocity_gives_zero_stress():
    x, it = bc.newton_utau(0.0, 0.01, 1e-4, KAPPA, B, 0.05)
    assert x == 0.0 and it == 0


def test_iterations_from_previous_step_guess():
    """Sec. 2.2: 3 to 7 Newton iterations reach 0.01 % from the previous step's value.
    A guess within a few per cent of the root (a time step's change) must converge to
    1e-4 relative in at most 7 iterations."""
    for U, h, nu in ((1.0, 0.05, 5e-5), (0.8, 0.1, 8e-6), (1.2, 0.02, 1.6e-5)):
        ref = _bisect(U, h, nu, nu / h * math.exp(-KAPPA * B - 1.0), U + 1.0)
        for rel in (0.9, 0.97, 1.03, 1.2):
            x, it = bc.newton_utau(U, h, nu, KAPPA, B, rel * ref, tol=1e-4)
            assert 1 <= it <= 7
            assert abs(x - ref) <= 1e-4 * ref


def test_array_newton_equals_scalar():
    rng = np.random.Generator(np.random.PCG64(4))
    U = rng.uniform(0.0, 2.0, 50)
    U[3] = 0.0
    guess = rng.uniform(0.0, 0.1, 50)
    xa, _ = bc.newton_utau_array(U, 0.03, 5e-5, KAPPA, B, guess)
    for i in range(50):
        xs, _ = bc.newton_utau(U[i], 0.03, 5e-5, KAPPA, B, guess[i])
        assert xa[i] == xs


def test_wall_stress_direction_and_log_law():
    """tau_x / tau_y follow the local velocity direction and u_tau satisfies the log law at
    the matching height; for a uniform wall-parallel velocity every face is identical."""
    case = Case(6, 4, 8, 1.0, 1.0, 2.0, zbc=ZBC_WALLMODEL, beta=1.5, nu=1e-4)
    g = Grid(case)
    u = np.zeros((10, 4, 6)) + 0.8
    v = np.zeros((10, 4, 6)) + 0.6
    tau, utau, _ = bc.wall_stress(case, g, u, v, None)
    h = g.zc[1]
    ut = utau["botx"][0, 0]
    assert abs(ut * (math.log(ut * h / case.nu) / KAPPA + B) - 1.0) < 1e-14
    assert np.allclose(tau[0], ut * ut * 0.8, rtol=1e-14)
    assert np.allclose(tau[1], ut * ut * 0.6, rtol=1e-14)
    assert np.allclose(tau[2], tau[0], rtol=1e-13)
