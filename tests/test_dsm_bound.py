"""The derived rounding bound of the dynamic model (tests/dsm_bound.py) against evaluations
whose differences it must cover: the oracle in float64 against the same oracle in x87
extended precision (64-bit significand, a stand-in for the exact values: one side's error
must stay within half the two-sided bound), the plain-loop re-derivation against the
vectorised oracle (two float64 orders: within the bound), and its own coefficient.  A
planted difference of a few bounds is reported as such."""
import numpy as np
import pytest

from oracle import Case, Grid, bc, sgs
from oracle.case import ZBC_PERIODIC, ZBC_NOSLIP, ZBC_WALLMODEL, SGS_DSM
from synth import random_state
from tests import dsm_bound
from tests.test_oracle_sgs import _bruteforce_cs, _ghosted

CASES = [
    ("periodic", dict(nx=12, ny=10, nz=8, lx=1.0, ly=1.3, lz=1.1, zbc=ZBC_PERIODIC)),
    ("noslip stretched", dict(nx=12, ny=10, nz=9, lx=1.0, ly=1.3, lz=2.0, zbc=ZBC_NOSLIP, beta=1.3)),
    ("wall model stretched", dict(nx=16, ny=8, nz=10, lx=2.0, ly=1.0, lz=2.0, zbc=ZBC_WALLMODEL, beta=1.5)),
    ("duct wall model", dict(nx=10, ny=8, nz=8, lx=2.0, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL, ybc=1)),
    ("duct noslip", dict(nx=10, ny=8, nz=6, lx=2.0, ly=2.0, lz=2.0, zbc=ZBC_NOSLIP, beta=1.1, ybc=1)),
]


def _state(cfg, seed=7):
    case = Case(cfg["nx"], cfg["ny"], cfg["nz"], cfg["lx"], cfg["ly"], cfg["lz"], zbc=cfg["zbc"],
                beta=cfg.get("beta", 0.0), nu=1e-3, sgs=SGS_DSM, ybc=cfg.get("ybc", 0))
    g = Grid(case)
    u, v, w, _ = random_state(case.nx, g.nys, case.nz, seed)
    if case.zbc != ZBC_PERIODIC:
        # a mean shear on top of the noise, so that some planes keep c_s > 0
        u[1:g.nz + 1] += 2.0 * np.linspace(0, 1, g.nz)[:, None, None]
    if g.ywalls:
        z = np.zeros((g.nys, g.nx))
        zy = np.zeros((g.nz + 2, g.nx))
        u, v, w = u.copy(), v.copy(), w.copy()
        bc.fill_velocity(case, g, u, v, w, tau=(z, z, z, z), tauy=(zy, zy, zy, zy))
    else:
        u, v, w = _ghosted(case, g, u, v, w)
    return case, g, u, v, w


@pytest.mark.parametrize("name,cfg", CASES, ids=[c[0] for c in CASES])
def test_bound_covers_extended_precision(name, cfg):
    case, g, u, v, w = _state(cfg)
    bound, dc, cs_b = dsm_bound.nut_difference_bound(case, g, u, v, w)
    nut64, cs64 = sgs.dynamic_smagorinsky(case, g, u, v, w)
    L = np.longdouble
    nutL, csL = sgs.dynamic_smagorinsky(case, g, u.astype(L), v.astype(L), w.astype(L))
    assert nutL.dtype == np.longdouble
    err = np.abs(nut64 - nutL.astype(np.float64))
    ratio = np.max(err / (0.5 * bound + 1e-300))
    assert np.all(err <= 0.5 * bound), ratio
    assert np.all(np.abs(cs64 - csL.astype(np.float64)) <= 0.5 * dc)
    # the value parts are the oracle's coefficient up to its own rounding
    assert np.all(np.abs(cs_b - cs64) <= dc)
    assert np.any(cs64 > 0)
    # not vacuous: the bound stays far below the values
    assert np.max(bound) <= 1e-10 * np.max(np.abs(nut64))


@pytest.mark.parametrize("zbc", [ZBC_PERIODIC, ZBC_NOSLIP, ZBC_WALLMODEL])
def test_bound_covers_plain_loops(zbc):
    """Two float64 summation orders: the plain loops (tests/test_oracle_sgs.py) and the
    vectorised oracle's coefficients differ by less than the coefficient bound."""
    case = Case(5, 4, 6, 1.0, 1.3, 2.0, zbc=zbc, beta=1.1 if zbc else 0.0, nu=1e-3, sgs=SGS_DSM)
    g = Grid(case)
    u, v, w, _ = random_state(5, 4, 6, 103 if zbc == ZBC_PERIODIC else 99)
    if zbc != ZBC_PERIODIC:
        u[1:7] += 2.0 * np.linspace(0, 1, 6)[:, None, None]
    u, v, w = _ghosted(case, g, u, v, w)
    _, dc, _ = dsm_bound.nut_difference_bound(case, g, u, v, w)
    cs, _, _, _ = sgs.dynamic_coefficient(case, g, u, v, w)
    ref, _, _ = _bruteforce_cs(case, g, u, v, w)
    assert np.all(np.abs(cs - ref) <= dc)


def test_planted_difference_exceeds_bound():
    """A perturbation of 4 bounds on one cell is not covered."""
    case, g, u, v, w = _state(CASES[2][1])
    bound, _, _ = dsm_bound.nut_difference_bound(case, g, u, v, w)
    nut, _ = sgs.dynamic_smagorinsky(case, g, u, v, w)
    other = nut.copy()
    k, j, i = np.unravel_index(np.argmax(nut), nut.shape)
    other[k, j, i] += 4.0 * bound[k, j, i]
    assert not np.all(np.abs(other - nut) <= bound)
