"""Shared helpers of the GPU parity tests: the same seeded inputs go to the CPU oracle and
to the HIP library, and fields are compared element by element."""
import sys

import numpy as np

import oracle
from oracle import substep as S
from synth import isotropic_field, channel_field, duct_field, random_state


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_pair(nx, ny, nz, lx, ly, lz, **kw):
    """(oracle Case, Grid, library config) for one problem."""
    from paper_2411_09364_amd import les
    precision = kw.pop("precision", 0)
    case = oracle.Case(nx, ny, nz, lx, ly, lz, **kw)
    g = oracle.Grid(case)
    cfg = les.make_config(nx, ny, nz, lx, ly, lz, zbc=case.zbc, beta=case.beta, nu=case.nu,
                          sgs=case.sgs, cs=case.cs,
                          implicit_z=2 if case.implicit_3d else int(case.implicit_z),
                          precision=precision, ubulk=case.ubulk, h_wm=case.h_wm,
                          kappa=case.kappa, bconst=case.bconst, ybc=case.ybc)
    return case, g, cfg


def initial_fields(case, g, seed, kind):
    if kind == "iso":
        assert case.nx == case.ny == case.nz
        return isotropic_field(case.nx, seed=seed, k0=4.0)
    if kind == "channel":
        return channel_field(case.nx, case.ny, case.nz, g.zc, seed=seed)
    if kind == "duct":
        return duct_field(case.nx, case.ny, case.nz, g.zc, case.ly, case.lz, seed=seed)
    u, v, w, _ = random_state(case.nx, g.nys, case.nz, seed)
    if case.walls:
        w[case.nz] = 0.0
    if case.ywalls:
        for a in (u, v, w):
            a[:, case.ny:] = 0.0
        v[:, case.ny - 1] = 0.0
    return u, v, w


def rel_err(a, b, sl):
    ref = np.max(np.abs(b[sl]))
    return np.max(np.abs(a[sl] - b[sl])) / (ref if ref > 0 else 1.0)


def mean_free(p, g):
    n = g.nz
    I = slice(1, n + 1)
    dzf = g.dzf[I]
    m = np.sum(p[I, :g.ny] * dzf[:, None, None]) / (np.sum(dzf) * g.nx * g.ny)
    q = p.copy()
    q[I] -= m
    return q


def round32(*arrs):
    return tuple(np.asarray(a, dtype=np.float32).astype(np.float64) for a in arrs)


UNIT_ROUNDOFF = 2.0 ** -53


def dsm_nut_check(case, g, st, nut, rel=1e-12):
    """Compare a dynamic-model nu_t with the oracle's cell by cell: the allowed difference is
    rel * max|nu_t| plus the derived rounding bound of two float64 evaluations of the model
    in different orders (tests/dsm_bound.py, from the oracle state's velocity).
    Returns (ok, worst ratio of difference to allowance, largest bound relative to
    max|nu_t|)."""
    from tests.dsm_bound import nut_difference_bound
    n = g.nz
    I = slice(1, n + 1)
    bound, _, _ = nut_difference_bound(case, g, st.u, st.v, st.w)
    J = slice(0, g.ny)
    ref = np.max(np.abs(st.nut[I, J]))
    diff = np.abs(nut[I, J] - st.nut[I, J])
    allow = rel * ref + bound[:, J]
    ratio = float(np.max(diff / allow))
    return ratio <= 1.0, ratio, float(np.max(bound[:, J]) / ref) if ref > 0 else 0.0


def poisson_condition(g):
    """Condition number lambda_max / lambda_min of the discrete Poisson operator D G of the
    grid (Sec. 2.2): lambda_max bounded by Gershgorin (4/dx^2 + 4/dy^2 + the largest z row
    sum), lambda_min the smallest nonzero magnitude among the first x and y modes (cosine in
    y for ducts) and the z operator's eigenvalues (Neumann at walls, periodic otherwise)."""
    n = g.nz
    lx = (2.0 - 2.0 * np.cos(2.0 * np.pi / g.nx)) / g.dx ** 2
    # first cosine mode with walls in y (square duct), first Fourier mode otherwise
    ly = (2.0 - 2.0 * np.cos((1.0 if g.ywalls else 2.0) * np.pi / g.ny)) / g.dy ** 2
    A = np.zeros((n, n))
    for k in range(1, n + 1):
        lo = 1.0 / (g.dzc[k - 1] * g.dzf[k])
        up = 1.0 / (g.dzc[k] * g.dzf[k])
        r = k - 1
        A[r, r] = -(lo + up)
        A[r, (r - 1) % n] += lo
        A[r, (r + 1) % n] += up
    if not g.periodic_z:
        A[0, n - 1] = A[n - 1, 0] = 0.0
        A[0, 0] += 1.0 / (g.dzc[0] * g.dzf[1])
        A[n - 1, n - 1] += 1.0 / (g.dzc[n] * g.dzf[n])
    ev = np.abs(np.linalg.eigvals(A))
    lz = np.min(ev[ev > 1e-9 * np.max(ev)])
    lmax = 4.0 / g.dx ** 2 + 4.0 / g.dy ** 2 + np.max(np.sum(np.abs(A), axis=1))
    return lmax / min(lx, ly, lz)


def pressure_tolerance(g):
    """FP64 tolerance of the mean-free pressure: the Poisson solve amplifies rounding by up to
    the operator's condition number, so max(1e-12, 4 eps kappa)."""
    return max(1e-12, 4.0 * UNIT_ROUNDOFF * 2.0 * poisson_condition(g))
