"""Pins of the oracle's SGS stress divergence (Sec. 2.1: Boussinesq closure of the deviatoric
SGS stress, tau_ij - tau_kk delta_ij / 3 = -2 nu_t S_ij; its divergence is the SGS part of
Eq. H_i) and of the way the substep adds it (Eq. onestar_exp), against mathematics that does
not use the oracle's own stress routine:

* with a uniform eddy viscosity c on a periodic grid, d_j(2 c S_ij) = c (L u_i + d_i(D u)),
  so for a discretely divergence-free field it is exactly c times the discrete Laplacian
  (written out here with index shifts);
* summation by parts: sum_faces u . d_j(2 nu_t S_ij) dV equals minus the staggered sum of
  2 nu_t S_ij S_ij over centres (diagonal) and edges (off-diagonal, with the edge viscosity
  of R18), for any positive nu_t field, so the term only removes energy;
* the predictor with a uniform eddy viscosity c equals the predictor with no SGS term and
  molecular viscosity nu + c (explicit viscous terms), or with viscosity c in the explicit
  part when all viscous terms are Crank-Nicolson (Eq. twostar_imp3d).
Planted mistakes each of these catches: a flipped or halved SGS term."""
import numpy as np
import pytest

from oracle import Case, Grid, ops
from oracle import substep as S
from oracle.case import ZBC_PERIODIC, SGS_SMAG


def _periodic_case(nx=8, ny=6, nz=10, nu=1e-3):
    return Case(nx, ny, nz, 1.3, 0.9, 1.7, zbc=ZBC_PERIODIC, nu=nu, sgs=SGS_SMAG)


def _roll(a, shift, axis):
    return np.roll(a, shift, axis=axis)


def _ghost_periodic(a):
    """(nz, ny, nx) interior -> (nz + 2, ny, nx) with periodic ghost planes."""
    return np.concatenate([a[-1:], a, a[:1]], axis=0)


def _solenoidal(g, seed):
    """u = curl A of a random vector potential on the staggered grid: A_x on the x-edges
    ((i+1/2) dx, (j+1) dy, zf_k), A_y on ((i+1) dx, (j+1/2) dy, zf_k), A_z on
    ((i+1) dx, (j+1) dy, zc_k).  The face differences commute, so D u = 0 exactly in exact
    arithmetic (uniform periodic grid)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shp = (g.nz, g.ny, g.nx)
    ax, ay, az = (rng.standard_normal(shp) for _ in range(3))
    dz = g.lz / g.nz
    # axis 0 = z (k), 1 = y (j), 2 = x (i); "a at k-1" is roll(+1)
    u = (az - _roll(az, 1, 1)) / g.dy - (ay - _roll(ay, 1, 0)) / dz
    v = (ax - _roll(ax, 1, 0)) / dz - (az - _roll(az, 1, 2)) / g.dx
    w = (ay - _roll(ay, 1, 2)) / g.dx - (ax - _roll(ax, 1, 1)) / g.dy
    return _ghost_periodic(u), _ghost_periodic(v), _ghost_periodic(w)


def _laplacian(g, a):
    """Seven-point Laplacian of an interior periodic array (uniform spacings)."""
    dz = g.lz / g.nz
    out = np.zeros_like(a)
    for axis, h in ((2, g.dx), (1, g.dy), (0, dz)):
        out += (_roll(a, -1, axis) - 2.0 * a + _roll(a, 1, axis)) / h ** 2
    return out


def test_solenoidal_construction_is_divergence_free():
    g = Grid(_periodic_case())
    u, v, w = _solenoidal(g, 1)
    d = ops.divergence(g, u, v, w)
    assert np.max(np.abs(d)) <= 1e-12 * np.max(np.abs(u))


def test_uniform_eddy_viscosity_gives_the_laplacian():
    g = Grid(_periodic_case())
    u, v, w = _solenoidal(g, 2)
    c = 0.37
    nut = np.full_like(u, c)
    fx, fy, fz = ops.sgs_divergence(g, u, v, w, nut)
    I = slice(1, g.nz + 1)
    for f, a in ((fx, u), (fy, v), (fz, w)):
        ref = c * _laplacian(g, a[I])
        assert np.max(np.abs(f - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_uniform_eddy_viscosity_on_a_compressible_field():
    """Without continuity the identity keeps the gradient of the divergence:
    d_j(2 c S_ij) = c (L u_i + d_i(D u)) at the u, v, w faces."""
    g = Grid(_periodic_case())
    rng = np.random.Generator(np.random.PCG64(3))
    u, v, w = (_ghost_periodic(rng.standard_normal((g.nz, g.ny, g.nx))) for _ in range(3))
    c = 0.21
    fx, fy, fz = ops.sgs_divergence(g, u, v, w, np.full_like(u, c))
    I = slice(1, g.nz + 1)
    dz = g.lz / g.nz
    uI, vI, wI = u[I], v[I], w[I]
    div = (uI - _roll(uI, 1, 2)) / g.dx + (vI - _roll(vI, 1, 1)) / g.dy + (wI - _roll(wI, 1, 0)) / dz
    grads = ((_roll(div, -1, 2) - div) / g.dx, (_roll(div, -1, 1) - div) / g.dy, (_roll(div, -1, 0) - div) / dz)
    for f, a, gd in ((fx, uI, grads[0]), (fy, vI, grads[1]), (fz, wI, grads[2])):
        ref = c * (_laplacian(g, a) + gd)
        assert np.max(np.abs(f - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("seed", [4, 5])
def test_sgs_work_is_minus_the_staggered_dissipation(seed):
    g = Grid(_periodic_case(nx=7, ny=6, nz=5))
    rng = np.random.Generator(np.random.PCG64(seed))
    shp = (g.nz, g.ny, g.nx)
    u, v, w = (_ghost_periodic(rng.standard_normal(shp)) for _ in range(3))
    nut = _ghost_periodic(0.1 + rng.random(shp))     # positive, far from uniform
    fx, fy, fz = ops.sgs_divergence(g, u, v, w, nut)
    I = slice(1, g.nz + 1)
    dz = g.lz / g.nz
    vol = g.dx * g.dy * dz
    work = np.sum(u[I] * fx + v[I] * fy + w[I] * fz) * vol
    uI, vI, wI, nI = u[I], v[I], w[I], nut[I]
    # strain at centres (diagonal) and at the three edge families (off-diagonal)
    s11 = (uI - _roll(uI, 1, 2)) / g.dx
    s22 = (vI - _roll(vI, 1, 1)) / g.dy
    s33 = (wI - _roll(wI, 1, 0)) / dz
    e12 = 0.5 * ((_roll(uI, -1, 1) - uI) / g.dy + (_roll(vI, -1, 2) - vI) / g.dx)   # (i+1, j+1, k)
    e13 = 0.5 * ((_roll(uI, -1, 0) - uI) / dz + (_roll(wI, -1, 2) - wI) / g.dx)     # (i+1, j, k+1/2)
    e23 = 0.5 * ((_roll(vI, -1, 0) - vI) / dz + (_roll(wI, -1, 1) - wI) / g.dy)     # (i, j+1, k+1/2)
    # R18: edge viscosity = mean of the four cell centres around the edge
    n12 = 0.25 * (nI + _roll(nI, -1, 2) + _roll(nI, -1, 1) + _roll(_roll(nI, -1, 1), -1, 2))
    n13 = 0.25 * (nI + _roll(nI, -1, 2) + _roll(nI, -1, 0) + _roll(_roll(nI, -1, 0), -1, 2))
    n23 = 0.25 * (nI + _roll(nI, -1, 1) + _roll(nI, -1, 0) + _roll(_roll(nI, -1, 0), -1, 1))
    diss = (np.sum(2.0 * nI * (s11 ** 2 + s22 ** 2 + s33 ** 2))
            + np.sum(4.0 * (n12 * e12 ** 2 + n13 * e13 ** 2 + n23 * e23 ** 2))) * vol
    assert diss > 0.0
    assert work < 0.0
    assert abs(work + diss) <= 1e-12 * diss


def _state_with_uniform_nut(case, g, c, seed):
    u, v, w = _solenoidal(g, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    p = _ghost_periodic(rng.standard_normal((g.nz, g.ny, g.nx)))
    rprev = tuple(rng.standard_normal((g.nz, g.ny, g.nx)) for _ in range(3))
    return S.State(u, v, w, p, nut=np.full_like(u, c), rprev=rprev)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_predictor_with_uniform_eddy_viscosity_equals_added_viscosity(k):
    """Eq. onestar_exp with nu_t = c everywhere equals the same substep with nu_t = 0 and
    molecular viscosity nu + c (explicit viscous terms): the SGS term enters the
    right-hand side with the sign and weight of the viscous term."""
    nu, c, dt = 2e-3, 0.05, 0.013
    case = _periodic_case(nu=nu)
    g = Grid(case)
    st = _state_with_uniform_nut(case, g, c, 6)
    ref_case = _periodic_case(nu=nu + c)
    st0 = st.copy()
    st0.nut = np.zeros_like(st.nut)
    a, ra = S.predictor(case, g, st, k, dt)
    b, rb = S.predictor(ref_case, g, st0, k, dt)
    for x, y in zip(ra, rb):
        assert np.max(np.abs(x - y)) <= 1e-11 * np.max(np.abs(y))
    for x, y in zip(a, b):
        assert np.max(np.abs(x - y)) <= 1e-12 * np.max(np.abs(y))


def test_explicit_part_with_all_viscous_terms_implicit():
    """Eq. twostar_imp3d: the explicit part H_i keeps advection and the SGS divergence; with
    nu_t = c it equals the explicit right-hand side of a case without SGS term whose molecular
    viscosity is c."""
    c = 0.08
    case = _periodic_case(nu=1e-3)
    case.implicit_3d = True
    g = Grid(case)
    st = _state_with_uniform_nut(case, g, c, 7)
    ref_case = _periodic_case(nu=c)
    st0 = st.copy()
    st0.nut = np.zeros_like(st.nut)
    ra = S.explicit_rhs(case, g, st)
    rb = S.explicit_rhs(ref_case, g, st0)
    for x, y in zip(ra, rb):
        assert np.max(np.abs(x - y)) <= 1e-11 * np.max(np.abs(y))
