"""Pins of the oracle's RK3 substep (Alg. 1) against closed forms and exact invariants."""
import numpy as np
import pytest

from oracle import Case, Grid, ops, substep as S
from oracle.case import ZBC_PERIODIC, ZBC_NOSLIP, ZBC_WALLMODEL, SGS_NONE, SGS_SMAG, SGS_DSM
from synth import taylor_green_field, isotropic_field, channel_field, random_state


def _step(case, g, st, dt):
    for k in range(3):
        st = S.substep(case, g, st, k, dt)
    return st


def test_rk3_coefficients():
    """Sec. 2.2: gamma = alpha + beta = (8/15, 2/15, 1/3) and sum(gamma) = 1."""
    assert np.allclose(S.GAMMA, (8 / 15, 2 / 15, 1 / 3), rtol=0, atol=1e-16)
    assert abs(sum(S.GAMMA) - 1.0) < 1e-15


@pytest.mark.parametrize("n,nu,dt", [(16, 0.05, 0.05), (8, 0.3, 0.02)])
def test_taylor_green_viscous_amplification(n, nu, dt):
    """Advection off: u = eps sin x cos y is discretely divergence-free and an eigenmode of
    the viscous operator with lambda = -(8/dx^2) sin^2(dx/2); one full RK3 step multiplies
    it by R(z) = 1 + z + z^2/2 + z^3/6, z = nu lambda dt (derived from alpha, beta)."""
    case = Case(n, n, 4, 2 * np.pi, 2 * np.pi, 2.0, zbc=ZBC_PERIODIC, nu=nu, advection=False)
    g = Grid(case)
    u, v, w = taylor_green_field(n, 4, 1.0)
    st = S.initial_state(case, g, u, v, w)
    u0 = st.u.copy()
    st = _step(case, g, st, dt)
    lam = -(8.0 / g.dx ** 2) * np.sin(g.dx / 2) ** 2
    z = nu * lam * dt
    R = 1 + z + z * z / 2 + z ** 3 / 6
    assert np.max(np.abs(st.u[1:5] - R * u0[1:5])) < 1e-13
    assert np.max(np.abs(st.p)) < 1e-12


def test_taylor_green_decay_with_advection_second_order():
    """Finite amplitude: the decay of the kinetic energy follows exp(-4 nu t) with an error
    that falls by about 4x per grid doubling (second order in space)."""
    nu, T = 0.05, 0.4
    errs = []
    for n in (16, 32):
        case = Case(n, n, 2, 2 * np.pi, 2 * np.pi, 1.0, zbc=ZBC_PERIODIC, nu=nu)
        g = Grid(case)
        u, v, w = taylor_green_field(n, 2, 1.0)
        st = S.initial_state(case, g, u, v, w)
        e0 = np.mean(st.u[1:3] ** 2 + st.v[1:3] ** 2)
        steps = 40
        for _ in range(steps):
            st = _step(case, g, st, T / steps)
        e = np.mean(st.u[1:3] ** 2 + st.v[1:3] ** 2)
        errs.append(abs(e / e0 - np.exp(-4 * nu * T)))
    assert errs[1] < errs[0] / 3.0


def test_cn_z_eigen_ratio():
    """CN in z (Eqs. twostar_imp1d, onestar_imp1d): for a discrete eigenvector of the
    no-slip L_zz (found with numpy.linalg.eig on the assembled matrix), each substep
    multiplies the profile by (1 + gamma z/2)/(1 - gamma z/2), z = nu mu dt."""
    nz = 10
    case = Case(4, 4, nz, 1.0, 1.0, 2.0, zbc=ZBC_NOSLIP, beta=1.3, nu=0.02, implicit_z=True)
    g = Grid(case)
    A = np.zeros((nz, nz))
    for c in range(nz):
        a = np.zeros((nz + 2, 1, 1))
        a[c + 1] = 1.0
        a[0], a[nz + 1] = -a[1], -a[nz]
        A[:, c] = S.ops.lap_z_centre(g, a)[:, 0, 0]
    mu, vec = np.linalg.eig(A)
    q = np.argsort(np.abs(mu))[2]
    prof = np.real(vec[:, q])
    u = np.zeros((nz + 2, 4, 4))
    u[1:nz + 1] = prof[:, None, None]
    st = S.initial_state(case, g, u, np.zeros_like(u), np.zeros_like(u))
    dt = 0.7
    ratio = 1.0
    for k in range(3):
        st = S.substep(case, g, st, k, dt)
        z = case.nu * np.real(mu[q]) * dt
        ratio *= (1 + S.GAMMA[k] * z / 2) / (1 - S.GAMMA[k] * z / 2)
        assert np.allclose(st.u[1:nz + 1], ratio * u[1:nz + 1], rtol=0, atol=1e-13)


@pytest.mark.parametrize("zbc,implicit,model", [(ZBC_PERIODIC, False, SGS_SMAG),
                                                (ZBC_NOSLIP, True, SGS_SMAG),
                                                (ZBC_WALLMODEL, True, SGS_DSM),
                                                (ZBC_WALLMODEL, False, SGS_DSM)])
def test_divergence_free_and_bulk_after_substep(zbc, implicit, model):
    """Eq. correc makes D u = 0 up to roundoff: max|D u| <= 1e-13 max|u| / min spacing;
    the flow-rate shift keeps <u> = U_b to roundoff."""
    nx, ny, nz = 16, 8, 12
    per = zbc == ZBC_PERIODIC
    case = Case(nx, ny, nz, 2 * np.pi, np.pi, 2.0, zbc=zbc, beta=0.0 if per else 1.5,
                nu=1e-3 if per else 5e-5, sgs=model, cs=0.17, implicit_z=implicit,
                ubulk=0.0 if per else 1.0)
    g = Grid(case)
    if per:
        u, v, w, _ = random_state(nx, ny, nz, 3)
    else:
        u, v, w = channel_field(nx, ny, nz, g.zc, seed=2)
    st = S.initial_state(case, g, u, v, w)
    dt = 0.2 * S.time_step(case, g, st)
    for k in range(3):
        st = S.substep(case, g, st, k, dt)
        d = ops.divergence(g, st.u, st.v, st.w)
        hmin = min(g.dx, g.dy, np.min(g.dzf[1:nz + 1]))
        umax = max(np.abs(st.u).max(), np.abs(st.v).max(), np.abs(st.w).max())
        assert np.max(np.abs(d)) <= 1e-13 * umax / hmin
        if not per:
            assert abs(S.bulk_velocity(g, st.u) - 1.0) < 1e-14
            assert np.all(st.w[0] == 0) and np.all(st.w[nz] == 0)


def test_inviscid_energy_error_is_fourth_order_in_dt():
    """With nu = nu_t = 0 the divergence-form advection conserves energy on a uniform
    periodic grid when D u = 0 (Sec. 1: energy preserving in the inviscid limit); the only
    error left is the RK3 one, O(dt^4) per step: halving dt cuts it by ~16x."""
    n = 12
    case = Case(n, n, n, 2 * np.pi, 2 * np.pi, 2 * np.pi, zbc=ZBC_PERIODIC, nu=0.0)
    g = Grid(case)
    u, v, w = isotropic_field(n, seed=5, k0=2.0)
    st0 = S.initial_state(case, g, u, v, w)
    st0 = S.substep(case, g, st0, 0, 1e-6)          # project to discrete divergence-free
    st0.p[:] = 0.0
    st0.rprev = None
    I = slice(1, n + 1)
    # Spatial pin: sum u . C(u) = 0 exactly for the projected field
    ax, ay, az = ops.advection(g, st0.u, st0.v, st0.w)
    dot = np.sum(st0.u[I] * ax) + np.sum(st0.v[I] * ay) + np.sum(st0.w[I] * az)
    assert abs(dot) < 1e-12 * np.sum(st0.u[I] ** 2)
    E = lambda st: np.sum(st.u[I] ** 2 + st.v[I] ** 2 + st.w[I] ** 2)
    errs = []
    for dt in (0.08, 0.04):
        st = _step(case, g, st0.copy(), dt)
        errs.append(abs(E(st) - E(st0)) / E(st0))
    assert 10.0 < errs[0] / errs[1] < 24.0


@pytest.mark.parametrize("implicit", [True, False])
def test_poiseuille_discrete_steady_state(implicit):
    """Laminar channel with constant flow rate and no model: the solution of the 1-D discrete
    problem nu L_zz U = -f, sum(U dzf) = U_b lz (solved directly as a bordered linear system)
    is a fixed point of the RK3 substep (explicit and CN in z), and it matches the parabola
    1.5 U_b (1 - (z-1)^2) to O(dz^2)."""
    nz = 16
    case = Case(4, 4, nz, 1.0, 1.0, 2.0, zbc=ZBC_NOSLIP, beta=1.2, nu=0.5, sgs=SGS_NONE,
                implicit_z=implicit, ubulk=1.0)
    g = Grid(case)
    A = np.zeros((nz + 1, nz + 1))
    for c in range(nz):
        a = np.zeros((nz + 2, 1, 1))
        a[c + 1] = 1.0
        a[0], a[nz + 1] = -a[1], -a[nz]
        A[:nz, c] = case.nu * S.ops.lap_z_centre(g, a)[:, 0, 0]
    A[:nz, nz] = 1.0
    A[nz, :nz] = g.dzf[1:nz + 1]
    rhs = np.zeros(nz + 1)
    rhs[nz] = 1.0 * 2.0
    sol = np.linalg.solve(A, rhs)[:nz]
    u = np.zeros((nz + 2, 4, 4))
    u[1:nz + 1] = sol[:, None, None]
    st = S.initial_state(case, g, u, np.zeros_like(u), np.zeros_like(u))
    dt = 0.5 * S.time_step(case, g, st)
    for _ in range(5):
        st = _step(case, g, st, dt)
    assert np.max(np.abs(st.u[1:nz + 1] - sol[:, None, None])) < 1e-12
    assert np.max(np.abs(st.v)) < 1e-13 and np.max(np.abs(st.w)) < 1e-13
    z = g.zc[1:nz + 1]
    assert np.max(np.abs(sol - 1.5 * (1 - (z - 1) ** 2))) < 0.05
    # a perturbed profile is not a fixed point (the check above has teeth)
    u2 = u.copy()
    u2[3] += 1e-3
    st2 = _step(case, g, S.initial_state(case, g, u2, np.zeros_like(u), np.zeros_like(u)), dt)
    assert np.max(np.abs(st2.u[1:nz + 1] - u2[1:nz + 1])) > 1e-6


def test_time_step_limits():
    n = 8
    case = Case(n, n, n, 2 * np.pi, 2 * np.pi, 2 * np.pi, zbc=ZBC_PERIODIC, nu=1e-3, sgs=SGS_SMAG)
    g = Grid(case)
    u = np.zeros((n + 2, n, n)) + 2.0
    st = S.initial_state(case, g, u, np.zeros_like(u), np.zeros_like(u))
    assert abs(S.time_step(case, g, st, cfl=0.5) - 0.5 * g.dx / 2.0) < 1e-15
    case2 = Case(n, n, n, 2 * np.pi, 2 * np.pi, 2 * np.pi, zbc=ZBC_PERIODIC, nu=10.0)
    st2 = S.initial_state(case2, g, np.zeros_like(u), np.zeros_like(u), np.zeros_like(u))
    assert abs(S.time_step(case2, g, st2) - 0.95 * 2.51 / (4 * 10.0 * 3 / g.dx ** 2)) < 1e-15


@pytest.mark.parametrize("comp,zbc", [(0, ZBC_NOSLIP), (1, ZBC_NOSLIP), (2, ZBC_PERIODIC)])
def test_cn_3d_eigen_ratio(comp, zbc):
    """CN in all directions (Eqs. twostar_imp3d, onestar_imp3d): a divergence-free mode that
    is a discrete eigenfunction of the full viscous operator (Fourier in the periodic
    directions, an eigenvector of the no-slip L_zz found with numpy.linalg.eig) is multiplied
    by (1 + gamma z/2)/(1 - gamma z/2) per substep, z = nu (lambda_x + lambda_y + mu) dt.
    u varies in y and z, v in x and z (both divergence-free), w in x and y with periodic z."""
    nx, ny, nz = 8, 6, 10
    per = zbc == ZBC_PERIODIC
    case = Case(nx, ny, nz, 1.0, 1.5, 2.0, zbc=zbc, beta=0.0 if per else 1.3, nu=0.02,
                implicit_3d=True, advection=False)
    g = Grid(case)
    if per:
        prof, mu = np.ones(nz), 0.0
    else:
        A = np.zeros((nz, nz))
        for c in range(nz):
            a = np.zeros((nz + 2, 1, 1))
            a[c + 1] = 1.0
            a[0], a[nz + 1] = -a[1], -a[nz]
            A[:, c] = S.ops.lap_z_centre(g, a)[:, 0, 0]
        ev, vec = np.linalg.eig(A)
        q = np.argsort(np.abs(ev))[1]
        prof, mu = np.real(vec[:, q]), float(np.real(ev[q]))
    x = (np.arange(nx) + (1.0 if comp == 0 else 0.5)) * g.dx
    y = (np.arange(ny) + (1.0 if comp == 1 else 0.5)) * g.dy
    lam = 0.0
    shape = (nz + 2, ny, nx)
    fld = np.zeros(shape)
    if comp == 0:     # u(y, z)
        fld[1:nz + 1] = prof[:, None, None] * np.cos(2 * np.pi * 2 * y / case.ly)[None, :, None]
        lam = -(4 / g.dy ** 2) * np.sin(np.pi * 2 / ny) ** 2
    elif comp == 1:   # v(x, z)
        fld[1:nz + 1] = prof[:, None, None] * np.sin(2 * np.pi * 3 * x / case.lx)[None, None, :]
        lam = -(4 / g.dx ** 2) * np.sin(np.pi * 3 / nx) ** 2
    else:             # w(x, y), constant in periodic z
        fld[1:nz + 1] = (np.cos(2 * np.pi * x / case.lx)[None, None, :] * np.sin(2 * np.pi * y / case.ly)[None, :, None])
        lam = -(4 / g.dx ** 2) * np.sin(np.pi / nx) ** 2 - (4 / g.dy ** 2) * np.sin(np.pi / ny) ** 2
    vel = [np.zeros(shape), np.zeros(shape), np.zeros(shape)]
    vel[comp] = fld
    st = S.initial_state(case, g, *vel)
    dt = 0.9
    ratio = 1.0
    for k in range(3):
        st = S.substep(case, g, st, k, dt)
        z = case.nu * (lam + mu) * dt
        ratio *= (1 + S.GAMMA[k] * z / 2) / (1 - S.GAMMA[k] * z / 2)
        got = (st.u, st.v, st.w)[comp]
        assert np.allclose(got[1:nz + 1], ratio * fld[1:nz + 1], rtol=0, atol=1e-13)
        for other in range(3):
            if other != comp:
                assert np.max(np.abs((st.u, st.v, st.w)[other][1:nz + 1])) < 1e-14


def test_cn_3d_reduces_to_cn_z_for_z_profiles():
    """With no variation in x and y only the (0, 0) Fourier mode carries the field, and the
    fully implicit scheme takes the same steps as CN in z (to roundoff) on a wall-modelled
    channel profile with the dynamic model."""
    nz = 12
    kw = dict(zbc=ZBC_WALLMODEL, beta=1.4, nu=5e-4, sgs=SGS_DSM, ubulk=1.0)
    c1 = Case(8, 4, nz, 2.0, 1.0, 2.0, implicit_z=True, **kw)
    c3 = Case(8, 4, nz, 2.0, 1.0, 2.0, implicit_3d=True, **kw)
    g = Grid(c1)
    u = np.zeros((nz + 2, 4, 8))
    zc = g.zc[1:nz + 1]
    u[1:nz + 1] = (1.5 * (1 - (zc - 1) ** 2) + 0.1 * np.sin(3 * zc))[:, None, None]
    s1 = S.initial_state(c1, g, u, np.zeros_like(u), np.zeros_like(u))
    s3 = S.initial_state(c3, g, u, np.zeros_like(u), np.zeros_like(u))
    dt = 0.05
    for k in range(3):
        s1 = S.substep(c1, g, s1, k, dt)
        s3 = S.substep(c3, g, s3, k, dt)
    assert np.max(np.abs(s1.u - s3.u)) < 1e-13 * np.max(np.abs(s1.u))
    assert np.max(np.abs(s1.p - s3.p)) < 1e-12


def test_poiseuille_fixed_point_fully_implicit():
    """The discrete Poiseuille solution is also a fixed point of the fully implicit scheme."""
    nz = 16
    case = Case(4, 4, nz, 1.0, 1.0, 2.0, zbc=ZBC_NOSLIP, beta=1.2, nu=0.5, sgs=SGS_NONE,
                implicit_3d=True, ubulk=1.0)
    g = Grid(case)
    A = np.zeros((nz + 1, nz + 1))
    for c in range(nz):
        a = np.zeros((nz + 2, 1, 1))
        a[c + 1] = 1.0
        a[0], a[nz + 1] = -a[1], -a[nz]
        A[:nz, c] = case.nu * S.ops.lap_z_centre(g, a)[:, 0, 0]
    A[:nz, nz] = 1.0
    A[nz, :nz] = g.dzf[1:nz + 1]
    rhs = np.zeros(nz + 1)
    rhs[nz] = 2.0
    sol = np.linalg.solve(A, rhs)[:nz]
    u = np.zeros((nz + 2, 4, 4))
    u[1:nz + 1] = sol[:, None, None]
    st = S.initial_state(case, g, u, np.zeros_like(u), np.zeros_like(u))
    for _ in range(3):
        st = _step(case, g, st, 0.3)
    assert np.max(np.abs(st.u[1:nz + 1] - sol[:, None, None])) < 1e-12


def test_pressure_update_fully_implicit_identity():
    """Eq. p_update_imp3d with L = D G (the Poisson operator): since D G phi = D u*/(gamma dt),
    p^{k+1/2} - p^{k-1/2} - phi = -(nu/2) D u* exactly (to roundoff), on a random state of a
    no-slip channel."""
    nx, ny, nz = 8, 6, 10
    case = Case(nx, ny, nz, 1.0, 1.0, 2.0, zbc=ZBC_NOSLIP, beta=1.3, nu=0.05, sgs=SGS_SMAG,
                implicit_3d=True)
    g = Grid(case)
    u, v, w, _ = random_state(nx, ny, nz, 4)
    w[nz] = 0.0
    st = S.initial_state(case, g, u, v, w)
    k, dt = 1, 0.02
    ustar, _ = S.predictor(case, g, st, k, dt)
    ustar = S.helmholtz_3d(case, g, st, ustar, k, dt)
    un, vn, wn, p, phi = S.project(case, g, st, ustar, k, dt)
    I = slice(1, nz + 1)
    us, vs, ws = np.zeros_like(u), np.zeros_like(u), np.zeros_like(u)
    us[I], vs[I], ws[I] = ustar
    ws[0] = ws[nz] = 0.0
    div = ops.divergence(g, us, vs, ws)
    lhs = p[I] - st.p[I] - phi[I]
    assert np.max(np.abs(lhs + 0.5 * case.nu * div)) < 1e-12 * max(1.0, np.max(np.abs(div)))
    assert np.max(np.abs(div)) > 1e-3          # the identity is not trivially zero


# ------------------------------------------------------------------ initial projection
@pytest.mark.parametrize("kind", ["iso", "channel", "duct"])
def test_initial_projection(kind):
    """The initial fields' projection: the result is discretely divergence-free (to the
    Poisson solve's rounding), has the prescribed flow rate, leaves an already
    divergence-free field unchanged up to the flow-rate shift (projecting twice equals
    projecting once), and removes a gradient: the removed part is orthogonal to the result,
    sum(u_new . (u - u_new)) dV = 0, since D u_new = 0 and (u - u_new) = G phi."""
    from oracle import ops
    from oracle.case import YBC_WALL
    from synth import isotropic_field, channel_field, duct_field
    if kind == "iso":
        case = Case(12, 12, 12, 2 * np.pi, 2 * np.pi, 2 * np.pi, nu=1e-3)
        g = Grid(case)
        u, v, w = isotropic_field(12, seed=1)
    elif kind == "channel":
        case = Case(16, 8, 10, 2 * np.pi, np.pi, 2.0, zbc=ZBC_WALLMODEL, beta=1.5, nu=5e-4, ubulk=1.0)
        g = Grid(case)
        u, v, w = channel_field(16, 8, 10, g.zc, seed=2)
    else:
        case = Case(12, 8, 6, 3.0, 2.0, 2.0, zbc=ZBC_WALLMODEL, nu=5e-4, ubulk=1.0, ybc=YBC_WALL)
        g = Grid(case)
        u, v, w = duct_field(12, 8, 6, g.zc, 2.0, 2.0, seed=3)
    pu, pv, pw = S.initial_projection(case, g, u, v, w)
    n = g.nz
    I, J = slice(1, n + 1), slice(0, g.ny)

    def div(a, b, c):
        a, b, c = a.copy(), b.copy(), c.copy()
        if case.zbc == ZBC_PERIODIC:
            for f in (a, b, c):
                f[0], f[n + 1] = f[n], f[1]
        if g.ywalls:
            b[:, g.ny + 1] = 0.0
        return ops.divergence(g, a, b, c)[:, J]

    scale = max(np.max(np.abs(pu[I])), np.max(np.abs(pw[I])))
    hmin = min(g.dx, g.dy, np.min(g.dzf[I]))
    assert np.max(np.abs(div(pu, pv, pw))) <= 1e-12 * scale / hmin
    assert np.max(np.abs(div(u, v, w))) > 1e-3 * scale / hmin       # the input was not
    if case.ubulk > 0:
        assert abs(S.bulk_velocity(g, pu) - case.ubulk) <= 1e-14
    qu, qv, qw = S.initial_projection(case, g, pu, pv, pw)
    for a, b in ((qu, pu), (qv, pv), (qw, pw)):
        assert np.max(np.abs(a[I, J] - b[I, J])) <= 1e-12 * scale
    # orthogonality of the removed gradient (volume weights dx dy dzf at u, v; dzc at w)
    dzf = g.dzf[I][:, None, None]
    dzc = g.dzc[1:n + 1][:, None, None]
    # u - u_new = G phi minus the uniform flow-rate shift; G phi has zero mean in periodic x
    ru = u[I, J] - pu[I, J]
    if case.ubulk > 0:
        ru = ru - (ru * dzf).sum() / (dzf.sum() * g.nx * g.ny)
    rv, rw = v[I, J] - pv[I, J], w[I, J] - pw[I, J]
    inner = (np.sum(pu[I, J] * ru * dzf) + np.sum(pv[I, J] * rv * dzf) + np.sum(pw[I, J] * rw * dzc))
    norm = np.sum(pu[I, J] ** 2 * dzf) + np.sum(pv[I, J] ** 2 * dzf) + np.sum(pw[I, J] ** 2 * dzc)
    assert abs(inner) <= 1e-12 * norm
