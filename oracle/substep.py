"""One low-storage RK3 substep (Alg. 1; Eqs. onestar_exp, poi, correc, p_update_exp and,
with Crank-Nicolson in z, Eqs. twostar_imp1d, onestar_imp1d, p_update_imp1d).
Test infrastructure only.

State at a substep boundary (all float64, ghost planes valid, Alg. 2):
  u, v, w, p, nut : (nz + 2, ny, nx)
  rprev           : (ru, rv, rw), each (nz, ny, nx): the explicit right-hand side of the
                    previous substep (unused when beta_k = 0, i.e. on the first substep)
  utau            : dict of per-face friction velocities (wall model's Newton guess)
  tau             : wall stresses (tx_bot, ty_bot, tx_top, ty_top) (wall model)
  tauy            : y-wall stresses (tx_lo, tz_lo, tx_hi, tz_hi) (wall model with y walls)
With walls in y (square duct, Sec. 4.4) the arrays carry the ghost rows of grid.py,
(nz + 2, ny + 2, nx); v on the wall face row ny - 1 stays zero.
  cs              : dynamic coefficient per plane (dynamic model), else None
"""
import numpy as np

from . import bc, ops, poisson, sgs
from .case import ZBC_PERIODIC, ZBC_NOSLIP, ZBC_WALLMODEL

# Wray's low-storage RK3 (Sec. 2.2, after Eq. p_update_exp)
ALPHA = (8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0)
BETA = (0.0, -17.0 / 60.0, -5.0 / 12.0)
GAMMA = tuple(a + b for a, b in zip(ALPHA, BETA))


class State:
    def __init__(self, u, v, w, p, nut=None, rprev=None, utau=None, tau=None, cs=None, tauy=None):
        self.u, self.v, self.w, self.p = u, v, w, p
        self.nut = np.zeros_like(p) if nut is None else nut
        self.rprev = rprev
        self.utau, self.tau, self.cs = utau, tau, cs
        self.tauy = tauy

    def copy(self):
        cp = lambda x: None if x is None else x.copy()
        return State(self.u.copy(), self.v.copy(), self.w.copy(), self.p.copy(),
                     self.nut.copy(),
                     None if self.rprev is None else tuple(r.copy() for r in self.rprev),
                     None if self.utau is None else {k: x.copy() for k, x in self.utau.items()},
                     None if self.tau is None else tuple(t.copy() for t in self.tau),
                     cp(self.cs),
                     None if self.tauy is None else tuple(t.copy() for t in self.tauy))


# ---------------------------------------------------------------- boundary sequence
def apply_bc_and_model(case, g, st):
    """Alg. 2 followed by the eddy viscosity (Alg. 1, first and last substep lines):
    periodic/no-slip ghosts, then the wall stress, then the wall-model ghosts, then nu_t
    with its ghost planes.  Modifies st in place."""
    wm = case.zbc == ZBC_WALLMODEL
    bc.fill_velocity(case, g, st.u, st.v, st.w, tau=_zero_tau(g) if wm else None,
                     tauy=_zero_tauy(g) if wm and g.ywalls else None)
    bc.fill_scalar(case, g, st.p)
    if wm:
        # both wall models read interior values and wall faces only (R35)
        st.tau, utz, _ = bc.wall_stress(case, g, st.u, st.v, st.utau)
        if g.ywalls:
            st.tauy, uty, _ = bc.wall_stress_y(case, g, st.u, st.w, st.utau)
            utz = {**utz, **uty}
        st.utau = utz
        bc.fill_velocity(case, g, st.u, st.v, st.w, tau=st.tau, tauy=st.tauy)
    nut, cs = sgs.eddy_viscosity(case, g, st.u, st.v, st.w, tau=st.tau if wm else None,
                                 tauy=st.tauy if wm else None)
    st.nut = np.zeros_like(st.p)
    st.nut[1:g.nz + 1] = nut
    bc.fill_nut(case, g, st.nut)
    st.cs = cs


def _zero_tau(g):
    z = np.zeros((g.nys, g.nx))
    return (z, z, z, z)


def _zero_tauy(g):
    z = np.zeros((g.nz + 2, g.nx))
    return (z, z, z, z)


# ---------------------------------------------------------------- predictor
def explicit_rhs(case, g, st):
    """R_i = -d(u_i u_j)/dx_j + d(2 nu_t S_ij)/dx_j + nu L u_i: the bracketed terms of
    Eq. onestar_exp.  R4: the sign of H_i as printed in Eq. H_i conflicts with Eq. mom;
    the sign here follows Eq. mom.  With CN in z the viscous part keeps only L_xx + L_yy
    (Eq. twostar_imp1d)."""
    u, v, w = st.u, st.v, st.w
    if case.advection:
        ax, ay, az = ops.advection(g, u, v, w)
    else:
        ax = ay = az = 0.0
    sx, sy, sz = ops.sgs_divergence(g, u, v, w, st.nut)
    if case.implicit_3d:
        # Eq. twostar_imp3d: the explicit part H_i holds advection and SGS stresses only
        return (-ax + sx, -ay + sy, -az + sz)
    lu, lv, lw = ops.lap_xy(g, u), ops.lap_xy(g, v), ops.lap_xy(g, w)
    if not case.implicit_z:
        lu = lu + ops.lap_z_centre(g, u)
        lv = lv + ops.lap_z_centre(g, v)
        lw = lw + ops.lap_z_face(g, w)
    return (-ax + sx + case.nu * lu, -ay + sy + case.nu * lv, -az + sz + case.nu * lw)


def laplacian(g, vel, comp):
    """Full three-dimensional L of u, v (z-centred) or w (z-faces)."""
    lz = ops.lap_z_face(g, vel) if comp == 2 else ops.lap_z_centre(g, vel)
    return ops.lap_xy(g, vel) + lz


def predictor(case, g, st, k, dt):
    """u* (explicit, Eq. onestar_exp) or u** (CN in z, Eq. twostar_imp1d) on the interior
    planes, plus the new explicit right-hand side R^k.  The pressure term uses the
    pressure of the previous substep."""
    n = g.nz
    I = slice(1, n + 1)
    r = explicit_rhs(case, g, st)
    gpx, gpy, gpz = ops.gradient(g, st.p)
    a, b, c = ALPHA[k], BETA[k], GAMMA[k]
    rp = st.rprev if (st.rprev is not None and b != 0.0) else (0.0, 0.0, 0.0)
    out = []
    for comp, (vel, rk, rkm, gp) in enumerate(zip((st.u, st.v, st.w), r, rp, (gpx, gpy, gpz))):
        incr = a * rk + b * rkm - c * gp
        if case.implicit_z:
            lz = ops.lap_z_face(g, vel) if comp == 2 else ops.lap_z_centre(g, vel)
            incr = incr + c * case.nu * lz
        elif case.implicit_3d:
            incr = incr + c * case.nu * laplacian(g, vel, comp)
        out.append(vel[I] + dt * incr)
    if g.ywalls:
        out[1][:, g.ny - 1] = 0.0       # v on the wall face y = ly is not advanced
    return tuple(out), r


def helmholtz_z(case, g, st, ustar2, k, dt):
    """Eq. onestar_imp1d: (1 - gamma nu dt/2 L_zz) u* = u** - gamma nu dt/2 L_zz u^k,
    solved per (i, j) column by the Thomas algorithm in FP64.  Boundary rows: u, v
    no-slip (ghost -u_1 folded into the diagonal) or wall model (R15: the wall-stress flux
    from u^k moved to the right-hand side); w Dirichlet zero on both wall faces.
    Only for wall-bounded z."""
    n = g.nz
    c = GAMMA[k] * case.nu * dt / 2.0
    out = []
    for comp in range(3):
        vel = (st.u, st.v, st.w)[comp]
        lz = ops.lap_z_face(g, vel) if comp == 2 else ops.lap_z_centre(g, vel)
        rhs = ustar2[comp] - c * lz
        if comp < 2:
            # L_zz rows for cells 1..n acting on the unknowns x_1..x_n
            lo = np.array([1.0 / (g.dzc[kk - 1] * g.dzf[kk]) for kk in range(1, n + 1)])
            up = np.array([1.0 / (g.dzc[kk] * g.dzf[kk]) for kk in range(1, n + 1)])
            dg = -(lo + up)
            if case.zbc == ZBC_WALLMODEL:
                # ghost x_0 = x_1 - dzc_0 tau/nu: the wall flux is the known stress
                txb, tyb, txt, tyt = st.tau
                tb, tt = (txb, txt) if comp == 0 else (tyb, tyt)
                dg[0] += lo[0]
                dg[n - 1] += up[n - 1]
                rhs = rhs.copy()
                rhs[0] = rhs[0] + c * (-(tb / case.nu) / g.dzf[1])
                rhs[n - 1] = rhs[n - 1] + c * (-(tt / case.nu) / g.dzf[n])
            else:
                dg[0] -= lo[0]            # ghost x_0 = -x_1
                dg[n - 1] -= up[n - 1]
            lo[0] = 0.0
            up[n - 1] = 0.0
            sol = _tridiag(-c * lo, 1.0 - c * dg, -c * up, rhs)
        else:
            # unknown faces 1..n-1; faces 0 and n are walls (w = 0)
            m = n - 1
            lo = np.array([1.0 / (g.dzf[kk] * g.dzc[kk]) for kk in range(1, m + 1)])
            up = np.array([1.0 / (g.dzf[kk + 1] * g.dzc[kk]) for kk in range(1, m + 1)])
            dg = -(lo + up)
            lo[0] = 0.0
            up[m - 1] = 0.0
            sol = np.zeros_like(rhs)
            sol[:m] = _tridiag(-c * lo, 1.0 - c * dg, -c * up, rhs[:m])
        out.append(sol)
    return tuple(out)


def helmholtz_3d(case, g, st, ustar2, k, dt):
    """Eq. onestar_imp3d: (1 - gamma nu dt/2 L) u* = u** - gamma nu dt/2 L u^k with the full
    Laplacian, solved with the Poisson solver's method (Sec. 2.2): Fourier transforms in x
    and y, then per wavenumber pair (l, m) the z system with the diagonal shifted by
    -c (lambda_x(l) + lambda_y(m)), c = gamma nu dt/2, by the Thomas algorithm in FP64 (an
    FFT in z as well when z is periodic).  Boundary rows as in helmholtz_z: u, v no-slip
    (ghost -x_1 folded into the diagonal) or wall model (wall-stress flux from u^k on the
    right-hand side); w zero on the wall faces."""
    n = g.nz
    c = GAMMA[k] * case.nu * dt / 2.0
    lam = poisson.eigenvalues(g.ny, g.dy)[:, None] + poisson.eigenvalues(g.nx, g.dx)[None, :]
    out = []
    for comp in range(3):
        vel = (st.u, st.v, st.w)[comp]
        rhs = ustar2[comp] - c * laplacian(g, vel, comp)
        if case.zbc == ZBC_PERIODIC:
            lzv = poisson.eigenvalues(n, g.lz / n)
            spec = np.fft.fftn(rhs, axes=(0, 1, 2))
            spec = spec / (1.0 - c * (lzv[:, None, None] + lam[None, :, :]))
            out.append(np.real(np.fft.ifftn(spec, axes=(0, 1, 2))))
            continue
        if comp < 2:
            lo = np.array([1.0 / (g.dzc[kk - 1] * g.dzf[kk]) for kk in range(1, n + 1)])
            up = np.array([1.0 / (g.dzc[kk] * g.dzf[kk]) for kk in range(1, n + 1)])
            dg = -(lo + up)
            rhs = rhs.copy()
            if case.zbc == ZBC_WALLMODEL:
                txb, tyb, txt, tyt = st.tau
                tb, tt = (txb, txt) if comp == 0 else (tyb, tyt)
                dg[0] += lo[0]
                dg[n - 1] += up[n - 1]
                rhs[0] = rhs[0] + c * (-(tb / case.nu) / g.dzf[1])
                rhs[n - 1] = rhs[n - 1] + c * (-(tt / case.nu) / g.dzf[n])
            else:
                dg[0] -= lo[0]
                dg[n - 1] -= up[n - 1]
            lo[0] = 0.0
            up[n - 1] = 0.0
            m = n
        else:
            m = n - 1
            lo = np.array([1.0 / (g.dzf[kk] * g.dzc[kk]) for kk in range(1, m + 1)])
            up = np.array([1.0 / (g.dzf[kk + 1] * g.dzc[kk]) for kk in range(1, m + 1)])
            dg = -(lo + up)
            lo[0] = 0.0
            up[m - 1] = 0.0
        spec = np.fft.fft2(rhs[:m], axes=(1, 2))
        diag = 1.0 - c * dg[:, None, None] - c * lam[None, :, :]
        sol = np.zeros_like(rhs)
        sol[:m] = np.real(np.fft.ifft2(_tridiag_columns(-c * lo, diag, -c * up, spec), axes=(1, 2)))
        out.append(sol)
    return tuple(out)


def _tridiag_columns(lo, dg, up, rhs):
    """Thomas algorithm for every column of rhs[k, m, l] with a per-column diagonal
    dg[k, m, l] and shared off-diagonals lo[k], up[k]."""
    n = rhs.shape[0]
    cp = np.zeros(dg.shape)
    dp = np.zeros(rhs.shape, dtype=rhs.dtype)
    cp[0] = up[0] / dg[0]
    dp[0] = rhs[0] / dg[0]
    for k in range(1, n):
        m = dg[k] - lo[k] * cp[k - 1]
        cp[k] = up[k] / m
        dp[k] = (rhs[k] - lo[k] * dp[k - 1]) / m
    x = np.zeros(rhs.shape, dtype=rhs.dtype)
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def _tridiag(lo, dg, up, rhs):
    """Thomas algorithm per column for rows lo_k x_{k-1} + dg_k x_k + up_k x_{k+1} = rhs_k."""
    n = rhs.shape[0]
    cp = np.zeros(n)
    dp = np.zeros(rhs.shape)
    cp[0] = up[0] / dg[0]
    dp[0] = rhs[0] / dg[0]
    for k in range(1, n):
        m = dg[k] - lo[k] * cp[k - 1]
        cp[k] = up[k] / m
        dp[k] = (rhs[k] - lo[k] * dp[k - 1]) / m
    x = np.zeros(rhs.shape)
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


# ---------------------------------------------------------------- projection
def project(case, g, st, ustar, k, dt):
    """Eqs. poi, correc and p_update_exp / p_update_imp1d.  ustar: interior planes of u*.
    Returns (u, v, w, p, phi) ghosted arrays (velocity ghosts not yet filled)."""
    n = g.nz
    I = slice(1, n + 1)
    gk = GAMMA[k]
    us, vs, ws = np.zeros_like(st.u), np.zeros_like(st.v), np.zeros_like(st.w)
    us[I], vs[I], ws[I] = ustar
    if case.zbc == ZBC_PERIODIC:
        bc.fill_velocity(case, g, us, vs, ws)
    else:
        ws[0] = ws[n] = ws[n + 1] = 0.0
    if g.ywalls:
        vs[:, g.ny - 1:] = 0.0          # wall faces (rows ny - 1 and ny + 1) and row ny
    f = ops.divergence(g, us, vs, ws) / (gk * dt)
    phi = np.zeros_like(st.p)
    phi[I] = poisson.solve(g, f)
    bc.fill_scalar(case, g, phi)
    gx, gy, gz = ops.gradient(g, phi)
    u, v, w = us.copy(), vs.copy(), ws.copy()
    u[I] = us[I] - gk * dt * gx
    v[I] = vs[I] - gk * dt * gy
    w[I] = ws[I] - gk * dt * gz
    if case.zbc != ZBC_PERIODIC:
        w[n] = 0.0
    if g.ywalls:
        v[:, g.ny - 1] = 0.0
    p = st.p.copy()
    p[I] = st.p[I] + phi[I]
    if case.implicit_z:
        p[I] = p[I] - gk * case.nu * dt / 2.0 * ops.lap_z_centre(g, phi)
    elif case.implicit_3d:
        # Eq. p_update_imp3d
        p[I] = p[I] - gk * case.nu * dt / 2.0 * (ops.lap_xy(g, phi) + ops.lap_z_centre(g, phi))
    return u, v, w, p, phi


def bulk_velocity(g, u):
    """Volume mean of u, sum(u dzf) / (nx ny lz)."""
    n = g.nz
    dzf = g.dzf[1:n + 1]
    return np.sum(u[1:n + 1, :g.ny] * dzf[:, None, None]) / (g.nx * g.ny * np.sum(dzf))


def bulk_profile(case, g, k, dt):
    """Shape q(z) of the flow-rate correction.  R21: the spatially uniform, time-varying
    body force of Sec. 4.2 enters the substep like the pressure gradient, gamma_k dt f.
    Explicit viscous terms: it shifts u uniformly (q = 1).  CN in z: it passes through the
    Helmholtz solve, so q = H^-1 1 with H the same tridiagonal matrix as the u rows of
    helmholtz_z (no-slip rows; wall-model rows have zero-flux form and give q = 1)."""
    n = g.nz
    if not (case.implicit_z or case.implicit_3d) or case.zbc != ZBC_NOSLIP:
        return np.ones(n)
    c = GAMMA[k] * case.nu * dt / 2.0
    lo = np.array([1.0 / (g.dzc[kk - 1] * g.dzf[kk]) for kk in range(1, n + 1)])
    up = np.array([1.0 / (g.dzc[kk] * g.dzf[kk]) for kk in range(1, n + 1)])
    dg = -(lo + up)
    dg[0] -= lo[0]
    dg[n - 1] -= up[n - 1]
    lo[0] = 0.0
    up[n - 1] = 0.0
    return _tridiag(-c * lo, 1.0 - c * dg, -c * up, np.ones(n))


def force_bulk(case, g, u, k, dt):
    """Constant flow rate: add s q(z) with s chosen so that <u> = U_b (the projection leaves
    <u> unchanged, so this may follow the correction).  Returns s."""
    if case.ubulk <= 0.0:
        return 0.0
    n = g.nz
    q = bulk_profile(case, g, k, dt)
    dzf = g.dzf[1:n + 1]
    qmean = np.sum(q * dzf) / np.sum(dzf)
    s = (case.ubulk - bulk_velocity(g, u)) / qmean
    u[1:n + 1] += s * q[:, None, None]
    return s


# ---------------------------------------------------------------- substep
def substep(case, g, st, k, dt):
    """One RK3 substep of Alg. 1 from a state whose ghosts and nu_t are valid.
    Returns the new State (ghosts, wall stress and nu_t of the new velocity included)."""
    ustar, r = predictor(case, g, st, k, dt)
    if case.implicit_z:
        ustar = helmholtz_z(case, g, st, ustar, k, dt)
    elif case.implicit_3d:
        ustar = helmholtz_3d(case, g, st, ustar, k, dt)
    u, v, w, p, _ = project(case, g, st, ustar, k, dt)
    force_bulk(case, g, u, k, dt)
    new = State(u, v, w, p, rprev=r, utau=st.utau, tau=st.tau, tauy=st.tauy)
    apply_bc_and_model(case, g, new)
    return new


def initial_projection(case, g, u, v, w):
    """Initial fields made discretely divergence-free by one projection with the substep's
    operators (Eq. poi and Eq. correc without the time factor): phi solves D(G phi) = D u with
    zero flux through walls (or periodic z), u <- u - G phi, the wall faces of w (and of v in a
    duct) at rest.  With a constant flow rate u is then shifted uniformly so that its volume
    mean is U_b (Sec. 4.2 forcing target).  Returns new interior-valued (u, v, w) in the
    ghosted layout (ghost planes zero, to be filled by initial_state)."""
    n = g.nz
    I = slice(1, n + 1)
    us, vs, ws = u.copy(), v.copy(), w.copy()
    if case.zbc == ZBC_PERIODIC:
        bc.fill_velocity(case, g, us, vs, ws)
    else:
        ws[0] = ws[n] = ws[n + 1] = 0.0
    if g.ywalls:
        vs[:, g.ny - 1:] = 0.0
    phi = np.zeros_like(us)
    phi[I] = poisson.solve(g, ops.divergence(g, us, vs, ws))
    bc.fill_scalar(case, g, phi)
    gx, gy, gz = ops.gradient(g, phi)
    ou, ov, ow = np.zeros_like(u), np.zeros_like(v), np.zeros_like(w)
    ou[I], ov[I], ow[I] = us[I] - gx, vs[I] - gy, ws[I] - gz
    if case.zbc != ZBC_PERIODIC:
        ow[n] = 0.0
    if g.ywalls:
        ov[:, g.ny - 1:] = 0.0
        for a in (ou, ow):
            a[:, g.ny:] = 0.0
    if case.ubulk > 0.0:
        ou[I, :g.ny] += case.ubulk - bulk_velocity(g, ou)
    return ou, ov, ow


def initial_state(case, g, u, v, w, p=None):
    """Alg. 1 lines 1-2: take the initial velocity (and pressure), fill ghosts, compute nu_t."""
    st = State(u.copy(), v.copy(), w.copy(), np.zeros_like(u) if p is None else p.copy())
    apply_bc_and_model(case, g, st)
    return st


# ---------------------------------------------------------------- time step
def time_step(case, g, st, cfl=0.5, visc_safety=0.95):
    """R22 (the paper takes the largest stable dt times 0.95, Sec. 4 intro, once per step):
    convective limit cfl / max(|u|/dx + |v|/dy + |w|/dzf) over the face values sharing an
    index, viscous limit visc_safety * 2.51 / (4 max(nu + nu_t) (dx^-2 + dy^-2 [+ dz_min^-2]))
    (2.51: the RK3 stability bound on the negative real axis; the z term is dropped with CN
    in z).  R30: with CN in all directions the molecular viscosity is implicit and only the
    explicit SGS viscosity limits, in all three directions (no limit where nu_t = 0).
    Returns min of the two."""
    n = g.nz
    I = slice(1, n + 1)
    J = slice(0, g.ny)
    dzf = g.dzf[I][:, None, None]
    conv = np.max(np.abs(st.u[I, J]) / g.dx + np.abs(st.v[I, J]) / g.dy + np.abs(st.w[I, J]) / dzf)
    numax = (0.0 if case.implicit_3d else case.nu) + max(0.0, float(np.max(st.nut[I, J])))
    s = 1.0 / g.dx ** 2 + 1.0 / g.dy ** 2
    if not case.implicit_z:
        s += 1.0 / np.min(g.dzf[I]) ** 2
    dt_v = visc_safety * 2.51 / (4.0 * numax * s) if numax > 0.0 else np.inf
    dt_c = cfl / conv if conv > 0.0 else np.inf
    return min(dt_c, dt_v)
