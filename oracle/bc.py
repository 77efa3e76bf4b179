"""Ghost planes (Alg. 2) and the log-law wall model (Eq. wm; Sec. 2.2, wall-model
paragraph).  Test infrastructure only.

z is either periodic (ghost planes are copies) or bounded by two walls at z = 0 and
z = lz.  Wall treatment:
  w = 0 on the wall faces (impermeability);
  p Neumann (p_0 = p_1);
  u, v no-slip (ghost = -first interior value) or wall-modelled: the ghost is set so that
  the viscous flux nu (u_1 - u_0)/dzc_0 equals the modelled wall stress (Sec. 2.2: the
  wall-model stress is the boundary condition of the wall-parallel velocity);
  nu_t odd about the wall (R12), so the SGS flux through the wall is zero and the wall
  stress is carried by the viscous term alone.
With walls in y as well (square duct, Sec. 4.4; R35) the two ghost rows of grid.py follow
the same rules with the roles of the components exchanged: v = 0 on the wall faces (row
ny - 1 and ghost row ny + 1; ghost row ny, beyond the wall, is set to 0 and never read),
u and w odd (no-slip) or from the y-wall stresses, p even, nu_t odd.  z ghost planes are
filled first on every stored row, then the y ghost rows on every stored plane, so the
corner values come from the y rule.
"""
import math

import numpy as np

from .case import ZBC_PERIODIC, ZBC_NOSLIP, ZBC_WALLMODEL
from .ops import xm, xp, ym, yp


def periodic_z(a, nz):
    a[0] = a[nz]
    a[nz + 1] = a[1]


def fill_velocity(case, g, u, v, w, tau=None, tauy=None):
    """Ghost planes of u, v, w (Alg. 2, lines 1, 2 and 4).  tau = (tx_bot, ty_bot, tx_top,
    ty_top) from wall_stress() is required for the wall-model case, and with y walls tauy =
    (tx_lo, tz_lo, tx_hi, tz_hi) from wall_stress_y()."""
    _fill_velocity_z(case, g, u, v, w, tau)
    if g.ywalls:
        _fill_velocity_y(case, g, u, v, w, tauy)


def _fill_velocity_y(case, g, u, v, w, tauy):
    """y ghost rows (R35): row ny above y = ly, row ny + 1 below y = 0."""
    ny = g.ny
    v[:, ny - 1] = 0.0
    v[:, ny] = 0.0
    v[:, ny + 1] = 0.0
    if case.zbc == ZBC_WALLMODEL:
        txl, tzl, txh, tzh = tauy
        u[:, ny + 1] = u[:, 0] - g.dy * txl / case.nu
        w[:, ny + 1] = w[:, 0] - g.dy * tzl / case.nu
        u[:, ny] = u[:, ny - 1] - g.dy * txh / case.nu
        w[:, ny] = w[:, ny - 1] - g.dy * tzh / case.nu
    else:
        u[:, ny + 1] = -u[:, 0]
        w[:, ny + 1] = -w[:, 0]
        u[:, ny] = -u[:, ny - 1]
        w[:, ny] = -w[:, ny - 1]


def _fill_velocity_z(case, g, u, v, w, tau):
    nz = g.nz
    if case.zbc == ZBC_PERIODIC:
        for a in (u, v, w):
            periodic_z(a, nz)
        return
    w[0] = 0.0
    w[nz] = 0.0
    w[nz + 1] = 0.0
    if case.zbc == ZBC_NOSLIP:
        u[0] = -u[1]
        u[nz + 1] = -u[nz]
        v[0] = -v[1]
        v[nz + 1] = -v[nz]
    elif case.zbc == ZBC_WALLMODEL:
        txb, tyb, txt, tyt = tau
        u[0] = u[1] - g.dzc[0] * txb / case.nu
        v[0] = v[1] - g.dzc[0] * tyb / case.nu
        u[nz + 1] = u[nz] - g.dzc[nz] * txt / case.nu
        v[nz + 1] = v[nz] - g.dzc[nz] * tyt / case.nu
    else:
        raise ValueError(case.zbc)


def fill_scalar(case, g, p):
    """Cell-centred scalar (pressure, pressure correction): periodic copy or Neumann."""
    nz = g.nz
    if case.zbc == ZBC_PERIODIC:
        periodic_z(p, nz)
    else:
        p[0] = p[1]
        p[nz + 1] = p[nz]
    if g.ywalls:
        p[:, g.ny + 1] = p[:, 0]
        p[:, g.ny] = p[:, g.ny - 1]


def fill_nut(case, g, nut):
    """R12: odd reflection of nu_t about each wall; periodic copy otherwise."""
    nz = g.nz
    if case.zbc == ZBC_PERIODIC:
        periodic_z(nut, nz)
    else:
        nut[0] = -nut[1]
        nut[nz + 1] = -nut[nz]
    if g.ywalls:
        nut[:, g.ny + 1] = -nut[:, 0]
        nut[:, g.ny] = -nut[:, g.ny - 1]


def strain_ghosts(case, g, u, v, w):
    """Velocity ghosts used only to evaluate the strain rate for the SGS model.
    With the wall model the wall-normal derivative in the first layer is one-sided
    (Sec. 2.2): the ghost is the linear extrapolation, in z, of the first two interior
    values, so the central difference at the wall edge equals (u_2 - u_1)/dzc_1.
    With y walls u and w get the same extrapolation in y (uniform dy), after the z one.
    Otherwise the ordinary ghosts are used.  Returns modified copies (u, v, w)."""
    u2, v2, w2 = u.copy(), v.copy(), w.copy()
    if case.zbc == ZBC_WALLMODEL:
        nz = g.nz
        for a in (u2, v2):
            a[0] = a[1] - g.dzc[0] * (a[2] - a[1]) / g.dzc[1]
            a[nz + 1] = a[nz] + g.dzc[nz] * (a[nz] - a[nz - 1]) / g.dzc[nz - 1]
        if g.ywalls:
            ny = g.ny
            for a in (u2, w2):
                a[:, ny + 1] = a[:, 0] - (a[:, 1] - a[:, 0])
                a[:, ny] = a[:, ny - 1] + (a[:, ny - 1] - a[:, ny - 2])
    return u2, v2, w2


# ---------------------------------------------------------------- log-law wall model
def newton_utau(U, h, nu, kappa, bconst, guess, tol=1e-14, maxit=100):
    """Solve u_tau [ln(u_tau h / nu)/kappa + B] = U for u_tau (Eq. wm) by Newton-Raphson
    (Sec. 2.2).  R14: iterate to |du| <= tol * u_tau instead of the paper's 0.01 %.
    g(x) = x (ln(x h/nu)/kappa + B) is convex with its minimum at x_min where
    ln(x_min h/nu) = -kappa B - 1, and the root for U > 0 lies on the increasing branch;
    an iterate that falls to x_min or below is replaced by the midpoint (x + x_min)/2.
    A guess at or below x_min starts from max(sqrt(nu U/h), 2 x_min).
    Returns (u_tau, iterations).  U = 0 gives u_tau = 0."""
    if U <= 0.0:
        return 0.0, 0
    xmin = nu / h * math.exp(-kappa * bconst - 1.0)
    x = guess if guess > xmin else max(math.sqrt(nu * U / h), 2.0 * xmin)
    for it in range(1, maxit + 1):
        lg = math.log(x * h / nu)
        f = x * (lg / kappa + bconst) - U
        fp = lg / kappa + bconst + 1.0 / kappa
        xn = x - f / fp
        if xn <= xmin:
            xn = 0.5 * (x + xmin)
        if abs(xn - x) <= tol * xn:
            return xn, it
        x = xn
    return x, maxit


def newton_utau_array(U, h, nu, kappa, bconst, guess, tol=1e-14, maxit=100):
    """Element-wise newton_utau over an array: the same iteration for every element, each
    element frozen once its own stopping test holds.  Returns (u_tau, max iterations)."""
    U = np.asarray(U, dtype=np.float64)
    xmin = nu / h * math.exp(-kappa * bconst - 1.0)
    start = np.maximum(np.sqrt(nu * np.maximum(U, 0.0) / h), 2.0 * xmin)
    x = np.where(guess > xmin, guess, start)
    done = U <= 0.0
    x = np.where(done, 0.0, x)
    its = 0
    for it in range(1, maxit + 1):
        if done.all():
            break
        its = it
        xs = np.where(done, 1.0, x)
        lg = np.log(xs * h / nu)
        f = xs * (lg / kappa + bconst) - U
        fp = lg / kappa + bconst + 1.0 / kappa
        xn = xs - f / fp
        xn = np.where(xn <= xmin, 0.5 * (xs + xmin), xn)
        conv = np.abs(xn - xs) <= tol * xn
        x = np.where(done, x, xn)
        done = done | conv
    return x, its


def _wm_planes(case, g):
    """Interpolation planes and weights for each wall (R11, R13).  h_wm = 0 means the
    first off-wall cell centre (no interpolation)."""
    nz = g.nz
    if case.h_wm <= 0.0:
        return (1, 2, 0.0, g.zc[1]), (nz, nz - 1, 0.0, g.lz - g.zc[nz])
    h = case.h_wm
    kb = max(k for k in range(1, nz) if g.zc[k] <= h)
    tb = (h - g.zc[kb]) / (g.zc[kb + 1] - g.zc[kb])
    kt = min(k for k in range(2, nz + 1) if g.lz - g.zc[k] <= h)
    dt_lo, dt_hi = g.lz - g.zc[kt], g.lz - g.zc[kt - 1]
    tt = (h - dt_lo) / (dt_hi - dt_lo)
    return (kb, kb + 1, tb, h), (kt, kt - 1, tt, h)


def wall_stress(case, g, u, v, utau_prev):
    """Wall-model stresses (Eq. wm, Sec. 2.2).  For each wall and each wall-parallel
    component, at that component's own face points: interpolate u and v linearly in z to
    h_wm, bring the other component to the same point by the mean of its four surrounding
    faces, take U = sqrt(u^2 + v^2), solve for u_tau, and set tau = u_tau^2 * (component)/U.
    utau_prev: dict of previous u_tau arrays (Newton's starting guess) or None.
    Returns ((tx_bot, ty_bot, tx_top, ty_top), utau dict, max iteration count)."""
    bot, top = _wm_planes(case, g)
    out, utau, itmax = [], {}, 0
    for name, (k0, k1, t, h) in (("bot", bot), ("top", top)):
        ui = (1.0 - t) * u[k0] + t * u[k1]
        vi = (1.0 - t) * v[k0] + t * v[k1]
        v_at_u = 0.25 * (vi + xp(vi) + ym(vi) + xp(ym(vi)))
        u_at_v = 0.25 * (ui + xm(ui) + yp(ui) + xm(yp(ui)))
        for comp, a, b in (("x", ui, v_at_u), ("y", vi, u_at_v)):
            key = name + comp
            prev = utau_prev[key] if utau_prev is not None else np.zeros_like(a)
            U = np.sqrt(a * a + b * b)
            ut, its = newton_utau_array(U, h, case.nu, case.kappa, case.bconst, prev)
            itmax = max(itmax, its)
            safe = np.where(U > 0.0, U, 1.0)
            tau = np.where(U > 0.0, ut * ut * a / safe, 0.0)
            utau[key] = ut
            out.append(tau)
    txb, tyb, txt, tyt = out
    if g.ywalls:
        # R35: the y ghost rows carry no z-wall stress, and the v row on the wall face
        # y = ly has no wall-parallel velocity
        for a in out:
            a[g.ny:] = 0.0
        tyb[g.ny - 1] = 0.0
        tyt[g.ny - 1] = 0.0
    return (txb, tyb, txt, tyt), utau, itmax


def _wm_rows(case, g):
    """y-wall counterpart of _wm_planes (uniform dy, R35): (row, next row inward, weight,
    height) for the wall at y = 0 and the wall at y = ly."""
    ny = g.ny
    yc = g.yc
    if case.h_wm <= 0.0:
        return (0, 1, 0.0, yc[0]), (ny - 1, ny - 2, 0.0, g.ly - yc[ny - 1])
    h = case.h_wm
    jb = max(j for j in range(0, ny - 1) if yc[j] <= h)
    tb = (h - yc[jb]) / (yc[jb + 1] - yc[jb])
    jt = min(j for j in range(1, ny) if g.ly - yc[j] <= h)
    d_lo, d_hi = g.ly - yc[jt], g.ly - yc[jt - 1]
    tt = (h - d_lo) / (d_hi - d_lo)
    return (jb, jb + 1, tb, h), (jt, jt - 1, tt, h)


def wall_stress_y(case, g, u, w, utau_prev):
    """Wall-model stresses on the walls y = 0 and y = ly (square duct, Sec. 4.4; R35): the
    rule of wall_stress() with z replaced by y and v by w.  For each wall and each wall-
    parallel component (u at (i+1/2, k), w at (i, k+1/2)), at its own face points of the
    interior planes: interpolate u and w linearly in y to h_wm, bring the other component
    to the same point by the mean of its four surrounding faces (x and z neighbours), take
    U = sqrt(u^2 + w^2), solve for u_tau and set tau = u_tau^2 (component) / U.  w on the
    z wall faces (k = 0 and nz) has no stress.  Returns ((tx_lo, tz_lo, tx_hi, tz_hi) each
    (nz + 2, nx) with zero ghost planes, utau dict, max iteration count)."""
    lo, hi = _wm_rows(case, g)
    n = g.nz
    out, utau, itmax = [], {}, 0
    for name, (j0, j1, t, h) in (("ylo", lo), ("yhi", hi)):
        ui = (1.0 - t) * u[:, j0] + t * u[:, j1]          # (nz + 2, nx)
        wi = (1.0 - t) * w[:, j0] + t * w[:, j1]
        w_at_u = np.zeros_like(ui)
        u_at_w = np.zeros_like(ui)
        for k in range(1, n + 1):
            w_at_u[k] = 0.25 * (wi[k] + xp(wi[k]) + wi[k - 1] + xp(wi[k - 1]))
            u_at_w[k] = 0.25 * (ui[k] + xm(ui[k]) + ui[k + 1] + xm(ui[k + 1]))
        for comp, a, b in (("x", ui, w_at_u), ("z", wi, u_at_w)):
            key = name + comp
            prev = utau_prev[key] if (utau_prev is not None and key in utau_prev) else np.zeros_like(a)
            U = np.sqrt(a * a + b * b)
            ut, its = newton_utau_array(U, h, case.nu, case.kappa, case.bconst, prev)
            itmax = max(itmax, its)
            safe = np.where(U > 0.0, U, 1.0)
            tau = np.where(U > 0.0, ut * ut * a / safe, 0.0)
            tau[0] = 0.0
            tau[n + 1] = 0.0
            if comp == "z":
                tau[n] = 0.0
            utau[key] = ut
            out.append(tau)
    return tuple(out), utau, itmax


def noslip_wall_stress_y(case, g, u, w):
    """y-wall counterpart of noslip_wall_stress (R35): nu du/dy and nu dw/dy at the walls
    y = 0 and y = ly from the no-slip ghost rows, (tx_lo, tz_lo, tx_hi, tz_hi) each
    (nz + 2, nx), zero on the z ghost planes and, for w, on the z wall faces."""
    ny, n = g.ny, g.nz
    out = [case.nu * (u[:, 0] - u[:, ny + 1]) / g.dy, case.nu * (w[:, 0] - w[:, ny + 1]) / g.dy,
           case.nu * (u[:, ny - 1] - u[:, ny]) / g.dy, case.nu * (w[:, ny - 1] - w[:, ny]) / g.dy]
    for q, a in enumerate(out):
        a[0] = 0.0
        a[n + 1] = 0.0
        if q % 2 == 1 and not g.periodic_z:
            a[n] = 0.0
    return tuple(out)


def noslip_wall_stress(case, g, u, v):
    """Viscous wall stress nu du/dz at each wall from the no-slip ghosts, signed so that
    a positive value opposes positive velocity (same convention as wall_stress)."""
    nz = g.nz
    txb = case.nu * (u[1] - u[0]) / g.dzc[0]
    tyb = case.nu * (v[1] - v[0]) / g.dzc[0]
    txt = case.nu * (u[nz] - u[nz + 1]) / g.dzc[nz]
    tyt = case.nu * (v[nz] - v[nz + 1]) / g.dzc[nz]
    return txb, tyb, txt, tyt
