"""Eddy-viscosity models (Sec. 2.1, Eqs. smag, dsmag, cs, lij, mij; Sec. 2.2, SGS
evaluation and test-filter paragraph).  Test infrastructure only.

Inputs are ghosted velocity arrays whose ghost planes follow bc.fill_velocity; the strain
for the model uses bc.strain_ghosts.  Outputs are nu_t (or |S| and c_s) on the interior
planes k = 1..nz, shape (nz, ny, nx).
"""
import numpy as np

from . import bc
from .case import ZBC_PERIODIC, ZBC_WALLMODEL, SGS_SMAG, SGS_SMAG_VD, SGS_DSM
from .ops import centre_strain, strain_magnitude, xm, xp, ym, yp


def model_strain(case, g, u, v, w):
    """S_ij at cell centres with the SGS-strain ghosts (one-sided wall-normal derivative
    in the first layer when the wall model is on, Sec. 2.2)."""
    us, vs, ws = bc.strain_ghosts(case, g, u, v, w)
    return centre_strain(g, us, vs, ws)


def smagorinsky(case, g, u, v, w, utau_walls=None):
    """Static model, Eq. smag: nu_t = (C_s Delta D)^2 |S|.
    Delta per R5.  D = 1 - exp(-y*/25) (van Driest, Sec. 2.1) for SGS_SMAG_VD, with
    y* = d u_tau / nu, d the distance to the nearer wall and u_tau that wall's friction
    velocity (R6: utau_walls = (u_tau bottom, u_tau top)); D = 1 for SGS_SMAG."""
    s = model_strain(case, g, u, v, w)
    smag = strain_magnitude(s)
    delta = g.delta()[:, None, None]
    damp = np.ones((g.nz, 1, 1))
    if case.sgs == SGS_SMAG_VD and g.ywalls:
        damp = duct_damping(case, g, utau_walls)[:, :, None]
    elif case.sgs == SGS_SMAG_VD and case.zbc != ZBC_PERIODIC:
        zc = g.zc[1:g.nz + 1]
        lower = zc <= 0.5 * g.lz
        dist = np.where(lower, zc, g.lz - zc)
        ut = np.where(lower, utau_walls[0], utau_walls[1])
        damp = (1.0 - np.exp(-dist * ut / case.nu / 25.0))[:, None, None]
    return (case.cs * delta * damp) ** 2 * smag


def duct_damping(case, g, utau_walls):
    """R36: van Driest factor with four walls, per (k, j) (nz, nys): y* is the smallest of
    d_w u_tau,w / nu over the four walls w (d_w the distance to wall w): the nearest wall in
    its own wall units, a rule that needs no tie-break where two walls are equally far.
    utau_walls = (z bottom, z top, y = 0, y = ly).  Ghost rows get 1 (their values are
    replaced by the ghost rule)."""
    n, ny = g.nz, g.ny
    out = np.ones((n, g.nys))
    for k in range(1, n + 1):
        zc = g.zc[k]
        for j in range(ny):
            yc = g.yc[j]
            ys = min(zc * utau_walls[0], (g.lz - zc) * utau_walls[1], yc * utau_walls[2],
                     (g.ly - yc) * utau_walls[3]) / case.nu
            out[k - 1, j] = 1.0 - np.exp(-ys / 25.0)
    return out


def duct_friction_velocity(g, tau, tauy):
    """R36: per-wall friction velocity sqrt(|(<tau_1>, <tau_2>)|) for the four duct walls,
    each component averaged over its own points on that wall that are not wall faces: z
    walls over rows j < ny (the v stress over j < ny - 1), y walls over planes 1..nz (the w
    stress over faces 1..nz - 1).  Returns (z bottom, z top, y = 0, y = ly)."""
    ny, n = g.ny, g.nz
    txb, tyb, txt, tyt = tau
    txl, tzl, txh, tzh = tauy
    m = lambda a, sl: float(np.mean(a[sl]))
    zb = np.sqrt(np.hypot(m(txb, slice(0, ny)), m(tyb, slice(0, ny - 1))))
    zt = np.sqrt(np.hypot(m(txt, slice(0, ny)), m(tyt, slice(0, ny - 1))))
    yl = np.sqrt(np.hypot(m(txl, slice(1, n + 1)), m(tzl, slice(1, n))))
    yh = np.sqrt(np.hypot(m(txh, slice(1, n + 1)), m(tzh, slice(1, n))))
    return zb, zt, yl, yh


def friction_velocity(tau):
    """R6: per-wall friction velocity from the plane-mean wall-stress vector,
    u_tau = sqrt(|(<tau_x>, <tau_y>)|).  tau = (tx_bot, ty_bot, tx_top, ty_top)."""
    txb, tyb, txt, tyt = tau
    ub = np.sqrt(np.hypot(np.mean(txb), np.mean(tyb)))
    ut = np.sqrt(np.hypot(np.mean(txt), np.mean(tyt)))
    return ub, ut


# ---------------------------------------------------------------- dynamic model
def _filter_xy(q, g=None, centred_y=True):
    """Trapezoidal box filter (1/4, 1/2, 1/4) in x then y (R7, uniform weights, Sec. 2.2).
    With y walls (duct, R38) the y pass of a y-centred quantity uses the index-space
    extrapolation of R9 in the ghost rows, which makes it the identity on the first and last
    rows; a quantity on y faces (v) keeps its true wall values (zero ghost rows)."""
    q = 0.25 * xm(q) + 0.5 * q + 0.25 * xp(q)
    if g is not None and g.ywalls and centred_y:
        ny = g.ny
        q = q.copy()
        q[..., ny + 1, :] = 2.0 * q[..., 0, :] - q[..., 1, :]
        q[..., ny, :] = 2.0 * q[..., ny - 1, :] - q[..., ny - 2, :]
    return 0.25 * ym(q) + 0.5 * q + 0.25 * yp(q)


def _pad_z_centre(case, q):
    """Ghost planes for a z-centred quantity before the z pass of the test filter: periodic
    copy, or (R9) linear extrapolation in index space, q_0 = 2 q_1 - q_2, which makes the
    z pass the identity on the first off-wall layer (the paper's 2-D filter there)."""
    n = q.shape[0]
    out = np.empty((n + 2,) + q.shape[1:])
    out[1:n + 1] = q
    if case.zbc == ZBC_PERIODIC:
        out[0], out[n + 1] = q[n - 1], q[0]
    else:
        out[0] = 2.0 * q[0] - q[1]
        out[n + 1] = 2.0 * q[n - 1] - q[n - 2]
    return out


def test_filter_centre(case, q, g=None, centred_y=True):
    """3-D test filter of a z-centred quantity on the interior planes (nz, ny, nx)."""
    qp = _pad_z_centre(case, _filter_xy(q, g, centred_y))
    return 0.25 * qp[:-2] + 0.5 * qp[1:-1] + 0.25 * qp[2:]


def test_filter_velocity(case, g, u, v, w):
    """Test-filtered staggered velocity, each component on its own grid (R8).  u and v are
    z-centred (filtered like test_filter_centre); w lives on z-faces and uses the true
    wall values w = 0 (or periodic copies) as its z neighbours.  Ghost planes of the result
    follow the SGS-strain rule of the unfiltered field."""
    n = g.nz
    I = slice(1, n + 1)
    uf, vf, wf = np.zeros_like(u), np.zeros_like(v), np.zeros_like(w)
    uf[I] = test_filter_centre(case, u[I], g)
    vf[I] = test_filter_centre(case, v[I], g, centred_y=False)
    wxy = _filter_xy(w, g)
    wf[I] = 0.25 * wxy[0:n] + 0.5 * wxy[1:n + 1] + 0.25 * wxy[2:n + 2]
    if case.zbc == ZBC_PERIODIC:
        bc.fill_velocity(case, g, uf, vf, wf)
    else:
        wf[0] = 0.0
        wf[n] = 0.0
        wf[n + 1] = 0.0
        if case.zbc == ZBC_WALLMODEL:
            pass        # strain_ghosts() below extrapolates
        else:
            uf[0], uf[n + 1] = -uf[1], -uf[n]
            vf[0], vf[n + 1] = -vf[1], -vf[n]
    if g.ywalls:
        # duct (R38): v~ vanishes on the y wall faces; the y ghost rows of u~ and w~ follow
        # the strain ghost rule (odd with no-slip, extrapolated by strain_ghosts() with the
        # wall model), after the z ghost planes
        ny = g.ny
        vf[:, ny - 1:] = 0.0
        if case.zbc != ZBC_WALLMODEL:
            for a in (uf, wf):
                a[:, ny + 1] = -a[:, 0]
                a[:, ny] = -a[:, ny - 1]
    return uf, vf, wf


PAIRS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))   # order of s: 11 22 33 12 13 23


def germano_tensors(case, g, u, v, w):
    """Steps 1-5 of the dynamic procedure (Eqs. lij, mij; Sec. 2.2 test-filter paragraph):
    1. velocities averaged to cell centres; 2. S_ij and |S| at centres;
    3. L_ij = F(uc_i uc_j) - F(uc_i) F(uc_j);
    4. S~_ij from the test-filtered staggered velocity with the same strain routine;
    5. M_ij = 2 Delta^2 [F(|S| S_ij) - alpha^2 |S~| S~_ij] with alpha^2 = 4 (alpha = 2 in
       3-D) and alpha^2 = 4^(2/3) on the first off-wall layers (alpha = 4^(1/3)).
    Returns (L, M, |S|): L and M lists of six (nz, rows, nx) arrays in the order of PAIRS."""
    n = g.nz
    I, Im = slice(1, n + 1), slice(0, n)
    uc = 0.5 * (u[I] + xm(u[I]))
    vc = 0.5 * (v[I] + ym(v[I]))
    wc = 0.5 * (w[I] + w[Im])
    s = model_strain(case, g, u, v, w)
    smag = strain_magnitude(s)
    F = lambda q: test_filter_centre(case, q, g)
    vel = (uc, vc, wc)
    fvel = [F(q) for q in vel]
    uf, vf, wf = test_filter_velocity(case, g, u, v, w)
    st = model_strain(case, g, uf, vf, wf)
    stmag = strain_magnitude(st)
    delta2 = (g.delta() ** 2)[:, None, None]
    alpha2 = _alpha2(case, g)
    L, M = [], []
    for c, (a, b) in enumerate(PAIRS):
        L.append(F(vel[a] * vel[b]) - fvel[a] * fvel[b])
        M.append(2.0 * delta2 * (F(smag * s[c]) - alpha2 * stmag * st[c]))
    return L, M, smag


def dynamic_coefficient(case, g, u, v, w):
    """Dynamic procedure (Eqs. cs, lij, mij; Sec. 2.2 test-filter paragraph): L_ij and M_ij
    from germano_tensors, then
    6. c_s = <L_ij M_ij>/<M_ij M_ij> over each x-y plane (over the whole box when z is
       periodic), clipped at zero; R10: c_s = 0 where <M M> = 0.
    Returns (c_s per plane (nz,), |S| (nz, ny, nx), sum LM per plane, sum MM per plane)."""
    n = g.nz
    L, M, smag = germano_tensors(case, g, u, v, w)
    lm = np.zeros_like(smag)
    mm = np.zeros_like(smag)
    for c, (a, b) in enumerate(PAIRS):
        wgt = 1.0 if a == b else 2.0          # symmetric tensors: off-diagonals twice
        lm += wgt * L[c] * M[c]
        mm += wgt * M[c] * M[c]
    if case.zbc == ZBC_PERIODIC:
        slm = np.full(n, lm.sum())
        smm = np.full(n, mm.sum())
    elif g.ywalls:
        slm = lm.sum(axis=2)          # duct (R38): x lines, the only homogeneous direction
        smm = mm.sum(axis=2)
        slm[:, g.ny:] = 0.0
        smm[:, g.ny:] = 0.0
    else:
        slm = lm.sum(axis=(1, 2))
        smm = mm.sum(axis=(1, 2))
    cs = np.where(smm > 0.0, np.maximum(slm / np.where(smm > 0.0, smm, 1.0), 0.0), 0.0)
    return cs, smag, slm, smm


def _alpha2(case, g):
    """alpha^2 per cell (n, rows, 1): 4 for the 3-D test filter; 4^(2/3) where the filter is
    2-D (the first off-wall layer of one wall pair, R9); 2^(2/3) where it is 1-D (a duct's
    corner cells, first off-wall in y and z, R38)."""
    n = g.nz
    dims = np.full((n, g.nys, 1), 3)
    if case.zbc != ZBC_PERIODIC:
        dims[0] -= 1
        dims[n - 1] -= 1
    if g.ywalls:
        dims[:, 0] -= 1
        dims[:, g.ny - 1] -= 1
    table = {3: 4.0, 2: 4.0 ** (2.0 / 3.0), 1: 2.0 ** (2.0 / 3.0)}
    return np.vectorize(table.get)(dims).astype(np.float64)


def dynamic_smagorinsky(case, g, u, v, w):
    """Eq. dsmag: nu_t = c_s Delta^2 |S|.  Returns (nu_t, c_s); c_s per plane, or per x line
    (nz, ny + 2) in a duct."""
    cs, smag, _, _ = dynamic_coefficient(case, g, u, v, w)
    c3 = cs[:, :, None] if cs.ndim == 2 else cs[:, None, None]
    return c3 * (g.delta() ** 2)[:, None, None] * smag, cs


def eddy_viscosity(case, g, u, v, w, tau=None, tauy=None):
    """nu_t on the interior planes for the configured model (SGS_NONE gives zeros).
    With y walls (square duct) the learned closure is not defined here."""
    if g.ywalls and case.sgs > SGS_DSM:
        raise NotImplementedError("duct: the static and dynamic models")
    if case.sgs in (SGS_SMAG, SGS_SMAG_VD):
        ut = None
        if case.sgs == SGS_SMAG_VD and case.zbc != ZBC_PERIODIC:
            if tau is None:
                tau = bc.noslip_wall_stress(case, g, u, v)
            if g.ywalls:
                if tauy is None:
                    tauy = bc.noslip_wall_stress_y(case, g, u, w)
                ut = duct_friction_velocity(g, tau, tauy)
            else:
                ut = friction_velocity(tau)
        return smagorinsky(case, g, u, v, w, ut), None
    if case.sgs == SGS_DSM:
        return dynamic_smagorinsky(case, g, u, v, w)
    return np.zeros((g.nz, g.nys, g.nx)), None
