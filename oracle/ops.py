"""Second-order staggered finite-difference operators (Sec. 2.2: central differences on a
staggered grid; Eq. H_i for the advective and SGS terms).  Test infrastructure only.

All inputs are ghosted arrays of shape (nz + 2, ny, nx) whose ghost planes are already
valid (bc.py); x and y are periodic and handled by np.roll.  Outputs cover the nz
interior planes k = 1..nz (for w: faces 1..nz, of which face nz is the top wall when
z is wall-bounded; the caller ignores it there).
"""
import numpy as np


def xp(a):
    """a at i + 1."""
    return np.roll(a, -1, axis=-1)


def xm(a):
    """a at i - 1."""
    return np.roll(a, 1, axis=-1)


def yp(a):
    return np.roll(a, -1, axis=-2)


def ym(a):
    return np.roll(a, 1, axis=-2)


def col(a):
    """1-D z metric broadcast over (ny, nx)."""
    return np.asarray(a)[:, None, None]


def interior(g):
    return slice(1, g.nz + 1)


# ---------------------------------------------------------------- divergence / gradient
def divergence(g, u, v, w):
    """D u at cell centres: (u_i - u_{i-1})/dx + (v_j - v_{j-1})/dy + (w_k - w_{k-1})/dzf_k."""
    n = g.nz
    I, Im = slice(1, n + 1), slice(0, n)
    return ((u[I] - xm(u[I])) / g.dx + (v[I] - ym(v[I])) / g.dy
            + (w[I] - w[Im]) / col(g.dzf[I]))


def gradient(g, p):
    """G p at the u, v, w faces of the interior planes: forward differences over dx, dy, dzc_k."""
    n = g.nz
    I, Ip = slice(1, n + 1), slice(2, n + 2)
    gx = (xp(p[I]) - p[I]) / g.dx
    gy = (yp(p[I]) - p[I]) / g.dy
    gz = (p[Ip] - p[I]) / col(g.dzc[1:n + 1])
    return gx, gy, gz


# ---------------------------------------------------------------- viscous operators
def lap_xy(g, a):
    """Three-point second differences in x and y (uniform spacing)."""
    I = interior(g)
    b = a[I]
    return (xp(b) - 2.0 * b + xm(b)) / g.dx ** 2 + (yp(b) - 2.0 * b + ym(b)) / g.dy ** 2


def lap_z_centre(g, a):
    """L_zz of a quantity at z-centres (u, v, p):
    [(a_{k+1} - a_k)/dzc_k - (a_k - a_{k-1})/dzc_{k-1}] / dzf_k."""
    n = g.nz
    I, Ip, Im = slice(1, n + 1), slice(2, n + 2), slice(0, n)
    return ((a[Ip] - a[I]) / col(g.dzc[1:n + 1]) - (a[I] - a[Im]) / col(g.dzc[0:n])) / col(g.dzf[I])


def lap_z_face(g, a):
    """L_zz of a quantity at z-faces (w): dzf and dzc swap roles,
    [(a_{k+1} - a_k)/dzf_{k+1} - (a_k - a_{k-1})/dzf_k] / dzc_k."""
    n = g.nz
    I, Ip, Im = slice(1, n + 1), slice(2, n + 2), slice(0, n)
    return ((a[Ip] - a[I]) / col(g.dzf[2:n + 2]) - (a[I] - a[Im]) / col(g.dzf[1:n + 1])) / col(g.dzc[1:n + 1])


# ---------------------------------------------------------------- advection
def advection(g, u, v, w):
    """Divergence form d(u_i u_j)/dx_j at the u, v, w faces (the advective part of Eq. H_i).
    R3: every interpolation is an arithmetic two-point mean, also along stretched z."""
    n = g.nz
    I, Ip, Im = slice(1, n + 1), slice(2, n + 2), slice(0, n)
    dzf, dzc = col(g.dzf[I]), col(g.dzc[1:n + 1])
    uI, vI, wI = u[I], v[I], w[I]
    # u-momentum at (i+1/2, j, k)
    fxx_r = (0.5 * (uI + xp(uI))) ** 2
    fxx_l = (0.5 * (xm(uI) + uI)) ** 2
    fxy_t = 0.5 * (uI + yp(uI)) * 0.5 * (vI + xp(vI))
    fxy_b = ym(fxy_t)
    fxz_t = 0.5 * (uI + u[Ip]) * 0.5 * (wI + xp(wI))
    fxz_b = 0.5 * (u[Im] + uI) * 0.5 * (w[Im] + xp(w[Im]))
    ax = (fxx_r - fxx_l) / g.dx + (fxy_t - fxy_b) / g.dy + (fxz_t - fxz_b) / dzf
    # v-momentum at (i, j+1/2, k)
    fyx_r = 0.5 * (vI + xp(vI)) * 0.5 * (uI + yp(uI))
    fyx_l = xm(fyx_r)
    fyy_t = (0.5 * (vI + yp(vI))) ** 2
    fyy_b = (0.5 * (ym(vI) + vI)) ** 2
    fyz_t = 0.5 * (vI + v[Ip]) * 0.5 * (wI + yp(wI))
    fyz_b = 0.5 * (v[Im] + vI) * 0.5 * (w[Im] + yp(w[Im]))
    ay = (fyx_r - fyx_l) / g.dx + (fyy_t - fyy_b) / g.dy + (fyz_t - fyz_b) / dzf
    # w-momentum at (i, j, k+1/2)
    fzx_r = 0.5 * (wI + xp(wI)) * 0.5 * (uI + u[Ip])
    fzx_l = xm(fzx_r)
    fzy_t = 0.5 * (wI + yp(wI)) * 0.5 * (vI + v[Ip])
    fzy_b = ym(fzy_t)
    fzz_t = (0.5 * (wI + w[Ip])) ** 2
    fzz_b = (0.5 * (w[Im] + wI)) ** 2
    az = (fzx_r - fzx_l) / g.dx + (fzy_t - fzy_b) / g.dy + (fzz_t - fzz_b) / dzc
    return ax, ay, az


# ---------------------------------------------------------------- strain rate
def edge_strains(g, u, v, w):
    """Off-diagonal strain at cell edges (Sec. 2.2, SGS evaluation):
    e12[k, j, i] at (i+1/2, j+1/2, zc_k)   for k = 1..nz
    e13[k, j, i] at (i+1/2, j, zf_k)       for k = 0..nz (z-edges incl. both walls)
    e23[k, j, i] at (i, j+1/2, zf_k)       for k = 0..nz"""
    n = g.nz
    I = slice(1, n + 1)
    e12 = 0.5 * ((yp(u[I]) - u[I]) / g.dy + (xp(v[I]) - v[I]) / g.dx)
    K0, K1 = slice(0, n + 1), slice(1, n + 2)
    dzc = col(g.dzc[0:n + 1])
    e13 = 0.5 * ((u[K1] - u[K0]) / dzc + (xp(w[K0]) - w[K0]) / g.dx)
    e23 = 0.5 * ((v[K1] - v[K0]) / dzc + (yp(w[K0]) - w[K0]) / g.dy)
    return e12, e13, e23


def centre_strain(g, u, v, w):
    """S_ij at cell centres (Sec. 2.2): diagonal components directly from face differences,
    off-diagonal ones computed at the edges and averaged over the four edges around the
    centre.  Returns (S11, S22, S33, S12, S13, S23), each (nz, ny, nx)."""
    n = g.nz
    I, Im = slice(1, n + 1), slice(0, n)
    s11 = (u[I] - xm(u[I])) / g.dx
    s22 = (v[I] - ym(v[I])) / g.dy
    s33 = (w[I] - w[Im]) / col(g.dzf[I])
    e12, e13, e23 = edge_strains(g, u, v, w)
    s12 = 0.25 * (e12 + xm(e12) + ym(e12) + xm(ym(e12)))
    s13 = 0.25 * (e13[1:n + 1] + xm(e13[1:n + 1]) + e13[0:n] + xm(e13[0:n]))
    s23 = 0.25 * (e23[1:n + 1] + ym(e23[1:n + 1]) + e23[0:n] + ym(e23[0:n]))
    return s11, s22, s33, s12, s13, s23


def strain_magnitude(s):
    """|S| = sqrt(2 S_ij S_ij) (Sec. 2.1, after Eq. smag)."""
    s11, s22, s33, s12, s13, s23 = s
    return np.sqrt(2.0 * (s11 ** 2 + s22 ** 2 + s33 ** 2) + 4.0 * (s12 ** 2 + s13 ** 2 + s23 ** 2))


# ---------------------------------------------------------------- SGS flux divergence
def sgs_divergence(g, u, v, w, nut):
    """d(2 nu_t S_ij)/dx_j at the u, v, w faces: the SGS part of Eq. H_i with the deviatoric
    stress of the Boussinesq closure (Sec. 2.1).  nu_t lives at cell centres (ghosted);
    diagonal stresses use it there, edge stresses use R18, the mean of the four centres
    around the edge.  Strain uses the arrays as given (velocity ghosts of bc.py)."""
    n = g.nz
    I, Ip, Im = slice(1, n + 1), slice(2, n + 2), slice(0, n)
    uI, vI, wI = u[I], v[I], w[I]
    nI = nut[I]
    s11 = (uI - xm(uI)) / g.dx
    s22 = (vI - ym(vI)) / g.dy
    # s33 at centres k = 1..nz+1 (k = nz + 1 needed for the top w faces)
    s33_all = (w[1:n + 2] - w[0:n + 1]) / col(g.dzf[1:n + 2])
    e12, e13, e23 = edge_strains(g, u, v, w)
    nu12 = 0.25 * (nI + xp(nI) + yp(nI) + xp(yp(nI)))
    K0, K1 = slice(0, n + 1), slice(1, n + 2)
    nu13 = 0.25 * (nut[K0] + xp(nut[K0]) + nut[K1] + xp(nut[K1]))
    nu23 = 0.25 * (nut[K0] + yp(nut[K0]) + nut[K1] + yp(nut[K1]))
    t11 = 2.0 * nI * s11
    t22 = 2.0 * nI * s22
    t12 = 2.0 * nu12 * e12
    t13 = 2.0 * nu13 * e13          # edges k = 0..nz
    t23 = 2.0 * nu23 * e23
    t33 = 2.0 * nut[1:n + 2] * s33_all   # centres k = 1..nz+1
    dzf, dzc = col(g.dzf[I]), col(g.dzc[1:n + 1])
    fx = (xp(t11) - t11) / g.dx + (t12 - ym(t12)) / g.dy + (t13[1:n + 1] - t13[0:n]) / dzf
    fy = (t12 - xm(t12)) / g.dx + (yp(t22) - t22) / g.dy + (t23[1:n + 1] - t23[0:n]) / dzf
    fz = ((t13[1:n + 1] - xm(t13[1:n + 1])) / g.dx + (t23[1:n + 1] - ym(t23[1:n + 1])) / g.dy
          + (t33[1:n + 1] - t33[0:n]) / dzc)
    return fx, fy, fz
