"""Rounding bound of the dynamic Smagorinsky model (Sec. 2.1 Eqs. cs, lij, mij; Sec. 2.2
test-filter paragraph) for comparing two float64 implementations that evaluate the same
formulas in different orders (the oracle's separable passes and numpy sums, the fused
kernel's 9-point filter and tree sums).  Test infrastructure, an error-analysis aid: it is
not part of the model.

Every intermediate is carried as a pair (value, bound): the value is the oracle's float64
result, the bound a first-order bound on |computed - exact| that holds for either
implementation.  Rules, with u the unit roundoff 2^-53 (inputs u, v, w are exact):
  a +- b       bound(a) + bound(b) + u |a +- b|
  a * b        |a| bound(b) + |b| bound(a) + bound(a) bound(b) + u |a b|
  a * c        |c| bound(a) + 2 u |a c| for a rounded constant c (a reciprocal, a table entry,
               alpha^2, 2 Delta^2; one rounding for the constant, one for the product), exact
               for a power of two
  sum of n weighted terms with power-of-two weights, in any order and with or without fused
               multiply-adds: sum |w| bound + (n - 1) u sum |w| |term|
  |S| = sqrt(2 S_ij S_ij) is a weighted 2-norm, so |fl|S| - |S|| <= norm(bound(S_ij))
               + 4 u |S| (six squares, their sum and the root)
  the test filter is a sum of at most 36 weighted terms (27, and the wall-layer
               extrapolations q_0 = 2 q_1 - q_2 of R9 add one term per z tap), so its bound is
               F(bound) + 35 u F(|q|), F(|q|) the filter of magnitudes with every
               extrapolation taken as 2 |q_1| + |q_2|
  plane sums of N cells: depth D of the summation tree (the oracle's numpy reduction and the
               kernel's wave shuffles, per-thread strides and block tree; the larger of the
               two) bounds the rounding by D u sum |term|
  c = max(0, a / b): two results a_1, b_1 and a_2, b_2, each within (Ea, Eb) of exact,
               differ by at most 2 (Ea + cbar Eb) / (b - 2 Eb) + 2 u cbar, cbar = max(0, a +
               2 Ea) / (b - 2 Eb) an upper bound of either coefficient (the clip at zero is
               1-Lipschitz)
The bound is first order: products of two bounds are kept where they appear, higher
powers of u are dropped (they are below 1e-30 relative here).
"""
import math

import numpy as np

from oracle.case import ZBC_PERIODIC, ZBC_WALLMODEL
from oracle.ops import xm, xp, ym, yp
from oracle.sgs import _alpha2, PAIRS

U = 2.0 ** -53


class D:
    """A float64 value array and a bound on its rounding error."""
    __slots__ = ("v", "e")

    def __init__(self, v, e=None):
        self.v = np.asarray(v, dtype=np.float64)
        self.e = np.zeros_like(self.v) if e is None else e

    def map(self, f):
        """An exact rearrangement (shift, slice, copy) applied to both parts."""
        return D(f(self.v), f(self.e))


def add(a, b, sign=1.0):
    v = a.v + sign * b.v
    return D(v, a.e + b.e + U * np.abs(v))


def mul(a, b):
    v = a.v * b.v
    return D(v, np.abs(a.v) * b.e + np.abs(b.v) * a.e + a.e * b.e + U * np.abs(v))


def scale(a, c, exact=False):
    v = a.v * c
    return D(v, np.abs(c) * a.e + (0.0 if exact else 2.0 * U) * np.abs(v))


def wsum(terms, weights):
    n = len(terms)
    v = sum(w * t.v for t, w in zip(terms, weights))
    e = sum(abs(w) * t.e for t, w in zip(terms, weights))
    m = sum(abs(w) * np.abs(t.v) for t, w in zip(terms, weights))
    return D(v, e + (n - 1) * U * m)


def col(a):
    return np.asarray(a)[:, None, None]


# ---------------------------------------------------------------- strain (Sec. 2.2)
def strain_ghosts(case, g, u, v, w):
    """Dual version of bc.strain_ghosts: the wall model's linear extrapolation in z of u and
    v (and in y of u and w in a duct) rounds; the other ghosts are copies."""
    u2, v2, w2 = (D(a.v.copy(), a.e.copy()) for a in (u, v, w))
    if case.zbc == ZBC_WALLMODEL:
        nz = g.nz
        for a in (u2, v2):
            lo = add(D(a.v[1], a.e[1]), scale(add(D(a.v[2], a.e[2]), D(a.v[1], a.e[1]), -1.0),
                                              g.dzc[0] / g.dzc[1]), -1.0)
            hi = add(D(a.v[nz], a.e[nz]), scale(add(D(a.v[nz], a.e[nz]), D(a.v[nz - 1], a.e[nz - 1]), -1.0),
                                                g.dzc[nz] / g.dzc[nz - 1]))
            a.v[0], a.e[0] = lo.v, lo.e
            a.v[nz + 1], a.e[nz + 1] = hi.v, hi.e
        if g.ywalls:
            ny = g.ny
            for a in (u2, w2):
                r0, r1 = D(a.v[:, 0], a.e[:, 0]), D(a.v[:, 1], a.e[:, 1])
                lo = add(r0, add(r1, r0, -1.0), -1.0)
                s0, s1 = D(a.v[:, ny - 1], a.e[:, ny - 1]), D(a.v[:, ny - 2], a.e[:, ny - 2])
                hi = add(s0, add(s0, s1, -1.0))
                a.v[:, ny + 1], a.e[:, ny + 1] = lo.v, lo.e
                a.v[:, ny], a.e[:, ny] = hi.v, hi.e
    return u2, v2, w2


def centre_strain(g, u, v, w):
    """Dual version of ops.centre_strain (diagonal terms from face differences, off-diagonal
    terms as four-edge means)."""
    n = g.nz
    I, Im = slice(1, n + 1), slice(0, n)
    K0, K1 = slice(0, n + 1), slice(1, n + 2)
    uI, vI, wI = u.map(lambda a: a[I]), v.map(lambda a: a[I]), w.map(lambda a: a[I])
    s11 = scale(add(uI, uI.map(xm), -1.0), 1.0 / g.dx)
    s22 = scale(add(vI, vI.map(ym), -1.0), 1.0 / g.dy)
    s33 = scale(add(wI, w.map(lambda a: a[Im]), -1.0), col(1.0 / g.dzf[I]))
    e12 = scale(add(scale(add(uI.map(yp), uI, -1.0), 1.0 / g.dy), scale(add(vI.map(xp), vI, -1.0), 1.0 / g.dx)),
                0.5, exact=True)
    rz = col(1.0 / g.dzc[0:n + 1])
    uk1, uk0 = u.map(lambda a: a[K1]), u.map(lambda a: a[K0])
    vk1, vk0 = v.map(lambda a: a[K1]), v.map(lambda a: a[K0])
    wk0 = w.map(lambda a: a[K0])
    e13 = scale(add(scale(add(uk1, uk0, -1.0), rz), scale(add(wk0.map(xp), wk0, -1.0), 1.0 / g.dx)), 0.5, exact=True)
    e23 = scale(add(scale(add(vk1, vk0, -1.0), rz), scale(add(wk0.map(yp), wk0, -1.0), 1.0 / g.dy)), 0.5, exact=True)
    q = (0.25, 0.25, 0.25, 0.25)
    s12 = wsum([e12, e12.map(xm), e12.map(ym), e12.map(lambda a: xm(ym(a)))], q)
    t1, t0 = e13.map(lambda a: a[1:n + 1]), e13.map(lambda a: a[0:n])
    s13 = wsum([t1, t1.map(xm), t0, t0.map(xm)], q)
    t1, t0 = e23.map(lambda a: a[1:n + 1]), e23.map(lambda a: a[0:n])
    s23 = wsum([t1, t1.map(ym), t0, t0.map(ym)], q)
    return [s11, s22, s33, s12, s13, s23]


def strain_magnitude(s):
    v = np.sqrt(2.0 * (s[0].v ** 2 + s[1].v ** 2 + s[2].v ** 2) + 4.0 * (s[3].v ** 2 + s[4].v ** 2 + s[5].v ** 2))
    e = np.sqrt(2.0 * (s[0].e ** 2 + s[1].e ** 2 + s[2].e ** 2) + 4.0 * (s[3].e ** 2 + s[4].e ** 2 + s[5].e ** 2))
    return D(v, e + 4.0 * U * v)


# ---------------------------------------------------------------- test filter (R7, R9, R38)
def _fxy(q, g, centred_y, magnitude):
    q = 0.25 * xm(q) + 0.5 * q + 0.25 * xp(q)
    if g.ywalls and centred_y:
        ny = g.ny
        q = q.copy()
        sg = 1.0 if magnitude else -1.0
        q[..., ny + 1, :] = 2.0 * q[..., 0, :] + sg * q[..., 1, :]
        q[..., ny, :] = 2.0 * q[..., ny - 1, :] + sg * q[..., ny - 2, :]
    return 0.25 * ym(q) + 0.5 * q + 0.25 * yp(q)


def _fz_centre(case, q, magnitude):
    n = q.shape[0]
    out = np.empty((n + 2,) + q.shape[1:])
    out[1:n + 1] = q
    if case.zbc == ZBC_PERIODIC:
        out[0], out[n + 1] = q[n - 1], q[0]
    else:
        sg = 1.0 if magnitude else -1.0
        out[0] = 2.0 * q[0] + sg * q[1]
        out[n + 1] = 2.0 * q[n - 1] + sg * q[n - 2]
    return 0.25 * out[:-2] + 0.5 * out[1:-1] + 0.25 * out[2:]


def filter_centre(case, g, q, centred_y=True):
    """Test filter of a z-centred quantity on the interior planes."""
    v = _fz_centre(case, _fxy(q.v, g, centred_y, False), False)
    mag = _fz_centre(case, _fxy(np.abs(q.v), g, centred_y, True), True)
    err = _fz_centre(case, _fxy(q.e, g, centred_y, True), True)
    return D(v, err + 35.0 * U * mag)


def filter_velocity(case, g, u, v, w):
    """Dual version of sgs.test_filter_velocity (each component on its own grid; ghosts of
    the result as the unfiltered field's strain ghosts)."""
    n = g.nz
    I = slice(1, n + 1)
    out = []
    for a, cy in ((u, True), (v, False)):
        f = D(np.zeros_like(a.v), np.zeros_like(a.e))
        r = filter_centre(case, g, a.map(lambda x: x[I]), centred_y=cy)
        f.v[I], f.e[I] = r.v, r.e
        out.append(f)
    wv = _fxy(w.v, g, True, False)
    wm = _fxy(np.abs(w.v), g, True, True)
    we = _fxy(w.e, g, True, True)
    f = D(np.zeros_like(w.v), np.zeros_like(w.e))
    f.v[I] = 0.25 * wv[0:n] + 0.5 * wv[1:n + 1] + 0.25 * wv[2:n + 2]
    f.e[I] = (0.25 * we[0:n] + 0.5 * we[1:n + 1] + 0.25 * we[2:n + 2]
              + 35.0 * U * (0.25 * wm[0:n] + 0.5 * wm[1:n + 1] + 0.25 * wm[2:n + 2]))
    out.append(f)
    uf, vf, wf = out
    if case.zbc == ZBC_PERIODIC:
        for a in (uf, vf, wf):
            for arr in (a.v, a.e):
                arr[0], arr[n + 1] = arr[n], arr[1]
    else:
        for arr in (wf.v, wf.e):
            arr[0] = 0.0
            arr[n] = 0.0
            arr[n + 1] = 0.0
        if case.zbc != ZBC_WALLMODEL:
            for a in (uf, vf):
                a.v[0], a.v[n + 1] = -a.v[1], -a.v[n]
                a.e[0], a.e[n + 1] = a.e[1], a.e[n]
    if g.ywalls:
        ny = g.ny
        vf.v[:, ny - 1:] = 0.0
        vf.e[:, ny - 1:] = 0.0
        if case.zbc != ZBC_WALLMODEL:
            for a in (uf, wf):
                a.v[:, ny + 1], a.v[:, ny] = -a.v[:, 0], -a.v[:, ny - 1]
                a.e[:, ny + 1], a.e[:, ny] = a.e[:, 0], a.e[:, ny - 1]
    return uf, vf, wf


# ---------------------------------------------------------------- summation depths
def _depth(n):
    return int(math.ceil(math.log2(max(n, 2))))


def plane_sum_depth(case, g):
    """Depth of the summation trees of the plane (x-line, volume) sums: the oracle's numpy
    reduction (pairwise along the contiguous axis: at most log2(n) + 20 levels, plus one level
    per row when the outer axes are not merged) and the kernel's (16-lane row trees, then the
    four rows of a wave added in turn, each thread's strided share of the per-wave partials
    of 32 x 8 tiles, a 256-thread block tree); the larger."""
    nx, ny, nz = g.nx, g.ny, g.nz
    ntile = ((nx + 31) // 32) * ((ny + 7) // 8)
    if g.ywalls:
        d_or = _depth(nx) + 20
        d_gpu = 5 + (nx + 31) // 32
    elif case.zbc == ZBC_PERIODIC:
        d_or = nz * ny + _depth(nx) + 20
        d_gpu = 7 + (nz * ntile * 4 + 255) // 256 + 8
    else:
        d_or = ny + _depth(nx) + 20
        d_gpu = 7 + (ntile * 4 + 255) // 256 + 8
    return max(d_or, d_gpu)


# ---------------------------------------------------------------- the dynamic procedure
def nut_difference_bound(case, g, u, v, w):
    """Per-cell bound on the difference of two float64 evaluations of the dynamic model's
    nu_t = c_s Delta^2 |S| from the same ghosted velocity (the oracle state's arrays), shape
    (nz, rows, nx); also returns the per-plane (per-line) coefficient difference bound and
    the coefficient itself (the value parts: the oracle's c_s up to its own rounding)."""
    n = g.nz
    I, Im = slice(1, n + 1), slice(0, n)
    U3 = [D(a) for a in (u, v, w)]
    us, vs, ws = strain_ghosts(case, g, *U3)
    s = centre_strain(g, us, vs, ws)
    smag = strain_magnitude(s)
    uI = U3[0].map(lambda a: a[I])
    vI = U3[1].map(lambda a: a[I])
    uc = scale(add(uI, uI.map(xm)), 0.5, exact=True)
    vc = scale(add(vI, vI.map(ym)), 0.5, exact=True)
    wc = scale(add(U3[2].map(lambda a: a[I]), U3[2].map(lambda a: a[Im])), 0.5, exact=True)
    vel = (uc, vc, wc)
    F = lambda q: filter_centre(case, g, q)
    fvel = [F(q) for q in vel]
    uf, vf, wf = filter_velocity(case, g, *U3)
    st = centre_strain(g, *strain_ghosts(case, g, uf, vf, wf))
    stmag = strain_magnitude(st)
    d2x2 = col(2.0 * g.delta() ** 2)
    alpha2 = _alpha2(case, g)
    lm_terms, mm_terms, wts = [], [], []
    for c, (a, b) in enumerate(PAIRS):
        L = add(F(mul(vel[a], vel[b])), mul(fvel[a], fvel[b]), -1.0)
        T = scale(mul(stmag, st[c]), alpha2)
        M = scale(add(F(mul(smag, s[c])), T, -1.0), d2x2)
        lm_terms.append(mul(L, M))
        mm_terms.append(mul(M, M))
        wts.append(1.0 if a == b else 2.0)
    lm = wsum(lm_terms, wts)
    mm = wsum(mm_terms, wts)
    depth = plane_sum_depth(case, g)
    if g.ywalls:
        red = lambda q: q.sum(axis=2)
    elif case.zbc == ZBC_PERIODIC:
        red = lambda q: np.full(n, q.sum())
    else:
        red = lambda q: q.sum(axis=(1, 2))
    a, b = red(lm.v), red(mm.v)
    ea = red(lm.e) + depth * U * red(np.abs(lm.v))
    eb = red(mm.e) + depth * U * red(np.abs(mm.v))
    if g.ywalls:
        for q in (a, b, ea, eb):
            q[:, g.ny:] = 0.0   # the ghost rows' lines carry no coefficient
    den = b - 2.0 * eb
    with np.errstate(divide="ignore", invalid="ignore"):
        cbar = np.where(den > 0.0, np.maximum(a + 2.0 * ea, 0.0) / np.where(den > 0.0, den, 1.0), np.inf)
        dc = np.where(den > 0.0, 2.0 * (ea + cbar * eb) / np.where(den > 0.0, den, 1.0) + 2.0 * U * cbar, np.inf)
    # planes where both sides see <M M> = 0 exactly (an at-rest plane) have c_s = 0 on both
    zero = (b == 0.0) & (eb == 0.0)
    cbar = np.where(zero, 0.0, cbar)
    dc = np.where(zero, 0.0, dc)
    d2 = g.delta() ** 2
    if g.ywalls:
        cb, dcc, dd = cbar[:, :, None], dc[:, :, None], col(d2)
    else:
        cb, dcc, dd = col(cbar), col(dc), col(d2)
    nut_bar = cb * dd * smag.v
    bound = dd * (smag.v * dcc + cb * 2.0 * smag.e) + 4.0 * U * nut_bar
    with np.errstate(divide="ignore", invalid="ignore"):
        cs = np.where(b > 0.0, np.maximum(a / np.where(b > 0.0, b, 1.0), 0.0), 0.0)
    return bound, dc, cs
