"""Pins of the oracle's eddy-viscosity models: closed forms on uniform shear, the
dynamic model's invariances and its laminar switch-off, and a plain-loop re-derivation
of the dynamic procedure on tiny grids."""
import math

import numpy as np
import pytest

from oracle import Case, Grid, bc, sgs
from oracle.case import (ZBC_PERIODIC, ZBC_NOSLIP, ZBC_WALLMODEL, SGS_SMAG, SGS_SMAG_VD,
                         SGS_DSM)
from oracle.substep import initial_state
from synth import uniform_shear_field, random_state


def _shear_case(zbc, sgs_model, beta=1.4):
    return Case(8, 6, 12, 2 * np.pi, np.pi, 2.0, zbc=zbc, beta=beta, nu=1e-3,
                sgs=sgs_model, cs=0.1)


def test_smagorinsky_uniform_shear_closed_form():
    """u = S0 z, v = w = 0: |S| = |S0| and nu_t = (C_s Delta)^2 |S0| in every cell whose
    strain stencil sees the linear profile (with the one-sided wall-model strain ghosts
    that is every cell)."""
    s0 = 2.5
    case = _shear_case(ZBC_WALLMODEL, SGS_SMAG)
    g = Grid(case)
    u, v, w = uniform_shear_field(8, 6, 12, g.zc, s0)
    st = initial_state(case, g, u, v, w)
    expect = (case.cs * g.delta()) ** 2 * s0
    assert np.allclose(st.nut[1:g.nz + 1], expect[:, None, None], rtol=1e-13, atol=0)


def test_smagorinsky_noslip_lower_half():
    """No-slip ghosts reproduce the linear profile at the bottom wall (u_0 = -u_1 = S0 zc_0)."""
    s0 = -1.5
    case = _shear_case(ZBC_NOSLIP, SGS_SMAG)
    g = Grid(case)
    u, v, w = uniform_shear_field(8, 6, 12, g.zc, s0)
    st = initial_state(case, g, u, v, w)
    expect = (case.cs * g.delta()) ** 2 * abs(s0)
    n = g.nz
    assert np.allclose(st.nut[1:n], expect[:n - 1, None, None], rtol=1e-13, atol=0)


def test_van_driest_closed_form():
    """With no-slip walls and u = S0 z the bottom-wall stress is nu S0, so
    u_tau = sqrt(nu S0) and D = 1 - exp(-zc u_tau / (25 nu)) in the lower half."""
    s0 = 3.0
    case = _shear_case(ZBC_NOSLIP, SGS_SMAG_VD)
    g = Grid(case)
    u, v, w = uniform_shear_field(8, 6, 12, g.zc, s0)
    st = initial_state(case, g, u, v, w)
    ut = math.sqrt(case.nu * s0)
    n = g.nz
    for k in range(1, n // 2 + 1):
        d = 1.0 - math.exp(-g.zc[k] * ut / case.nu / 25.0)
        expect = (case.cs * g.delta()[k - 1] * d) ** 2 * s0
        assert np.allclose(st.nut[k], expect, rtol=1e-12, atol=0)


@pytest.mark.parametrize("zbc", [ZBC_NOSLIP, ZBC_WALLMODEL])
def test_dsm_switches_off_in_one_dimensional_shear(zbc):
    """Sec. 2.1: the dynamic model vanishes in laminar flow.  For u = U(z), v = w = 0,
    L_ij = 0 except L_11 (F(u^2) - F(u)^2) while M_11 = 0 (S_11 = 0), so <L M> = 0."""
    case = _shear_case(zbc, SGS_DSM)
    g = Grid(case)
    u, v, w = uniform_shear_field(8, 6, 12, g.zc, 1.0)
    u[1:g.nz + 1] = (1.5 * (1.0 - (g.zc[1:g.nz + 1] - 1.0) ** 2))[:, None, None]
    st = initial_state(case, g, u, v, w)
    assert np.all(st.cs == 0.0)
    assert np.all(st.nut == 0.0)


def _random_channel(case, seed):
    g = Grid(case)
    u, v, w, _ = random_state(case.nx, case.ny, case.nz, seed)
    return g, u, v, w


@pytest.mark.parametrize("zbc", [ZBC_PERIODIC, ZBC_NOSLIP, ZBC_WALLMODEL])
def test_dsm_galilean_and_scale_invariance(zbc):
    case = Case(8, 8, 8, 2.0, 2.0, 2.0, zbc=zbc, beta=1.2 if zbc else 0.0, nu=1e-3, sgs=SGS_DSM)
    g, u, v, w = _random_channel(case, 21)
    cs0, _, _, _ = sgs.dynamic_coefficient(case, g, *_ghosted(case, g, u, v, w))
    # Galilean: add a uniform wall-parallel velocity (w must stay zero on walls)
    u2, v2 = u.copy(), v.copy()
    u2[1:g.nz + 1] += 3.7
    v2[1:g.nz + 1] -= 1.1
    w2 = w.copy()
    if zbc == ZBC_PERIODIC:
        w2[1:g.nz + 1] += 0.6
    cs1, _, _, _ = sgs.dynamic_coefficient(case, g, *_ghosted(case, g, u2, v2, w2))
    if zbc == ZBC_NOSLIP:
        # no-slip ghosts are not Galilean invariant at the walls; interior planes are
        sl = slice(2, g.nz - 2)
        assert np.allclose(cs1[sl], cs0[sl], rtol=1e-9, atol=1e-14)
    else:
        assert np.allclose(cs1, cs0, rtol=1e-9, atol=1e-14)
    # scaling u -> a u leaves c_s unchanged (L ~ a^2, M ~ a^2)
    a = 3.0
    cs2, _, _, _ = sgs.dynamic_coefficient(case, g, *_ghosted(case, g, a * u, a * v, a * w))
    assert np.allclose(cs2, cs0, rtol=1e-11, atol=1e-15)
    assert np.any(cs0 > 0)


def _ghosted(case, g, u, v, w):
    u, v, w = u.copy(), v.copy(), w.copy()
    z = np.zeros((g.ny, g.nx))
    bc.fill_velocity(case, g, u, v, w, tau=(z, z, z, z))
    return u, v, w


# ------------------------------------------------------------------ plain-loop DSM
def _bruteforce_cs(case, g, u, v, w):
    """The dynamic procedure written with scalar loops and explicit index arithmetic,
    independently of the vectorised oracle (velocity ghosts must be filled)."""
    nx, ny, nz = g.nx, g.ny, g.nz
    dx, dy = g.dx, g.dy
    wm = case.zbc == ZBC_WALLMODEL
    per = case.zbc == ZBC_PERIODIC

    def U(k, j, i):
        return u[k, j % ny, i % nx]

    def V(k, j, i):
        return v[k, j % ny, i % nx]

    def W(k, j, i):
        return w[k, j % ny, i % nx]

    def ughost(arr, k, j, i):
        # strain ghosts: one-sided (linear extrapolation in z) with the wall model
        if wm and k == 0:
            return arr(1, j, i) - g.dzc[0] * (arr(2, j, i) - arr(1, j, i)) / g.dzc[1]
        if wm and k == nz + 1:
            return arr(nz, j, i) + g.dzc[nz] * (arr(nz, j, i) - arr(nz - 1, j, i)) / g.dzc[nz - 1]
        return arr(k, j, i)

    def strain(Uf, Vf, Wf, k, j, i):
        s11 = (Uf(k, j, i) - Uf(k, j, i - 1)) / dx
        s22 = (Vf(k, j, i) - Vf(k, j - 1, i)) / dy
        s33 = (Wf(k, j, i) - Wf(k - 1, j, i)) / g.dzf[k]
        s12 = s13 = s23 = 0.0
        for di in (0, -1):
            for dj in (0, -1):
                ii, jj = i + di, j + dj
                s12 += 0.125 * ((Uf(k, jj + 1, ii) - Uf(k, jj, ii)) / dy
                                + (Vf(k, jj, ii + 1) - Vf(k, jj, ii)) / dx)
        for di in (0, -1):
            for dk in (0, -1):
                ii, kk = i + di, k + dk
                s13 += 0.125 * ((ughost(Uf, kk + 1, j, ii) - ughost(Uf, kk, j, ii)) / g.dzc[kk]
                                + (Wf(kk, j, ii + 1) - Wf(kk, j, ii)) / dx)
        for dj in (0, -1):
            for dk in (0, -1):
                jj, kk = j + dj, k + dk
                s23 += 0.125 * ((ughost(Vf, kk + 1, jj, i) - ughost(Vf, kk, jj, i)) / g.dzc[kk]
                                + (Wf(kk, jj + 1, i) - Wf(kk, jj, i)) / dy)
        S = np.array([[s11, s12, s13], [s12, s22, s23], [s13, s23, s33]])
        return S, math.sqrt(2.0 * np.sum(S * S))

    # centre quantities on interior cells
    Sc = {}
    vel = {}
    for k in range(1, nz + 1):
        for j in range(ny):
            for i in range(nx):
                Sc[k, j, i] = strain(U, V, W, k, j, i)
                vel[k, j, i] = np.array([0.5 * (U(k, j, i) + U(k, j, i - 1)),
                                         0.5 * (V(k, j, i) + V(k, j - 1, i)),
                                         0.5 * (W(k, j, i) + W(k - 1, j, i))])

    wts = (0.25, 0.5, 0.25)

    def cval(q, k, j, i):
        """centred quantity with periodic wrap in x, y and the z ghost rule of the filter"""
        j, i = j % ny, i % nx
        if per:
            return q(((k - 1) % nz) + 1, j, i)
        if k == 0:
            return 2.0 * q(1, j, i) - q(2, j, i)
        if k == nz + 1:
            return 2.0 * q(nz, j, i) - q(nz - 1, j, i)
        return q(k, j, i)

    def filt(q, k, j, i):
        acc = 0.0
        for a, dk in zip(wts, (-1, 0, 1)):
            for b, dj in zip(wts, (-1, 0, 1)):
                for c, di in zip(wts, (-1, 0, 1)):
                    acc = acc + a * b * c * cval(q, k + dk, j + dj, i + di)
        return acc

    # filtered staggered velocity
    def filt_face_w(k, j, i):
        acc = 0.0
        for a, dk in zip(wts, (-1, 0, 1)):
            for b, dj in zip(wts, (-1, 0, 1)):
                for c, di in zip(wts, (-1, 0, 1)):
                    kk = k + dk
                    if per:
                        kk = ((kk - 1) % nz) + 1
                    acc += a * b * c * W(kk, j + dj, i + di)
        return acc

    uf = np.zeros_like(u)
    vf = np.zeros_like(v)
    wf = np.zeros_like(w)
    for k in range(1, nz + 1):
        for j in range(ny):
            for i in range(nx):
                uf[k, j, i] = filt(lambda kk, jj, ii: u[kk, jj, ii], k, j, i)
                vf[k, j, i] = filt(lambda kk, jj, ii: v[kk, jj, ii], k, j, i)
                wf[k, j, i] = filt_face_w(k, j, i)
    if per:
        for a in (uf, vf, wf):
            a[0], a[nz + 1] = a[nz], a[1]
    else:
        wf[nz] = 0.0
        wf[0] = 0.0
        if not wm:
            uf[0], uf[nz + 1] = -uf[1], -uf[nz]
            vf[0], vf[nz + 1] = -vf[1], -vf[nz]
    UF = lambda k, j, i: uf[k, j % ny, i % nx]
    VF = lambda k, j, i: vf[k, j % ny, i % nx]
    WF = lambda k, j, i: wf[k, j % ny, i % nx]

    lm = np.zeros(nz + 1)
    mm = np.zeros(nz + 1)
    for k in range(1, nz + 1):
        a2 = 4.0 if (per or 1 < k < nz) else 4.0 ** (2.0 / 3.0)
        d2 = (dx * dy * g.dzf[k]) ** (2.0 / 3.0)
        for j in range(ny):
            for i in range(nx):
                St, stm = strain(UF, VF, WF, k, j, i)
                for p in range(3):
                    for q in range(3):
                        L = (filt(lambda kk, jj, ii: vel[kk, jj, ii][p] * vel[kk, jj, ii][q], k, j, i)
                             - filt(lambda kk, jj, ii: vel[kk, jj, ii][p], k, j, i)
                             * filt(lambda kk, jj, ii: vel[kk, jj, ii][q], k, j, i))
                        M = 2.0 * d2 * (filt(lambda kk, jj, ii: Sc[kk, jj, ii][1] * Sc[kk, jj, ii][0][p, q], k, j, i)
                                        - a2 * stm * St[p, q])
                        lm[k] += L * M
                        mm[k] += M * M
    if per:
        tl, tm = lm.sum(), mm.sum()
        return np.full(nz, max(0.0, tl / tm) if tm > 0 else 0.0), np.full(nz, tl), np.full(nz, tm)
    cs = np.array([max(0.0, lm[k] / mm[k]) if mm[k] > 0 else 0.0 for k in range(1, nz + 1)])
    return cs, lm[1:], mm[1:]


@pytest.mark.parametrize("zbc", [ZBC_PERIODIC, ZBC_NOSLIP, ZBC_WALLMODEL])
def test_dsm_matches_plain_loops(zbc):
    """The unclipped plane sums <L M> and <M M> (the volume sums when z is periodic) and the
    clipped c_s of the vectorised oracle equal the plain loops.  The periodic field (seed 103)
    has <L M> > 0, so its coefficient is not clipped away."""
    case = Case(5, 4, 6, 1.0, 1.3, 2.0, zbc=zbc, beta=1.1 if zbc else 0.0, nu=1e-3, sgs=SGS_DSM)
    g = Grid(case)
    u, v, w, _ = random_state(5, 4, 6, 103 if zbc == ZBC_PERIODIC else 99)
    if zbc != ZBC_PERIODIC:
        u[1:7] += 2.0 * np.linspace(0, 1, 6)[:, None, None]    # some mean shear
    u, v, w = _ghosted(case, g, u, v, w)
    cs, _, slm, smm = sgs.dynamic_coefficient(case, g, u, v, w)
    ref, rlm, rmm = _bruteforce_cs(case, g, u, v, w)
    assert np.allclose(slm, rlm, rtol=1e-11, atol=1e-14 * np.max(np.abs(rlm)))
    assert np.allclose(smm, rmm, rtol=1e-11, atol=0)
    assert np.allclose(cs, ref, rtol=1e-11, atol=1e-15)
    if zbc == ZBC_PERIODIC:
        assert cs[0] > 0.0
    else:
        assert np.any(slm < 0) and np.any(cs > 0)


# ------------------------------------------------------------------ closed forms of the filter and of L, M
def _mode_phase(g, a, b, c):
    """Phase 2 pi (a i/nx + b j/ny + c k/nz) of the cell-centred index grid (nz, ny, nx)."""
    k, j, i = np.meshgrid(np.arange(1, g.nz + 1), np.arange(g.ny), np.arange(g.nx), indexing="ij")
    return 2 * np.pi * (a * i / g.nx + b * j / g.ny + c * k / g.nz)


def _transfer(g, a, b, c):
    """Transfer function of the (1/4, 1/2, 1/4) tensor-product filter on the mode (a, b, c):
    1/2 + cos(theta)/2 = cos^2(theta/2) per direction."""
    return (np.cos(np.pi * a / g.nx) * np.cos(np.pi * b / g.ny) * np.cos(np.pi * c / g.nz)) ** 2


@pytest.mark.parametrize("mode", [(1, 0, 0), (0, 2, 0), (0, 0, 3), (2, 1, 1), (3, 2, 5)])
def test_test_filter_transfer_function(mode):
    """R7 pinned by its transfer function: on a triply periodic grid every Fourier mode is an
    eigenfunction of the test filter with eigenvalue prod cos^2(pi m_d / N_d), for the
    cell-centred quantities and for each staggered velocity component."""
    case = Case(8, 6, 10, 1.0, 1.0, 1.0, zbc=ZBC_PERIODIC, sgs=SGS_DSM)
    g = Grid(case)
    ph = _mode_phase(g, *mode) + 0.3
    q = np.cos(ph)
    T = _transfer(g, *mode)
    assert np.allclose(sgs.test_filter_centre(case, q, g), T * q, rtol=0, atol=1e-14)
    u = np.zeros((g.nz + 2, g.ny, g.nx))
    v, w = u.copy(), u.copy()
    I = slice(1, g.nz + 1)
    u[I], v[I], w[I] = np.cos(ph + 0.1), np.sin(ph), np.cos(ph - 0.7)
    u, v, w = _ghosted(case, g, u, v, w)
    uf, vf, wf = sgs.test_filter_velocity(case, g, u, v, w)
    for f, a in ((uf, u), (vf, v), (wf, w)):
        assert np.allclose(f[I], T * a[I], rtol=0, atol=1e-14)


def test_leonard_tensor_closed_form():
    """Eq. lij on two Fourier modes.  With centre velocities uc = A cos(p1), vc = B cos(p2)
    and wc = 0 (u, v on their faces shifted by half a cell), products of modes are sums of
    modes, so with T the filter's transfer function:
      L11 = A^2/2 [1 - T(m1)^2 + (T(2 m1) - T(m1)^2) cos 2 p1],
      L12 = AB/2 [T(m1 + m2) cos(p1 + p2) + T(m1 - m2) cos(p1 - p2)] - AB T(m1) T(m2) cos p1 cos p2,
      L13 = L23 = L33 = 0."""
    case = Case(8, 6, 10, 1.0, 1.3, 0.7, zbc=ZBC_PERIODIC, sgs=SGS_DSM)
    g = Grid(case)
    m1, m2 = (1, 1, 0), (2, 0, 1)
    A, B = 1.3, -0.6
    p1, p2 = _mode_phase(g, *m1) + 0.2, _mode_phase(g, *m2) - 0.4
    u = np.zeros((g.nz + 2, g.ny, g.nx))
    v, w = u.copy(), u.copy()
    I = slice(1, g.nz + 1)
    # u[i] sits half a cell in x after the centre, v[j] half a cell in y after it
    ax, by = np.pi * m1[0] / g.nx, np.pi * m2[1] / g.ny
    u[I] = A / np.cos(ax) * np.cos(p1 + ax)
    v[I] = B / np.cos(by) * np.cos(p2 + by)
    u, v, w = _ghosted(case, g, u, v, w)
    L, _, _ = sgs.germano_tensors(case, g, u, v, w)
    T = lambda m: _transfer(g, *m)
    add = tuple(a + b for a, b in zip(m1, m2))
    sub = tuple(a - b for a, b in zip(m1, m2))
    dbl = tuple(2 * a for a in m1)
    l11 = 0.5 * A * A * (1 - T(m1) ** 2 + (T(dbl) - T(m1) ** 2) * np.cos(2 * p1))
    l12 = (0.5 * A * B * (T(add) * np.cos(p1 + p2) + T(sub) * np.cos(p1 - p2))
           - A * B * T(m1) * T(m2) * np.cos(p1) * np.cos(p2))
    l22 = 0.5 * B * B * (1 - T(m2) ** 2 + (T(tuple(2 * a for a in m2)) - T(m2) ** 2) * np.cos(2 * p2))
    assert np.allclose(L[0], l11, rtol=0, atol=1e-14)
    assert np.allclose(L[1], l22, rtol=0, atol=1e-14)
    assert np.allclose(L[3], l12, rtol=0, atol=1e-14)
    for c in (2, 4, 5):
        assert np.all(L[c] == 0.0)


@pytest.mark.parametrize("s0", [1.7, -0.8])
def test_model_tensor_plane_sums_on_uniform_shear(s0):
    """Eq. mij on u = S0 z (v = w = 0) between walls with uniform spacing and the wall model's
    one-sided strain ghosts: every linear profile passes the test filter unchanged (its z
    pass is the identity on the first layers, R9, and exact in between), so
    S~ = S = S0/2 in the 13 slot, |S| = |S~| = |S0| and
      M13 = 2 Delta^2 (1 - alpha^2) |S0| S0 / 2,  every other M_ij = 0,
    giving <M M>_k = 2 nx ny Delta_k^4 (1 - alpha_k^2)^2 S0^4 with alpha^2 = 4 inside and
    4^(2/3) on the first off-wall layers (2-D filter), and <L M>_k = 0 (M11 = 0 where
    L11 = F(u^2) - F(u)^2 is not)."""
    case = Case(6, 4, 8, 1.5, 0.9, 2.0, zbc=ZBC_WALLMODEL, beta=0.0, nu=1e-3, sgs=SGS_DSM)
    g = Grid(case)
    u, v, w = uniform_shear_field(6, 4, 8, g.zc, s0)
    u, v, w = _ghosted(case, g, u, v, w)
    _, _, slm, smm = sgs.dynamic_coefficient(case, g, u, v, w)
    n = g.nz
    alpha2 = np.full(n, 4.0)
    alpha2[0] = alpha2[n - 1] = 4.0 ** (2.0 / 3.0)
    d2 = (g.dx * g.dy * g.dzf[1:n + 1]) ** (2.0 / 3.0)
    ref = 2.0 * g.nx * g.ny * d2 ** 2 * (1.0 - alpha2) ** 2 * s0 ** 4
    assert np.allclose(smm, ref, rtol=1e-12, atol=0)
    assert np.all(slm == 0.0)
