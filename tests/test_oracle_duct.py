"""Pins of the square-duct oracle (Sec. 4.4: walls in y and z, periodic x; R35-R38, R40).

- The duct Poisson solve against the dense matrix of the oracle's own divergence and
  gradient with the Neumann ghost rows (brute force on a tiny grid) and against single
  eigenmodes (cosine in y, Fourier in x, a z eigenvector), whose solution is the mode over
  its eigenvalue.
- The discrete laminar duct flow, solved directly, is a fixed point of the substep.
- Exchanging y and z on a square duct with uniform spacing maps a state to another state,
  and the substep commutes with that exchange: every y-wall rule must equal its z-wall
  counterpart (ghost rows, wall model, van Driest, Poisson, forcing, and for the dynamic
  model the test filter's wall rows, alpha at the walls and corners, and the averages along
  x lines, whose coefficients must form a symmetric (z, y) array).
- The y-wall model on a profile u(y) returns the log-law stress at the interpolated
  velocity, found by bisection.
- The learned closure's inputs (R40): they commute with the exchange of y and z; a single
  constant velocity gradient gives the closed-form invariants at every cell, wall rows
  included; y+ at hand-worked cells takes the nearest wall in its own units.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import bc, ops, poisson, substep as S
from oracle.case import ZBC_NOSLIP, ZBC_WALLMODEL, YBC_WALL, SGS_NONE, SGS_SMAG, SGS_SMAG_VD, SGS_DSM
from synth import duct_field


def _duct(nx=6, ny=6, nz=5, lx=1.5, ly=2.0, lz=2.0, **kw):
    case = oracle.Case(nx, ny, nz, lx, ly, lz, ybc=YBC_WALL, **kw)
    return case, oracle.Grid(case)


def _apply_dg(case, g, phi_int):
    """D G phi with the Neumann ghost rows and planes, from ops only."""
    n = g.nz
    phi = np.zeros((n + 2, g.nys, g.nx))
    phi[1:n + 1, :g.ny] = phi_int
    bc.fill_scalar(case, g, phi)
    gx, gy, gz = ops.gradient(g, phi)
    U, V, W = (np.zeros_like(phi) for _ in range(3))
    U[1:n + 1], V[1:n + 1], W[1:n + 1] = gx, gy, gz
    V[:, g.ny - 1:] = 0.0      # zero flux through the y walls
    W[n] = 0.0                 # and the top z wall (W[0] = 0 already)
    return ops.divergence(g, U, V, W)[:, :g.ny]


@pytest.mark.parametrize("beta", [0.0, 1.4])
def test_duct_poisson_dense(beta):
    case, g = _duct(nx=4, ny=6, nz=5, zbc=ZBC_NOSLIP, beta=beta)
    N = g.nz * g.ny * g.nx
    A = np.zeros((N, N))
    for e in range(N):
        x = np.zeros(N)
        x[e] = 1.0
        A[:, e] = _apply_dg(case, g, x.reshape(g.nz, g.ny, g.nx)).ravel()
    rng = np.random.default_rng(5)
    f = rng.standard_normal((g.nz, g.ny, g.nx))
    dzf = g.dzf[1:g.nz + 1][:, None, None]
    f -= np.sum(f * dzf) / (np.sum(dzf) * g.nx * g.ny)          # solvability (flux balance)
    fs = np.zeros((g.nz, g.nys, g.nx))
    fs[:, :g.ny] = f
    phi = poisson.solve(g, fs)
    assert np.all(phi[:, g.ny:] == 0.0)
    r = A @ phi[:, :g.ny].ravel() - f.ravel()
    assert np.max(np.abs(r)) < 1e-12 * np.max(np.abs(A)) * np.max(np.abs(phi))
    ref = np.linalg.lstsq(A, f.ravel(), rcond=None)[0].reshape(g.nz, g.ny, g.nx)
    ref -= np.sum(ref * dzf) / (np.sum(dzf) * g.nx * g.ny)
    assert np.max(np.abs(phi[:, :g.ny] - ref)) < 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("l,m", [(1, 0), (0, 2), (2, 3), (1, 5)])
def test_duct_poisson_single_mode(l, m):
    """f = cos(2 pi l x_i / nx) cos(pi m (j + 1/2) / ny) q(z) with q an eigenvector of the z
    operator (eigenvalue mu): phi = f / (lambda_x + lambda_y + mu)."""
    case, g = _duct(nx=8, ny=6, nz=7, zbc=ZBC_NOSLIP, beta=1.2)
    a, b, c = poisson.z_coefficients(g)
    Az = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
    mu, vecs = np.linalg.eig(Az)
    o = np.argsort(mu.real)
    q = vecs[:, o[1]].real                        # a non-constant eigenvector
    lam = (-(4.0 / g.dx ** 2) * math.sin(math.pi * l / g.nx) ** 2
           - (4.0 / g.dy ** 2) * math.sin(math.pi * m / (2 * g.ny)) ** 2 + mu[o[1]].real)
    xi = np.cos(2 * np.pi * l * np.arange(g.nx) / g.nx)
    yj = np.cos(np.pi * m * (np.arange(g.ny) + 0.5) / g.ny)
    f = q[:, None, None] * yj[None, :, None] * xi[None, None, :]
    fs = np.zeros((g.nz, g.nys, g.nx))
    fs[:, :g.ny] = f
    phi = poisson.solve(g, fs)[:, :g.ny]
    dzf = g.dzf[1:g.nz + 1][:, None, None]
    want = f / lam
    want -= np.sum(want * dzf) / (np.sum(dzf) * g.nx * g.ny)
    assert np.max(np.abs(phi - want)) < 1e-12 * np.max(np.abs(want))


def _laminar_duct(case, g, G):
    """Solve nu (L_yy + L_zz) u = -G on the (k, j) cross-section with no-slip ghosts (odd in
    y and z), by a dense solve; returns u (nz, ny)."""
    n, ny = g.nz, g.ny
    N = n * ny
    A = np.zeros((N, N))
    for e in range(N):
        x = np.zeros(N)
        x[e] = 1.0
        u = np.zeros((n + 2, g.nys, 1))
        u[1:n + 1, :ny, 0] = x.reshape(n, ny)
        u[0], u[n + 1] = -u[1], -u[n]
        u[:, ny + 1], u[:, ny] = -u[:, 0], -u[:, ny - 1]
        lap = ops.lap_z_centre(g, u) + (np.roll(u[1:n + 1], -1, 1) - 2 * u[1:n + 1] + np.roll(u[1:n + 1], 1, 1)) / g.dy ** 2
        A[:, e] = case.nu * lap[:, :ny, 0].ravel()
    return np.linalg.solve(A, -G * np.ones(N)).reshape(n, ny)


def test_laminar_duct_is_a_fixed_point():
    case, g = _duct(nx=4, ny=8, nz=6, lx=1.0, ly=2.0, lz=2.0, zbc=ZBC_NOSLIP, beta=1.3, nu=0.05,
                    sgs=SGS_NONE, ubulk=1.0)
    prof = _laminar_duct(case, g, 1.0)
    dzf = g.dzf[1:g.nz + 1]
    ub = np.sum(prof * dzf[:, None]) / (np.sum(dzf) * g.ny)
    prof /= ub
    u = np.zeros((g.nz + 2, g.nys, g.nx))
    u[1:g.nz + 1, :g.ny] = prof[:, :, None]
    v, w = np.zeros_like(u), np.zeros_like(u)
    st = S.initial_state(case, g, u, v, w)
    dt = 0.8 * S.time_step(case, g, st, 0.5)
    for k in range(3):
        st = S.substep(case, g, st, k, dt)
    I, J = slice(1, g.nz + 1), slice(0, g.ny)
    assert np.max(np.abs(st.u[I, J] - u[I, J])) < 1e-13
    assert np.max(np.abs(st.v[I, J])) < 1e-13 and np.max(np.abs(st.w[I, J])) < 1e-13


def _swap(g, u, v, w, p):
    """Exchange y and z on a square duct with uniform spacing (ny = nz, dy = dz): a cell
    (k, j) goes to (j + 1, k - 1); v and w exchange roles (v at y-face j goes to the w face
    j + 1, w at z-face k to the v face k - 1); ghost planes and rows are refilled later."""
    n = g.nz
    out = [np.zeros_like(u) for _ in range(4)]
    for k in range(1, n + 1):
        for j in range(g.ny):
            out[0][j + 1, k - 1] = u[k, j]
            out[3][j + 1, k - 1] = p[k, j]
            out[2][j + 1, k - 1] = v[k, j]
            out[1][j + 1, k - 1] = w[k, j]
    return out


@pytest.mark.parametrize("zbc,sgs,h_wm", [(ZBC_NOSLIP, SGS_SMAG_VD, 0.0), (ZBC_WALLMODEL, SGS_SMAG_VD, 0.0),
                                          (ZBC_WALLMODEL, SGS_SMAG, 0.45), (ZBC_NOSLIP, SGS_DSM, 0.0),
                                          (ZBC_WALLMODEL, SGS_DSM, 0.45)])
def test_substep_commutes_with_exchanging_y_and_z(zbc, sgs, h_wm):
    case, g = _duct(nx=6, ny=6, nz=6, lx=2.0, ly=2.0, lz=2.0, zbc=zbc, nu=2e-3, sgs=sgs, cs=0.12,
                    ubulk=1.0, h_wm=h_wm)
    u, v, w = duct_field(g.nx, g.ny, g.nz, g.zc, 2.0, 2.0, seed=11)
    p = np.zeros_like(u)
    # symmetrise the start: average the field with its exchanged image
    su, sv, sw, _ = _swap(g, u, v, w, p)
    u, v, w = 0.5 * (u + su), 0.5 * (v + sv), 0.5 * (w + sw)
    v[:, g.ny - 1] = 0.0
    w[g.nz] = 0.0
    st = S.initial_state(case, g, u, v, w)
    dt = S.time_step(case, g, st, 0.5)
    I, J = slice(1, g.nz + 1), slice(0, g.ny)
    for k in range(3):
        st = S.substep(case, g, st, k, dt)
        tu, tv, tw, tp = _swap(g, st.u, st.v, st.w, st.p - st.p[I, J].mean())
        pm = st.p - st.p[I, J].mean()
        for a, b in ((tu, st.u), (tv, st.v), (tw, st.w), (tp, pm)):
            scale = max(np.max(np.abs(b[I, J])), 1e-300)
            assert np.max(np.abs(a[I, J] - b[I, J])) < 1e-12 * max(scale, 1.0), k
        assert np.max(np.abs(st.v[:, g.ny - 1])) == 0.0
        tn = _swap(g, st.nut, st.nut, st.nut, st.nut)[0]
        assert np.max(np.abs(tn[I, J] - st.nut[I, J])) < 1e-12 * np.max(np.abs(st.nut[I, J])), k
        if sgs == SGS_DSM:
            # x-line coefficients: line (k, j) goes to line (j + 1, k - 1)
            cs = st.cs[:, :g.ny]
            assert cs.shape == (g.nz, g.ny) and np.max(cs) > 0.0
            assert np.max(np.abs(cs - cs.T)) < 1e-10 * np.max(cs), k
    if zbc == ZBC_WALLMODEL:
        # the y-wall stress at (k, i) equals the z-wall stress at (j = k - 1, i)
        txb = st.tau[0][:g.ny]
        txl = st.tauy[0][1:g.nz + 1]
        assert np.max(np.abs(txb - txl)) < 1e-12 * np.max(np.abs(txb))


def _loglaw_utau(U, h, nu, kappa, B):
    lo, hi = 1e-12, 10.0 * U + 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        f = mid * (math.log(mid * h / nu) / kappa + B) - U
        if f > 0.0 and mid > nu / h * math.exp(-kappa * B - 1.0):
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("h_wm", [0.0, 0.37])
def test_y_wall_model_on_a_profile(h_wm):
    case, g = _duct(nx=4, ny=10, nz=6, lx=1.0, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL, nu=1e-4, h_wm=h_wm)
    yc = g.yc
    prof = 1.0 + 0.3 * np.sin(1.3 * yc) + 0.1 * yc          # not symmetric: the walls differ
    u = np.zeros((g.nz + 2, g.nys, g.nx))
    u[1:g.nz + 1, :g.ny] = prof[None, :, None]
    w = np.zeros_like(u)
    tauy, _, _ = bc.wall_stress_y(case, g, u, w, None)
    for name, tau, dist in (("lo", tauy[0], yc), ("hi", tauy[2], g.ly - yc)):
        h = h_wm if h_wm > 0 else dist[0 if name == "lo" else g.ny - 1]
        Uh = np.interp(h, dist[::-1], prof[::-1]) if name == "hi" else np.interp(h, dist, prof)
        ut = _loglaw_utau(Uh, h, case.nu, case.kappa, case.bconst)
        assert np.max(np.abs(tau[1:g.nz + 1] - ut * ut)) < 1e-10 * ut * ut, name
        assert np.all(tau[0] == 0.0) and np.all(tau[g.nz + 1] == 0.0)
    assert np.all(tauy[1] == 0.0) and np.all(tauy[3] == 0.0)


# ---------------------------------------------------------------- learned closure inputs (R40)
def _features(case, g, st, ut4):
    from oracle import mlp as OM, sgs as OS
    s6 = OS.model_strain(case, g, st.u, st.v, st.w)
    return OM.raw_features(case, g, st.u, st.v, st.w, s6, ut4)


@pytest.mark.parametrize("zbc", [ZBC_NOSLIP, ZBC_WALLMODEL])
def test_learned_inputs_commute_with_exchanging_y_and_z(zbc):
    """The invariants are unchanged by the reflection that exchanges y and z, and y+ follows
    the walls: the inputs of the exchanged state, with the friction velocities of the y and
    z walls exchanged, are the transposed (z, y) inputs of the original one."""
    case, g = _duct(nx=6, ny=6, nz=6, lx=2.0, ly=2.0, lz=2.0, zbc=zbc, nu=2e-3, sgs=SGS_DSM)
    u, v, w = duct_field(g.nx, g.ny, g.nz, g.zc, 2.0, 2.0, seed=5, noise=0.3)
    st = S.initial_state(case, g, u, v, w)
    su, sv, sw, _ = _swap(g, st.u, st.v, st.w, st.p)
    st2 = S.initial_state(case, g, su, sv, sw)
    ut4 = (0.031, 0.047, 0.053, 0.029)
    f = _features(case, g, st, ut4)
    f2 = _features(case, g, st2, (ut4[2], ut4[3], ut4[0], ut4[1]))
    assert f.shape == (g.nz, g.ny, g.nx, 7)
    scale = np.max(np.abs(f), axis=(0, 1, 2))
    assert np.all(scale[:6] > 0.0)
    d = np.abs(f2.transpose(1, 0, 2, 3) - f)
    assert np.all(np.max(d, axis=(0, 1, 2)) <= 1e-12 * np.maximum(scale, 1.0))


@pytest.mark.parametrize("grad", ["dudz", "dudy", "dwdy"])
def test_learned_inputs_of_a_single_velocity_gradient(grad):
    """A flow with one constant off-diagonal gradient G has S and Omega with entries +-G/2 in
    one pair, n = |G|, so the five invariants are (1/2, -1/2, 0, 0, -1/8) at every cell whose
    stencil sees the linear field, the wall rows included (the y strain ghosts of R9 extend
    u and w linearly; the z ones extend u and v).  w = b y vanishes on the z-wall faces, so
    its check leaves out the first and last planes."""
    case, g = _duct(nx=4, ny=8, nz=6, lx=1.0, ly=2.0, lz=1.5, zbc=ZBC_WALLMODEL, beta=1.2, nu=1e-3,
                    sgs=SGS_DSM)
    n = g.nz
    u, v, w = (np.zeros((n + 2, g.nys, g.nx)) for _ in range(3))
    zc = g.zc[1:n + 1][:, None, None]
    yc = g.yc[None, :, None]
    if grad == "dudz":
        u[1:n + 1, :g.ny] = 0.7 * zc + 0.0 * yc
    elif grad == "dudy":
        u[1:n + 1, :g.ny] = -1.3 * yc + 0.0 * zc
    else:
        w[1:n, :g.ny] = 0.9 * yc + 0.0 * g.zf[1:n][:, None, None]
    st = S.initial_state(case, g, u, v, w)
    f = _features(case, g, st, (0.05, 0.05, 0.05, 0.05))
    ks = slice(1, n - 1) if grad == "dwdy" else slice(0, n)
    ref = np.array([0.5, -0.5, 0.0, 0.0, -0.125])
    assert np.max(np.abs(f[ks, :, :, :5] - ref)) < 1e-12


def test_learned_y_plus_takes_the_nearest_wall_in_its_own_units():
    """R40: y+ = min over the four walls of d_w u_tau,w / nu; with friction velocities
    (1, 2, 3, 4) (z bottom, z top, y = 0, y = ly) on a uniform 8 x 8 section of side 2
    (spacing 1/4), checked at cells worked by hand."""
    case, g = _duct(nx=4, ny=8, nz=8, lx=1.0, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL, nu=0.5, sgs=SGS_DSM)
    u, v, w = duct_field(g.nx, g.ny, g.nz, g.zc, 2.0, 2.0, seed=3)
    st = S.initial_state(case, g, u, v, w)
    f = _features(case, g, st, (1.0, 2.0, 3.0, 4.0))[..., 5]
    assert np.all(f == f[:, :, :1])
    # (plane, row): distances (z bottom, z top, y = 0, y = ly) -> the smallest product / nu
    cases = {(0, 7): 0.125 * 1.0 / 0.5,                 # z bottom 1/8 x 1 beats y = ly 1/8 x 4
             (4, 7): 0.125 * 4.0 / 0.5,                 # mid-height: y = ly, 1/8 x 4 = 1/2
             (7, 3): 0.125 * 2.0 / 0.5,                 # z top 1/8 x 2
             (3, 0): 0.125 * 3.0 / 0.5,                 # y = 0, 1/8 x 3 beats z bottom 7/8 x 1
             (1, 1): 0.375 * 1.0 / 0.5}                 # z bottom 3/8 x 1 beats y = 0 3/8 x 3
    for (k, j), val in cases.items():
        assert abs(f[k, j, 0] - val) < 1e-14, (k, j, f[k, j, 0], val)
