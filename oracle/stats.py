"""Long-run statistics of a channel run (Secs. 4.2 and 4.3 channel cases: mean velocity, resolved
Reynolds stresses, friction velocity, friction Reynolds number Re_tau = u_tau h / nu and
skin friction C_f = tau_w / (rho u_b^2 / 2); Eq. eps_f and Eq. error for the errors against
a reference; the standard uncertainty of C_f by batch means).  Test infrastructure only.

Readings (the paper names the quantities, not their discrete form):
  R32  samples are plane (x-y) sums of one state, accumulated over samples; every quantity
       is taken where its staggered components meet: u, u^2 at the u points (z_c(k)), v, v^2
       at the v points, w, w^2 at the top face z_f(k) of cell k, p and nu_t at the centres;
       uv on the (x, y) edge ((i+1) dx, (j+1) dy, z_c(k)) from the y-mean of u and the x-mean
       of v; uw on the (x, z) edge ((i+1) dx, (j+1/2) dy, z_f(k)) from the z-mean of u (cells
       k, k+1) and the x-mean of w; vw on the (y, z) edge likewise.  Covariances are the
       sample-and-plane mean of the product minus the product of the means of the two
       interpolated factors.  tau_w is the time mean of the plane-mean streamwise wall
       stress averaged over the two walls (wall model: its stress; no-slip: nu du/dz from the
       ghosts); u_b is the dzf-weighted mean of the mean-velocity profile; h = L_z / 2.
  R33  the paper estimates the uncertainty of C_f with a modified batch-means method whose
       details it does not give; plain batch means are used: the series of per-sample
       tau_w is cut into nb equal consecutive batches (the oldest samples beyond nb * floor(n
       / nb) dropped), sigma = std of the batch means (ddof 1) / sqrt(nb), scaled by 2 / u_b^2.
  R34  Eq. error integrates over y/h in [0.1, 1]; the profiles are known at their own points,
       so phi - phi_ref and phi_ref are taken piecewise linear between those points and the
       integrals are exact for that interpolant, clipped to [z0, z1].
  R39  Square duct (Sec. 4.4): x is the only homogeneous direction, so the sums run along x
       lines and the profiles are (z, y) cross-sections; the products sit on the same edges as
       in R32, and a covariance subtracts the product of the means of its two edge factors
       (the two-point means of the neighbouring lines' means).  tau_w is the perimeter mean
       of the streamwise wall stress: each wall's mean (over x and its own direction, the y
       walls weighted by dzf) weighted by the wall's length in the cross-section; u_b is the
       area mean of U; h = L_z / 2 (half the side of the square).
"""
import numpy as np

from .case import ZBC_PERIODIC, ZBC_WALLMODEL
from . import bc

QUANTITIES = ("u", "v", "w", "p", "nut", "uu", "vv", "ww", "uv", "uw", "vw")


def plane_sums(case, g, st):
    """Raw sums over (i, j) of the quantities of R32 for one state, array [11][nz] (row order
    QUANTITIES); plane k of the arrays is interior plane k + 1 (for w, uw, vw: face k + 1)."""
    n = g.nz
    out = np.zeros((len(QUANTITIES), n))
    for kk in range(1, n + 1):
        u, v, w = st.u[kk], st.v[kk], st.w[kk]
        u_up, v_up = st.u[kk + 1], st.v[kk + 1]   # ghost plane nz + 1 on the top face
        u_xy = 0.5 * (u + np.roll(u, -1, axis=0))          # y-mean of u: (i+1, j+1) edge
        v_xy = 0.5 * (v + np.roll(v, -1, axis=1))          # x-mean of v
        u_xz = 0.5 * (u + u_up)                             # z-mean of u: (i+1, j+1/2) at z_f
        w_xz = 0.5 * (w + np.roll(w, -1, axis=1))          # x-mean of w
        v_yz = 0.5 * (v + v_up)                             # z-mean of v: (i+1/2, j+1) at z_f
        w_yz = 0.5 * (w + np.roll(w, -1, axis=0))          # y-mean of w
        vals = (u, v, w, st.p[kk], st.nut[kk], u * u, v * v, w * w, u_xy * v_xy, u_xz * w_xz,
                v_yz * w_yz)
        for q, a in enumerate(vals):
            out[q, kk - 1] = np.sum(a)
    return out


def line_sums(case, g, st):
    """Duct (R39): sums over i of the quantities of R32, array [11][nz][ny] (row order
    QUANTITIES); line (k, j) is interior plane k + 1 (for w, uw, vw: face k + 1), row j."""
    n, ny = g.nz, g.ny
    out = np.zeros((len(QUANTITIES), n, ny))
    for kk in range(1, n + 1):
        u, v, w = st.u[kk], st.v[kk], st.w[kk]
        u_up, v_up = st.u[kk + 1], st.v[kk + 1]
        u_xy = 0.5 * (u + np.roll(u, -1, axis=0))      # row j + 1 of the stored rows (ghost at the top)
        v_xy = 0.5 * (v + np.roll(v, -1, axis=1))
        u_xz = 0.5 * (u + u_up)
        w_xz = 0.5 * (w + np.roll(w, -1, axis=1))
        v_yz = 0.5 * (v + v_up)
        w_yz = 0.5 * (w + np.roll(w, -1, axis=0))
        vals = (u, v, w, st.p[kk], st.nut[kk], u * u, v * v, w * w, u_xy * v_xy, u_xz * w_xz, v_yz * w_yz)
        for q, a in enumerate(vals):
            out[q, kk - 1] = np.sum(a[:ny], axis=1)
    return out


def perimeter_wall_stress(case, g, st):
    """Duct (R39): perimeter mean of the streamwise wall stress of one state."""
    n, ny = g.nz, g.ny
    if case.zbc == ZBC_WALLMODEL:
        txb, _, txt, _ = st.tau
        txl, _, txh, _ = st.tauy
    else:
        txb, _, txt, _ = bc.noslip_wall_stress(case, g, st.u, st.v)
        txl, _, txh, _ = bc.noslip_wall_stress_y(case, g, st.u, st.w)
    dzf = g.dzf[1:n + 1][:, None]
    zb, zt = float(np.mean(txb[:ny])), float(np.mean(txt[:ny]))
    yl = float(np.sum(txl[1:n + 1] * dzf) / (g.nx * g.lz))
    yh = float(np.sum(txh[1:n + 1] * dzf) / (g.nx * g.lz))
    return (g.ly * (zb + zt) + g.lz * (yl + yh)) / (2.0 * (g.ly + g.lz))


def wall_stress_sample(case, g, st):
    """Plane means of the streamwise wall stress at the bottom and top walls (R32): the wall
    model's stress, or nu du/dz from the no-slip ghosts; (0, 0) with periodic z."""
    if case.zbc == ZBC_PERIODIC:
        return 0.0, 0.0
    if case.zbc == ZBC_WALLMODEL:
        txb, _, txt, _ = st.tau
    else:
        txb, _, txt, _ = bc.noslip_wall_stress(case, g, st.u, st.v)
    return float(np.mean(txb)), float(np.mean(txt))


class Accumulator:
    """Running sums over samples (R32) and the per-sample wall-stress series (R33)."""

    def __init__(self, g):
        self.samples = 0
        self.sums = np.zeros((len(QUANTITIES), g.nz, g.ny) if g.ywalls else (len(QUANTITIES), g.nz))
        self.series = []

    def add(self, case, g, st):
        if g.ywalls:
            self.sums += line_sums(case, g, st)
            t = perimeter_wall_stress(case, g, st)
            self.series.append((t, t))
        else:
            self.sums += plane_sums(case, g, st)
            self.series.append(wall_stress_sample(case, g, st))
        self.samples += 1


def batch_means_sigma(x, nb):
    """Standard uncertainty of the mean of the series x by nb batches (R33); NaN if nb < 2
    or fewer samples than batches."""
    x = np.asarray(x, dtype=float)
    if nb < 2 or len(x) < nb:
        return float("nan")
    L = len(x) // nb
    xb = x[len(x) - nb * L:].reshape(nb, L).mean(axis=1)
    return float(np.std(xb, ddof=1) / np.sqrt(nb))


def finalize(case, g, acc, nb=8):
    """Profiles (dict of the means U, V, W, P, NUT and covariances uu, vv, ww, uv, uw, vw, each
    [nz]; [nz][ny] cross-sections for a duct) and scalars (dict: samples, tau_w, u_tau, re_tau,
    u_b, c_f, c_f_sigma)."""
    if g.ywalls:
        return _finalize_duct(case, g, acc, nb)
    n = g.nz
    N = acc.samples * g.nx * g.ny
    m = {q: acc.sums[i] / N for i, q in enumerate(QUANTITIES)}
    U, V, W = m["u"], m["v"], m["w"]
    per = case.zbc == ZBC_PERIODIC
    # mean of the z-interpolated u and v on face k (cells k, k+1); the top face of a wall run
    # carries w = 0, so its neighbour value does not enter
    Uup = np.append(U[1:], U[0] if per else U[n - 1])
    Vup = np.append(V[1:], V[0] if per else V[n - 1])
    prof = {"U": U, "V": V, "W": W, "P": m["p"], "NUT": m["nut"],
            "uu": m["uu"] - U * U, "vv": m["vv"] - V * V, "ww": m["ww"] - W * W,
            "uv": m["uv"] - U * V, "uw": m["uw"] - 0.5 * (U + Uup) * W,
            "vw": m["vw"] - 0.5 * (V + Vup) * W}
    dzf = g.dzf[1:n + 1]
    u_b = float(np.sum(U * dzf) / np.sum(dzf))
    ser = np.array(acc.series) if acc.series else np.zeros((0, 2))
    tw_series = 0.5 * (ser[:, 0] + ser[:, 1]) if len(ser) else np.zeros(0)
    tau_w = float(np.mean(tw_series)) if len(tw_series) else 0.0
    u_tau = float(np.sqrt(max(tau_w, 0.0)))
    h = 0.5 * case.lz
    sc = {"samples": acc.samples, "tau_w": tau_w, "u_tau": u_tau, "re_tau": u_tau * h / case.nu, "u_b": u_b,
          "c_f": 2.0 * tau_w / (u_b * u_b) if u_b != 0.0 else float("nan"),
          "c_f_sigma": 2.0 * batch_means_sigma(tw_series, nb) / (u_b * u_b) if u_b != 0.0 else float("nan")}
    return prof, sc


def _finalize_duct(case, g, acc, nb):
    """R39: cross-section profiles and perimeter-averaged wall quantities of a duct."""
    n, ny = g.nz, g.ny
    N = acc.samples * g.nx
    m = {q: acc.sums[i] / N for i, q in enumerate(QUANTITIES)}
    U, V, W = m["u"], m["v"], m["w"]
    # neighbour lines' means (row j + 1, plane k + 1); beyond the last row or plane the factor
    # they multiply is zero (v on the y wall face, w on the z wall face), any value will do
    Ujp = np.concatenate([U[:, 1:], U[:, -1:]], axis=1)
    Ukp = np.concatenate([U[1:], U[-1:]], axis=0)
    Vkp = np.concatenate([V[1:], V[-1:]], axis=0)
    Wjp = np.concatenate([W[:, 1:], W[:, -1:]], axis=1)
    prof = {"U": U, "V": V, "W": W, "P": m["p"], "NUT": m["nut"],
            "uu": m["uu"] - U * U, "vv": m["vv"] - V * V, "ww": m["ww"] - W * W,
            "uv": m["uv"] - 0.5 * (U + Ujp) * V, "uw": m["uw"] - 0.5 * (U + Ukp) * W,
            "vw": m["vw"] - 0.5 * (V + Vkp) * 0.5 * (W + Wjp)}
    dzf = g.dzf[1:n + 1][:, None]
    u_b = float(np.sum(U * dzf) / (ny * np.sum(dzf)))
    ser = np.array(acc.series) if acc.series else np.zeros((0, 2))
    tw_series = 0.5 * (ser[:, 0] + ser[:, 1]) if len(ser) else np.zeros(0)
    tau_w = float(np.mean(tw_series)) if len(tw_series) else 0.0
    u_tau = float(np.sqrt(max(tau_w, 0.0)))
    h = 0.5 * case.lz
    sc = {"samples": acc.samples, "tau_w": tau_w, "u_tau": u_tau, "re_tau": u_tau * h / case.nu, "u_b": u_b,
          "c_f": 2.0 * tau_w / (u_b * u_b) if u_b != 0.0 else float("nan"),
          "c_f_sigma": 2.0 * batch_means_sigma(tw_series, nb) / (u_b * u_b) if u_b != 0.0 else float("nan")}
    return prof, sc


def eps_f(cf, cf_ref):
    """Relative skin-friction error (Eq. eps_f)."""
    return (cf - cf_ref) / cf_ref


def eps_phi(z, phi, ref, z0, z1):
    """Relative profile error (Eq. error) over [z0, z1] (R34): z increasing, phi and ref at
    the points z; the integrands are the piecewise-linear interpolants."""
    z, phi, ref = (np.asarray(a, dtype=float) for a in (z, phi, ref))
    d = phi - ref
    num = 0.0
    den = 0.0
    for a in range(len(z) - 1):
        za, zb = z[a], z[a + 1]
        lo, hi = max(za, z0), min(zb, z1)
        if hi <= lo:
            continue
        ta, tb = (lo - za) / (zb - za), (hi - za) / (zb - za)
        da, db = d[a] + ta * (d[a + 1] - d[a]), d[a] + tb * (d[a + 1] - d[a])
        ra, rb = ref[a] + ta * (ref[a + 1] - ref[a]), ref[a] + tb * (ref[a + 1] - ref[a])
        num += (hi - lo) * (da * da + da * db + db * db) / 3.0
        den += (hi - lo) * 0.5 * (ra + rb)
    return float(np.sqrt(num) / abs(den))
