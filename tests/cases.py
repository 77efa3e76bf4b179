"""Shared helpers of the GPU parity tests: the same seeded inputs go to the CPU oracle and
to the HIP library, and fields are compared element by element."""
import sys

import numpy as np

import oracle
from oracle import substep as S
from synth import isotropic_field, channel_field, random_state


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_pair(nx, ny, nz, lx, ly, lz, **kw):
    """(oracle Case, Grid, library config) for one problem."""
    from paper_2411_09364_amd import les
    precision = kw.pop("precision", 0)
    case = oracle.Case(nx, ny, nz, lx, ly, lz, **kw)
    g = oracle.Grid(case)
    cfg = les.make_config(nx, ny, nz, lx, ly, lz, zbc=case.zbc, beta=case.beta, nu=case.nu,
                          sgs=case.sgs, cs=case.cs,
                          implicit_z=2 if case.implicit_3d else int(case.implicit_z),
                          precision=precision, ubulk=case.ubulk, h_wm=case.h_wm,
                          kappa=case.kappa, bconst=case.bconst)
    return case, g, cfg


def initial_fields(case, g, seed, kind):
    if kind == "iso":
        assert case.nx == case.ny == case.nz
        return isotropic_field(case.nx, seed=seed, k0=4.0)
    if kind == "channel":
        return channel_field(case.nx, case.ny, case.nz, g.zc, seed=seed)
    u, v, w, _ = random_state(case.nx, case.ny, case.nz, seed)
    if case.walls:
        w[case.nz] = 0.0
    return u, v, w


def rel_err(a, b, sl):
    ref = np.max(np.abs(b[sl]))
    return np.max(np.abs(a[sl] - b[sl])) / (ref if ref > 0 else 1.0)


def mean_free(p, g):
    n = g.nz
    I = slice(1, n + 1)
    dzf = g.dzf[I]
    m = np.sum(p[I] * dzf[:, None, None]) / (np.sum(dzf) * g.nx * g.ny)
    q = p.copy()
    q[I] -= m
    return q


def round32(*arrs):
    return tuple(np.asarray(a, dtype=np.float32).astype(np.float64) for a in arrs)


# Constant of the first-order rounding bound of the dynamic coefficient: covers the 27-term
# test-filter sums and the depth of the plane sums (pairwise on the CPU, tree on the GPU).
CS_ROUNDING_K = 64.0
UNIT_ROUNDOFF = 2.0 ** -53


def dsm_nut_check(case, g, st, nut, rel=1e-12):
    """Compare a dynamic-model nu_t with the oracle's plane by plane: the allowed difference
    on plane k is rel * max|nu_t| plus the propagated rounding bound of c_s(k)
    (oracle.sgs.coefficient_rounding_scale) times Delta_k^2 max|S| on that plane.
    Returns (ok, worst ratio of difference to allowance, largest bound-only allowance
    relative to max|nu_t|)."""
    from oracle import sgs
    from oracle.ops import strain_magnitude
    n = g.nz
    I = slice(1, n + 1)
    scale = sgs.coefficient_rounding_scale(case, g, st.u, st.v, st.w)
    smag = strain_magnitude(sgs.model_strain(case, g, st.u, st.v, st.w))
    ref = np.max(np.abs(st.nut[I]))
    d2 = g.delta() ** 2
    diff = np.max(np.abs(nut[I] - st.nut[I]), axis=(1, 2))
    bound = CS_ROUNDING_K * UNIT_ROUNDOFF * scale * d2 * np.max(smag, axis=(1, 2))
    allow = rel * ref + bound
    ratio = float(np.max(diff / allow))
    return ratio <= 1.0, ratio, float(np.max(bound) / ref) if ref > 0 else 0.0
