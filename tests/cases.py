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
                          sgs=case.sgs, cs=case.cs, implicit_z=int(case.implicit_z),
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
