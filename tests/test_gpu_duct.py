"""GPU parity of the square duct (Sec. 4.4: walls in y and z, no-slip or the log-law wall
model on all four, periodic x, constant flow rate): the y ghost rows, the y-wall model, the
four-wall van Driest factor and the cosine transform in y, against the FP64 oracle on the
same seeded inputs.

Tolerances as in test_gpu_parity.py: FP64 1e-12 per substep (the mean-free pressure held to
the Poisson operator's conditioning bound), mixed 1e-5 (pressure on the |u|^2 scale).  Fields
are compared on every stored row of the interior planes, ghost rows included, so the ghost
rules are checked as well.  Sizes span several 32 x 8 tiles with ragged tails, radix-3
and radix-5 cosine lengths (the paper's duct grids have ny = 80, 120, 160, 320), stretched
and uniform z, both line forms of the y transform (ping-pong and in-place for long lines)
and the interpolated wall-model height in y and z.
"""
import numpy as np
import pytest

from oracle import substep as S, poisson as OP
from oracle.case import ZBC_NOSLIP, ZBC_WALLMODEL, YBC_WALL, SGS_NONE, SGS_SMAG, SGS_SMAG_VD, SGS_DSM
from tests.cases import (make_pair, initial_fields, rel_err, mean_free, say, round32, pressure_tolerance,
                         dsm_nut_check)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def les():
    import torch
    assert torch.cuda.is_available()
    from paper_2411_09364_amd import les as L
    return L


DUCT = dict(ybc=YBC_WALL, ubulk=1.0)

POISSON_CASES = [
    dict(nx=16, ny=12, nz=10, lx=3.2, ly=2.0, lz=2.0, zbc=ZBC_NOSLIP, beta=1.3),
    dict(nx=40, ny=24, nz=9, lx=4.0, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL),
    dict(nx=30, ny=80, nz=20, lx=4.0, ly=2.0, lz=2.0, zbc=ZBC_NOSLIP, beta=1.1),     # radix 5 (and 3)
    dict(nx=16, ny=320, nz=6, lx=1.0, ly=2.0, lz=2.0, zbc=ZBC_NOSLIP),                # in-place, radix 5
    dict(nx=8, ny=512, nz=5, lx=1.0, ly=4.0, lz=2.0, zbc=ZBC_NOSLIP, beta=1.0),   # in-place lines
    dict(nx=64, ny=96, nz=96, lx=6.4, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL),
]


@pytest.mark.parametrize("cfgd", POISSON_CASES)
def test_duct_poisson_matches_oracle(les, cfgd):
    say("duct poisson case", cfgd)
    case, g, cfg = make_pair(ybc=YBC_WALL, **dict(cfgd))
    rng = np.random.Generator(np.random.PCG64(23))
    n, ny = g.nz, g.ny
    f = np.zeros((n + 2, g.nys, g.nx))
    f[1:n + 1, :ny] = rng.standard_normal((n, ny, g.nx))
    dzf = g.dzf[1:n + 1]
    f[1:n + 1, :ny] -= np.sum(f[1:n + 1, :ny] * dzf[:, None, None]) / (np.sum(dzf) * g.nx * ny)
    ref = OP.solve(g, f[1:n + 1])
    solver = les.Solver(cfg)
    phi = solver.poisson(f)
    err = np.max(np.abs(phi[1:n + 1, :ny] - ref[:, :ny])) / np.max(np.abs(ref))
    tol = pressure_tolerance(g)
    say(f"  rel err {err:.2e} (tolerance {tol:.1e})")
    assert err < tol
    # ghost rows and planes: zero flux through every wall
    assert np.array_equal(phi[:, ny + 1], phi[:, 0]) and np.array_equal(phi[:, ny], phi[:, ny - 1])
    assert np.array_equal(phi[0, :ny], phi[1, :ny]) and np.array_equal(phi[n + 1, :ny], phi[n, :ny])
    solver.close()


SUBSTEP_CASES = [
    ("noslip vd stretched", dict(nx=16, ny=12, nz=10, lx=3.2, ly=2.0, lz=2.0, zbc=ZBC_NOSLIP, beta=1.3, nu=2e-3,
                                 sgs=SGS_SMAG_VD, cs=0.12), "duct"),
    ("wm smag h_wm", dict(nx=24, ny=16, nz=16, lx=6.4, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL, nu=1e-4, sgs=SGS_SMAG,
                          cs=0.1, h_wm=0.3), "duct"),
    ("wm vd ragged tiles", dict(nx=40, ny=20, nz=12, lx=4.0, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL, nu=1e-4,
                                sgs=SGS_SMAG_VD, cs=0.1), "duct"),
    ("wm vd cn-z", dict(nx=16, ny=12, nz=14, lx=3.2, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL, beta=1.2, nu=1e-3,
                        sgs=SGS_SMAG_VD, cs=0.1, implicit_z=True), "duct"),
    ("noslip cn-z vd", dict(nx=16, ny=12, nz=10, lx=3.2, ly=2.0, lz=2.0, zbc=ZBC_NOSLIP, beta=1.3, nu=2e-3,
                            sgs=SGS_SMAG_VD, cs=0.12, implicit_z=True), "duct"),
    ("noslip no model radix3 random", dict(nx=12, ny=24, nz=9, lx=1.0, ly=2.0, lz=2.0, zbc=ZBC_NOSLIP, beta=1.0,
                                           nu=5e-3, sgs=SGS_NONE), "random"),
    ("wm smag long y", dict(nx=8, ny=512, nz=6, lx=1.0, ly=4.0, lz=2.0, zbc=ZBC_WALLMODEL, nu=1e-3, sgs=SGS_SMAG,
                            cs=0.1), "duct"),
    ("wm vd radix5 paper cross-section", dict(nx=20, ny=80, nz=80, lx=1.28, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL,
                                              nu=5e-5, sgs=SGS_SMAG_VD, cs=0.1, h_wm=0.1), "duct"),
    # dynamic model: coefficients along x lines, 1-D test filter at the corners
    ("wm dsm ragged tiles", dict(nx=40, ny=20, nz=12, lx=4.0, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL, nu=1e-4,
                                 sgs=SGS_DSM), "duct"),
    ("noslip dsm stretched", dict(nx=16, ny=12, nz=10, lx=3.2, ly=2.0, lz=2.0, zbc=ZBC_NOSLIP, beta=1.3, nu=2e-3,
                                  sgs=SGS_DSM), "duct"),
    ("wm dsm cn-z h_wm", dict(nx=24, ny=16, nz=16, lx=6.4, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL, nu=1e-4, sgs=SGS_DSM,
                              h_wm=0.3, implicit_z=True), "duct"),
    # the smallest duct: four rows and four planes (every row and plane next to a wall)
    ("fewest cells wm dsm", dict(nx=8, ny=4, nz=4, lx=1.0, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL, nu=1e-3, sgs=SGS_DSM),
     "duct"),
    ("fewest cells noslip vd radix3", dict(nx=12, ny=6, nz=4, lx=1.0, ly=2.0, lz=2.0, zbc=ZBC_NOSLIP, nu=1e-2,
                                           sgs=SGS_SMAG_VD, cs=0.12), "duct"),
]


def _compare(solver, case, g, st):
    I, J = slice(1, g.nz + 1), slice(0, g.ny)
    gu, gv, gw, gp = solver.fields()
    errs = dict(u=rel_err(gu, st.u, I), v=rel_err(gv, st.v, I), w=rel_err(gw, st.w, I))
    pm, pr = mean_free(gp, g), mean_free(st.p, g)
    errs["p"] = np.max(np.abs(pm[I, J] - pr[I, J])) / max(np.max(np.abs(pr[I, J])), 1e-300)
    nut = solver.eddy_viscosity()
    errs["nut"] = rel_err(nut, st.nut, I) if np.max(np.abs(st.nut[I])) > 0 else np.max(np.abs(nut[I]))
    if case.sgs == SGS_DSM:
        # x-line coefficients: a ratio of sums of cancelling differences (as in the channel
        # tests); nu_t against the propagated rounding bound, line by line
        ok, ratio, _ = dsm_nut_check(case, g, st, nut)
        errs["nut"] = 0.0 if ok else ratio
        gcs = solver.coefficient()
        errs["cs"] = np.max(np.abs(gcs - st.cs[:, :g.ny])) / max(np.max(st.cs[:, :g.ny]), 1e-300)
    if case.zbc == ZBC_WALLMODEL:
        tz = solver.wall_stress()
        ty = solver.wall_stress_y()
        errs["tau_z"] = max(rel_err(tz[q], st.tau[q], slice(None)) for q in range(4))
        errs["tau_y"] = max(rel_err(ty[q], st.tauy[q], slice(None)) for q in range(4))
    return errs, gv


@pytest.mark.parametrize("name,cfgd,kind", SUBSTEP_CASES, ids=[c[0] for c in SUBSTEP_CASES])
def test_duct_substeps_match_oracle(les, name, cfgd, kind):
    say("duct substep case", name)
    case, g, cfg = make_pair(**DUCT, **dict(cfgd))
    u, v, w = initial_fields(case, g, 5, kind)
    st = S.initial_state(case, g, u, v, w)
    dt = S.time_step(case, g, st, cfl=0.5)
    solver = les.Solver(cfg)
    solver.set_state(u, v, w)
    solver.nut()
    gdt = solver.dt(0.5)
    say(f"  dt {gdt!r} oracle {dt!r}")
    assert abs(gdt - dt) <= 1e-13 * dt
    solver.set_dt(dt)
    errs, _ = _compare(solver, case, g, st)
    say("  start: " + " ".join(f"{a}={b:.2e}" for a, b in errs.items()))
    for a in ("nut", "tau_z", "tau_y"):
        if a in errs:
            assert errs[a] < 1e-12, (a, errs[a])
    if "cs" in errs:
        assert errs["cs"] < 1e-9, errs["cs"]
    ptol = pressure_tolerance(g)
    for s in range(3):
        st = S.substep(case, g, st, s, dt)
        solver.substep(s)
        errs, gv = _compare(solver, case, g, st)
        say(f"  substep {s}: " + " ".join(f"{a}={b:.2e}" for a, b in errs.items()))
        for a, e in errs.items():
            assert e < {"p": ptol, "cs": 1e-9}.get(a, 1e-12), (s, a, e)
        assert np.all(gv[:, g.ny - 1] == 0.0) and np.all(gv[:, g.ny + 1] == 0.0)
    d, status = solver.diag()
    say(f"  max div {d.max_div:.2e} ubulk {d.ubulk!r}")
    assert status == 0 and abs(d.ubulk - 1.0) < 1e-12
    solver.close()


MIXED = [SUBSTEP_CASES[2], SUBSTEP_CASES[3], SUBSTEP_CASES[8]]


@pytest.mark.parametrize("name,cfgd,kind", MIXED, ids=["mixed " + c[0] for c in MIXED])
def test_duct_mixed_precision(les, name, cfgd, kind):
    say("duct mixed case", name)
    case, g, cfg = make_pair(precision=1, **DUCT, **dict(cfgd))
    u, v, w = round32(*initial_fields(case, g, 6, kind))
    st = S.initial_state(case, g, u, v, w)
    dt = S.time_step(case, g, st, cfl=0.5)
    solver = les.Solver(cfg)
    solver.set_state(u, v, w)
    solver.nut()
    solver.set_dt(dt)
    I, J = slice(1, g.nz + 1), slice(0, g.ny)
    for k in range(3):
        st = S.substep(case, g, st, k, dt)
        solver.substep(k)
        gu, gv, gw, gp = solver.fields()
        umax2 = max(np.max(np.abs(st.u[I])), np.max(np.abs(st.v[I])), np.max(np.abs(st.w[I]))) ** 2
        dp = np.max(np.abs(mean_free(gp, g)[I, J] - mean_free(st.p, g)[I, J])) / umax2
        errs = dict(u=rel_err(gu, st.u, I), v=rel_err(gv, st.v, I), w=rel_err(gw, st.w, I), p=dp)
        say(f"  substep {k}: " + " ".join(f"{a}={b:.2e}" for a, b in errs.items()))
        for a, e in errs.items():
            assert e < 1e-5, (k, a, e)
    solver.close()


@pytest.mark.parametrize("zbc,sgs", [(ZBC_NOSLIP, SGS_DSM), (ZBC_WALLMODEL, SGS_SMAG_VD)], ids=["noslip dsm", "wm vd"])
def test_duct_fluid_at_rest_stays_at_rest(les, zbc, sgs):
    """Degenerate case: no flow, no forcing.  Every stress, coefficient and pressure stays
    exactly zero (the wall models' Newton returns u_tau = 0 at U = 0, the dynamic model's
    <M M> = 0 gives c_s = 0)."""
    say("duct at rest", zbc, sgs)
    case, g, cfg = make_pair(nx=16, ny=12, nz=10, lx=3.2, ly=2.0, lz=2.0, zbc=zbc, nu=1e-3, sgs=sgs, ybc=YBC_WALL)
    solver = les.Solver(cfg)
    z = np.zeros((g.nz + 2, g.nys, g.nx))
    solver.set_state(z, z, z)
    solver.nut()
    solver.set_dt(1e-2)
    for k in range(3):
        solver.substep(k)
    for a in solver.fields():
        assert np.all(a == 0.0)
    assert np.all(solver.eddy_viscosity() == 0.0)
    if zbc == ZBC_WALLMODEL:
        assert np.all(solver.wall_stress() == 0.0) and np.all(solver.wall_stress_y() == 0.0)
    if sgs == SGS_DSM:
        assert np.all(solver.coefficient() == 0.0)
    solver.close()
