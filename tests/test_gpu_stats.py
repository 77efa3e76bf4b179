"""GPU statistics (Secs. 4.2 and 4.3 channel statistics; the square duct of Sec. 4.4 with x-line
sums and the perimeter-mean wall stress) against the oracle.  The device plane sums of
each sample equal the oracle's sums of the same fields read back, and the whole pipeline
(substeps, samples, finalisation) equals the oracle's own run.  Sums of the same terms in
another order differ by rounding of the order eps log2(terms) times the sum of |term|, so
means are compared against the mean |term| of their plane (1e-13; 1e-11 for the separate
runs, whose fields agree to 1e-12), covariances against the mean |products| and the
products of mean |factors|; the batch-means uncertainty within 1e-9 relative."""
import numpy as np
import pytest

from oracle import substep as S, stats as ST
from oracle.case import ZBC_NOSLIP, ZBC_WALLMODEL, ZBC_PERIODIC, SGS_SMAG_VD, SGS_SMAG, SGS_DSM, YBC_WALL
from oracle.substep import State
from tests.cases import make_pair, initial_fields, say, round32

pytestmark = pytest.mark.gpu
TWO_PI = 2 * np.pi
COV = ("uu", "vv", "ww", "uv", "uw", "vw")
MEANS = ("U", "V", "W", "P", "NUT")


@pytest.fixture(scope="module")
def les():
    import torch
    assert torch.cuda.is_available()
    from paper_2411_09364_amd import les as L
    return L


def _gpu_state(solver, case):
    u, v, w, p = solver.fields()
    tau = tuple(solver.wall_stress()) if case.zbc == ZBC_WALLMODEL else None
    tauy = tuple(solver.wall_stress_y()) if case.zbc == ZBC_WALLMODEL and case.ywalls else None
    return State(u, v, w, p, nut=solver.eddy_viscosity(), tau=tau, tauy=tauy)


def _abs_state(st):
    """Absolute values of a state: its plane sums bound the sums of |term| of every quantity
    (|(a + b)/2| <= (|a| + |b|)/2), the scale of the rounding error of a plane sum."""
    return State(np.abs(st.u), np.abs(st.v), np.abs(st.w), np.abs(st.p), nut=np.abs(st.nut), tau=st.tau,
                 tauy=st.tauy)


def _compare(prof, sc, oprof, osc, absprof, tol):
    """Means within tol of the mean |term| (max over planes); covariances within tol of the
    mean |products| and products of mean |factors|; scalars within tol relative (u_b against
    the mean |u|); the batch-means uncertainty (a difference of batch means) within 1e-9."""
    A = {q: np.max(a) for q, a in absprof.items()}
    for q in MEANS:
        e = np.max(np.abs(prof[q] - oprof[q]))
        assert e <= tol * max(A[q], 1e-300), (q, e, A[q])
    pairs = {"uu": ("U", "U"), "vv": ("V", "V"), "ww": ("W", "W"), "uv": ("U", "V"), "uw": ("U", "W"),
             "vw": ("V", "W")}
    for q, (a, b) in pairs.items():
        e = np.max(np.abs(prof[q] - oprof[q]))
        assert e <= tol * (A[q] + A[a] * A[b]), (q, e)
    assert sc["samples"] == osc["samples"]
    assert abs(sc["u_b"] - osc["u_b"]) <= tol * max(abs(osc["u_b"]), A["U"])
    if osc["tau_w"] == 0.0:
        assert sc["tau_w"] == 0.0
        return
    for key in ("tau_w", "u_tau", "c_f"):
        assert abs(sc[key] - osc[key]) <= tol * abs(osc[key]), (key, sc[key], osc[key])
    if np.isnan(osc["c_f_sigma"]):
        assert np.isnan(sc["c_f_sigma"])
    else:
        assert abs(sc["c_f_sigma"] - osc["c_f_sigma"]) <= 1e-9 * max(abs(osc["c_f_sigma"]), 1e-300)


def _abs_profiles(case, g, states):
    acc = ST.Accumulator(g)
    for st in states:
        acc.add(case, g, _abs_state(st))
    N = acc.samples * g.nx * (1 if g.ywalls else g.ny)   # x lines in a duct, planes otherwise
    names = ("U", "V", "W", "P", "NUT", "uu", "vv", "ww", "uv", "uw", "vw")
    return {nm: acc.sums[q] / N for q, nm in enumerate(names)}


CASES = [
    ("noslip vd", dict(nx=48, ny=24, nz=20, lx=TWO_PI, ly=np.pi, lz=2.0, zbc=ZBC_NOSLIP, beta=1.5, nu=1e-3,
                       sgs=SGS_SMAG_VD, cs=0.1, ubulk=1.0), "channel", 0),
    ("wm smag cn-z", dict(nx=32, ny=16, nz=12, lx=TWO_PI, ly=np.pi, lz=2.0, zbc=ZBC_WALLMODEL, beta=1.2,
                          nu=5e-5, sgs=SGS_SMAG, implicit_z=True, ubulk=1.0), "channel", 0),
    ("periodic smag", dict(nx=24, ny=24, nz=24, lx=TWO_PI, ly=TWO_PI, lz=TWO_PI, nu=1e-3, sgs=SGS_SMAG), "iso", 0),
    ("mixed wm dsm", dict(nx=48, ny=24, nz=20, lx=TWO_PI, ly=np.pi, lz=2.0, zbc=ZBC_WALLMODEL, beta=1.5, nu=5e-5,
                          sgs=SGS_DSM, ubulk=1.0), "channel", 1),
    # square duct: x-line sums (cross-section profiles), perimeter-mean wall stress
    ("duct wm dsm", dict(nx=40, ny=20, nz=12, lx=4.0, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL, nu=1e-4, sgs=SGS_DSM,
                         ubulk=1.0, ybc=YBC_WALL, h_wm=0.3), "duct", 0),
    ("duct noslip vd stretched", dict(nx=16, ny=12, nz=10, lx=3.2, ly=2.0, lz=2.0, zbc=ZBC_NOSLIP, beta=1.3,
                                      nu=2e-3, sgs=SGS_SMAG_VD, cs=0.12, ubulk=1.0, ybc=YBC_WALL), "duct", 0),
    ("mixed duct wm vd", dict(nx=40, ny=20, nz=12, lx=4.0, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL, nu=1e-4,
                              sgs=SGS_SMAG_VD, cs=0.1, ubulk=1.0, ybc=YBC_WALL), "duct", 1),
]


@pytest.mark.parametrize("name,cfgd,kind,prec", CASES, ids=[c[0] for c in CASES])
def test_sample_sums_equal_oracle_sums_of_the_same_fields(les, name, cfgd, kind, prec):
    """Per-sample device sums against the oracle's sums of the read-back fields, over six
    substeps, finalised on both sides (nbatch 3)."""
    say("stats case", name)
    case, g, cfg = make_pair(precision=prec, **dict(cfgd))
    u, v, w = initial_fields(case, g, 5, kind)
    if prec:
        u, v, w = round32(u, v, w)
    solver = les.Solver(cfg)
    solver.set_state(u, v, w)
    solver.nut()
    dt = solver.dt(0.5)
    solver.set_dt(dt)
    solver.stats_reset()
    acc = ST.Accumulator(g)
    states = []
    for s in range(6):
        solver.substep(s % 3)
        solver.stats_sample()
        states.append(_gpu_state(solver, case))
        acc.add(case, g, states[-1])
    sc, prof = solver.stats(nbatch=3)
    oprof, osc = ST.finalize(case, g, acc, nb=3)
    say(f"  samples {sc['samples']} u_b {sc['u_b']:.6f} c_f {sc['c_f']:.4e} +- {sc['c_f_sigma']:.2e}")
    _compare(prof, sc, oprof, osc, _abs_profiles(case, g, states), 1e-13)
    solver.close()


def test_pipeline_matches_oracle_run(les):
    """Substeps and samples on both sides from the same initial state (FP64, no-slip
    channel, van Driest model): the GPU statistics equal the oracle's own run."""
    case, g, cfg = make_pair(nx=48, ny=24, nz=20, lx=TWO_PI, ly=np.pi, lz=2.0, zbc=ZBC_NOSLIP, beta=1.5,
                             nu=1e-3, sgs=SGS_SMAG_VD, cs=0.1, ubulk=1.0)
    u, v, w = initial_fields(case, g, 7, "channel")
    st = S.initial_state(case, g, u, v, w)
    dt = S.time_step(case, g, st, cfl=0.5)
    solver = les.Solver(cfg)
    solver.set_state(u, v, w)
    solver.nut()
    solver.set_dt(dt)
    solver.stats_reset()
    acc = ST.Accumulator(g)
    states = []
    for s in range(9):
        st = S.substep(case, g, st, s % 3, dt)
        solver.substep(s % 3)
        if s % 3 == 2:
            acc.add(case, g, st)
            states.append(st)
            solver.stats_sample()
    sc, prof = solver.stats(nbatch=3)
    oprof, osc = ST.finalize(case, g, acc, nb=3)
    # the fields themselves agree to 1e-12 (substep parity), so do the statistics
    _compare(prof, sc, oprof, osc, _abs_profiles(case, g, states), 1e-11)
    # reset clears the sums
    solver.stats_reset()
    sc2, _ = solver.stats()
    assert sc2["samples"] == 0
    solver.close()


def test_full_size_sample(les):
    """One sample of the 256 x 128 x 96 wall-model channel after one graph-replayed step,
    against the oracle's sums of the same fields."""
    case, g, cfg = make_pair(nx=256, ny=128, nz=96, lx=TWO_PI, ly=np.pi, lz=2.0, zbc=ZBC_WALLMODEL, beta=1.5,
                             nu=5e-5, sgs=SGS_DSM, implicit_z=True, ubulk=1.0)
    u, v, w = initial_fields(case, g, 2, "channel")
    solver = les.Solver(cfg)
    solver.set_state(u, v, w)
    solver.nut()
    solver.set_dt(solver.dt(0.5))
    les.les_step(solver.ctx, True)
    solver.stats_reset()
    solver.stats_sample()
    acc = ST.Accumulator(g)
    st = _gpu_state(solver, case)
    acc.add(case, g, st)
    sc, prof = solver.stats(nbatch=8)
    oprof, osc = ST.finalize(case, g, acc, nb=8)
    say(f"  full size: u_b {sc['u_b']:.12f} tau_w {sc['tau_w']:.6e}")
    _compare(prof, sc, oprof, osc, _abs_profiles(case, g, [st]), 1e-13)
    solver.close()
