"""GPU tests of batched ensembles: per box the batched result equals an unbatched run of
the same box bit for bit (the kernels are the same code and each box's arithmetic does not
depend on the batching), and matches the oracle within the FP64 / mixed tolerances."""
import numpy as np
import pytest

from oracle import substep as S
from oracle.case import SGS_DSM, SGS_SMAG
from tests.cases import make_pair, initial_fields, rel_err, say, round32

pytestmark = pytest.mark.gpu
TWO_PI = 2 * np.pi


@pytest.fixture(scope="module")
def les():
    import torch
    assert torch.cuda.is_available()
    from paper_2411_09364_amd import les as L
    return L


BOXES = [(16, 1e-3, 4.0), (24, 7e-4, 3.0), (32, 1.5e-3, 6.0), (12, 2e-3, 3.0)]


def _cases(precision, sgs):
    out = []
    for n, nu, k0 in BOXES:
        out.append(make_pair(n, n, n, TWO_PI, TWO_PI, TWO_PI, nu=nu, sgs=sgs, cs=0.17, precision=precision) + (k0,))
    return out


@pytest.mark.parametrize("precision,sgs", [(0, SGS_DSM), (1, SGS_DSM), (0, SGS_SMAG)])
def test_batch_matches_unbatched_and_oracle(les, precision, sgs):
    cases = _cases(precision, sgs)
    say("batch", precision, sgs, [c[0].nx for c in cases])
    batch = les.Batch([c[2] for c in cases])
    singles = []
    fields = []
    for b, (case, g, cfg, k0) in enumerate(cases):
        u, v, w = initial_fields(case, g, 10 + b, "iso")
        if precision == 1:
            u, v, w = round32(u, v, w)
        fields.append((u, v, w))
        batch.set_state(b, u, v, w)
        s = les.Solver(cfg)
        s.set_state(u, v, w)
        s.nut()
        singles.append(s)
    batch.nut()
    dts = []
    for b, (case, g, cfg, k0) in enumerate(cases):
        st = S.initial_state(case, g, *fields[b])
        dts.append(S.time_step(case, g, st, cfl=0.5))
    # per-box time step computed on the device, then three substeps
    batch.dt(0.5)
    for b, s in enumerate(singles):
        s.dt(0.5)
    batch.synchronize()
    for b in range(len(cases)):
        d = batch.box_dt(b)
        assert abs(d.dt - dts[b]) <= 1e-6 * dts[b] if precision else abs(d.dt - dts[b]) <= 1e-13 * dts[b]
    for k in range(3):
        batch.substep(k)
        for s in singles:
            s.substep(k)
    tol = 1e-5 if precision else 1e-12
    for b, (case, g, cfg, k0) in enumerate(cases):
        gb = batch.fields(b)
        gs = singles[b].fields()
        for q in range(4):
            assert np.array_equal(gb[q], gs[q]), (b, q)
        assert np.array_equal(batch.eddy_viscosity(b), singles[b].eddy_viscosity())
        st = S.initial_state(case, g, *fields[b])
        dt = batch.box_dt(b).dt
        for k in range(3):
            st = S.substep(case, g, st, k, dt)
        I = slice(1, g.nz + 1)
        errs = [rel_err(gb[0], st.u, I), rel_err(gb[1], st.v, I), rel_err(gb[2], st.w, I)]
        say(f"  box {b} n={g.nx}: {['%.2e' % e for e in errs]}")
        assert max(errs) < tol * 3
    for s in singles:
        s.close()
    batch.close()


def test_batch_graph_replay_equals_eager(les):
    cases = _cases(1, SGS_DSM)
    runs = []
    for use_graph in (False, True):
        batch = les.Batch([c[2] for c in cases])
        for b, (case, g, cfg, k0) in enumerate(cases):
            batch.set_state(b, *round32(*initial_fields(case, g, 20 + b, "iso")))
        batch.nut()
        for it in range(3):
            batch.step(0.5, use_graph)
            batch.synchronize()
        runs.append([batch.fields(b) for b in range(len(cases))])
        batch.close()
    for b in range(len(cases)):
        for q in range(4):
            assert np.array_equal(runs[0][b][q], runs[1][b][q]), (b, q)


def test_autotune_keeps_results_bitwise(les):
    cases = _cases(1, SGS_DSM)
    outs = []
    for tune in (False, True):
        batch = les.Batch([c[2] for c in cases])
        if tune:
            batch.set_dt(1e-3)
            rep = batch.autotune(3)
            say("autotune", rep)
            assert "chosen" in rep
        for b, (case, g, cfg, k0) in enumerate(cases):
            batch.set_state(b, *round32(*initial_fields(case, g, 30 + b, "iso")))
        batch.nut()
        batch.step(0.5, False)
        outs.append([batch.fields(b) for b in range(len(cases))])
        batch.close()
    for b in range(len(cases)):
        for q in range(4):
            assert np.array_equal(outs[0][b][q], outs[1][b][q]), (b, q)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_sampling_matches_single_contexts(les, precision):
    """The ensemble as a training-data generator: box b of a batch draws the same training
    pairs as les_mlp_sample on an unbatched context in the same state with seed + b, bit for
    bit, after les_nut and after a batched step (which equals the unbatched step bit for bit)."""
    cases = _cases(precision, SGS_DSM)
    batch = les.Batch([c[2] for c in cases])
    singles = []
    for b, (case, g, cfg, k0) in enumerate(cases):
        u, v, w = initial_fields(case, g, 20 + b, "iso")
        if precision == 1:
            u, v, w = round32(u, v, w)
        batch.set_state(b, u, v, w)
        s = les.Solver(cfg)
        s.set_state(u, v, w)
        s.nut()
        singles.append(s)
    batch.nut()
    n, seed = 3000, 1234
    for rnd in range(2):
        x, y = batch.mlp_sample(seed, n)
        x, y = x.cpu().numpy(), y.cpu().numpy()
        assert x.shape == (len(cases) * n, 7) and y.shape == (len(cases) * n,)
        for b, s in enumerate(singles):
            xs, ys = s.mlp_sample(seed + b, n)
            assert np.array_equal(x[b * n:(b + 1) * n], xs.cpu().numpy()), (rnd, b)
            assert np.array_equal(y[b * n:(b + 1) * n], ys.cpu().numpy()), (rnd, b)
            assert np.all(np.isfinite(x[b * n:(b + 1) * n])) and np.all(y[b * n:(b + 1) * n] >= 0)
        say(f"  batch sampling round {rnd}: {len(cases)} boxes x {n} pairs, c_s per box",
            [float(y[b * n]) for b in range(len(cases))])
        # one step, batched and unbatched, then sample again
        batch.set_dt(2e-3)
        for s in singles:
            s.set_dt(2e-3)
        for k in range(3):
            batch.substep(k)
            for s in singles:
                s.substep(k)
    x0, _ = batch.mlp_sample(seed, 0)
    assert x0.shape == (0, 7)
    for s in singles:
        s.close()
    batch.close()
