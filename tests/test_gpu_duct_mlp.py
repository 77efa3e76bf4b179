"""GPU tests of the learned closure in the square duct (walls in y and z, Sec. 4.4) against
the oracle: training pairs (inputs with the four-wall y+ of R40, targets the x-line dynamic
coefficient), the fused inference with its per-x-line fallback, and whole substeps in which
every point falls back, which must then be the dynamic model's substeps.

Tolerances as in the channel tests of the learned closure: float32 roundoff on the inputs
and the network output, single bfloat16 flips at most on a few points; the substeps with
every point falling back take the dynamic-model duct substep tolerances.
"""
import numpy as np
import pytest

from oracle import mlp as OM, sgs as OS, bc as OBC
from oracle import substep as S
from oracle.case import ZBC_NOSLIP, ZBC_WALLMODEL, YBC_WALL, SGS_DSM, SGS_MLP
from tests.cases import make_pair, initial_fields, rel_err, mean_free, say, round32, pressure_tolerance, \
    dsm_nut_check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2411_09364_amd import les
    return les, torch


# ragged tiles in x (40 = 32 + 8) and y (20 rows over tiles of 8)
DUCT = dict(nx=40, ny=20, nz=12, lx=4.0, ly=2.0, lz=2.0, nu=1e-4, ybc=YBC_WALL, ubulk=1.0)


def _duct(sgs, zbc, **kw):
    extra = dict(beta=1.2) if zbc == ZBC_NOSLIP else {}
    return make_pair(**dict(DUCT, sgs=sgs, zbc=zbc, **extra, **kw))


def _utau4(case, g, st):
    """Friction velocities of the four walls (z bottom, z top, y = 0, y = ly), R36."""
    if case.zbc == ZBC_WALLMODEL:
        return OS.duct_friction_velocity(g, st.tau, st.tauy)
    return OS.duct_friction_velocity(g, OBC.noslip_wall_stress(case, g, st.u, st.v),
                                     OBC.noslip_wall_stress_y(case, g, st.u, st.w))


def _splitmix64(z):
    M = (1 << 64) - 1
    z = (z + 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


@pytest.mark.parametrize("zbc", [ZBC_WALLMODEL, ZBC_NOSLIP], ids=["wm", "noslip"])
def test_duct_sample_matches_oracle_features(env, zbc):
    les, torch = env
    case, g, cfg = _duct(SGS_DSM, zbc)
    u, v, w = initial_fields(case, g, 8, "duct")
    st = S.initial_state(case, g, u, v, w)
    solver = les.Solver(cfg)
    solver.set_state(u, v, w)
    solver.nut()
    n, seed = 2000, 4242
    x, y = solver.mlp_sample(seed, n)
    x, y = x.cpu().numpy().astype(np.float64), y.cpu().numpy().astype(np.float64)
    s6 = OS.model_strain(case, g, st.u, st.v, st.w)
    feats = OM.raw_features(case, g, st.u, st.v, st.w, s6, _utau4(case, g, st))
    cs = st.cs[:, :g.ny]
    ncell = g.nz * g.ny * g.nx
    rows = set()
    for s in range(n):
        e = _splitmix64(seed ^ _splitmix64(s)) % ncell
        k, r = divmod(e, g.ny * g.nx)
        j, i = divmod(r, g.nx)
        rows.add(j)
        ref = feats[k, j, i]
        assert np.allclose(x[s], ref, rtol=1e-5, atol=1e-6 * (1 + np.abs(ref).max())), (s, k, j, i, x[s], ref)
        assert abs(y[s] - cs[k, j]) <= 1e-6 * abs(cs[k, j]) + 1e-9 * np.max(cs), (s, k, j, y[s], cs[k, j])
    assert rows == set(range(g.ny))          # the wall rows are drawn, the ghost rows never
    solver.close()


@pytest.mark.parametrize("zbc,narrow,precision", [(ZBC_WALLMODEL, False, 0), (ZBC_WALLMODEL, True, 0),
                                                  (ZBC_NOSLIP, True, 0), (ZBC_WALLMODEL, False, 1)],
                         ids=["wm", "wm-narrow", "noslip-narrow", "wm-mixed"])
def test_duct_fused_inference_matches_oracle(env, zbc, narrow, precision):
    """les_nut with the learned closure against oracle.mlp.mlp_eddy_viscosity; with narrow
    ranges the cells beyond the median y+ fall back to the coefficient of their x line."""
    les, torch = env
    case_d, g, _ = _duct(SGS_DSM, zbc)
    _, _, cfg_m = _duct(SGS_MLP, zbc, precision=precision)
    u, v, w = initial_fields(case_d, g, 9, "duct")
    if precision:
        u, v, w = round32(u, v, w)
    st = S.initial_state(case_d, g, u, v, w)
    ut = _utau4(case_d, g, st)
    s6 = OS.model_strain(case_d, g, st.u, st.v, st.w)
    f = OM.raw_features(case_d, g, st.u, st.v, st.w, s6, ut).reshape(-1, 7)
    lo, hi = f.min(axis=0), f.max(axis=0)
    if narrow:
        hi[5] = np.median(f[:, 5])
    # an input constant over the grid up to rounding (Delta on a uniform grid) gets a unit
    # span: a span of rounding size would turn last-bit differences into O(1) inputs
    hi = np.where(hi - lo > 1e-9 * np.maximum(1.0, np.abs(hi)), hi, lo + 1.0)
    p = OM.init_params(21)
    p["b3"][:] = 0.03
    ref, flags = OM.mlp_eddy_viscosity(case_d, g, st.u, st.v, st.w, p, lo, hi, st.cs, ut, emulate_bf16=True)
    solver = les.Solver(cfg_m)
    solver.set_state(u, v, w)
    mlp = les.Mlp(OM.flatten(p), stream=solver.stream)
    solver.mlp_bind(mlp, lo, hi)
    solver.nut()
    nut = solver.eddy_viscosity()[1:g.nz + 1, :g.ny]
    d, _ = solver.diag()
    scale = np.max(np.abs(ref))
    diff = np.abs(nut - ref)
    say(f"duct fused inference zbc={zbc} narrow={narrow} precision={precision}: flagged {int(flags.sum())} "
        f"(gpu {d.mlp_flagged}), median {np.median(diff) / scale:.2e} max {diff.max() / scale:.2e}")
    if narrow:
        assert 0 < int(flags.sum()) < flags.size
    med, mx = (2e-6, 2e-3) if precision == 0 else (2e-5, 5e-3)
    assert abs(d.mlp_flagged - int(flags.sum())) <= (0 if precision == 0 else flags.size // 1000)
    assert np.median(diff) <= med * scale
    assert diff.max() <= mx * scale
    solver.close()


@pytest.mark.parametrize("zbc", [ZBC_WALLMODEL, ZBC_NOSLIP], ids=["wm", "noslip"])
def test_duct_learned_closure_falling_back_everywhere_is_the_dynamic_model(env, zbc):
    """Ranges that put every input out of range: every point takes the dynamic coefficient of
    its x line, every evaluation re-runs the dynamic model, and three substeps must equal the
    oracle's dynamic-model duct substeps."""
    les, torch = env
    case_d, g, _ = _duct(SGS_DSM, zbc)
    _, _, cfg_m = _duct(SGS_MLP, zbc)
    u, v, w = initial_fields(case_d, g, 5, "duct")
    st = S.initial_state(case_d, g, u, v, w)
    dt = S.time_step(case_d, g, st, cfl=0.5)
    solver = les.Solver(cfg_m)
    solver.set_state(u, v, w)
    mlp = les.Mlp(OM.flatten(OM.init_params(4)), stream=solver.stream)
    solver.mlp_bind(mlp, np.full(7, 1e3), np.full(7, 1e3 + 1.0))
    solver.nut()
    solver.set_dt(dt)
    I, J = slice(1, g.nz + 1), slice(0, g.ny)
    ptol = pressure_tolerance(g)
    for k in range(3):
        st = S.substep(case_d, g, st, k, dt)
        solver.substep(k)
        gu, gv, gw, gp = solver.fields()
        nut = solver.eddy_viscosity()
        ok, ratio, _ = dsm_nut_check(case_d, g, st, nut)
        pm, pr = mean_free(gp, g), mean_free(st.p, g)
        errs = dict(u=rel_err(gu, st.u, I), v=rel_err(gv, st.v, I), w=rel_err(gw, st.w, I),
                    p=np.max(np.abs(pm[I, J] - pr[I, J])) / max(np.max(np.abs(pr[I, J])), 1e-300))
        d, status = solver.diag()
        say(f"  substep {k}: " + " ".join(f"{a}={b:.2e}" for a, b in errs.items()) +
            f" nut ratio {ratio:.2e} flagged {d.mlp_flagged}")
        assert status == 0 and d.mlp_flagged == g.nx * g.ny * g.nz
        assert ok, ratio
        for a, e in errs.items():
            assert e < {"p": ptol}.get(a, 1e-12), (k, a, e)
    solver.close()


def test_duct_learned_closure_gains_over_constant_coefficient(env):
    """Train on x-line dynamic coefficients produced by the GPU solver itself (duct, dynamic
    model + wall model on four walls, four snapshots); on held-out cells of the same
    snapshots the network's error against the dynamic coefficient must be below that of the
    best constant coefficient.  The bar (0.9) is looser than the channel's: a duct target is
    an average over one x line of 64 cells, whose sampling scatter between lines at the same
    wall distance no pointwise input can predict (measured ratio 0.83 here).  The trained
    network then drives five steps of the duct."""
    les, torch = env
    case, g, cfg = make_pair(nx=64, ny=32, nz=32, lx=4.0, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL, nu=5e-5,
                             sgs=SGS_DSM, ybc=YBC_WALL, ubulk=1.0, h_wm=0.1)
    u, v, w = initial_fields(case, g, 2, "duct")
    solver = les.Solver(cfg)
    solver.set_state(u, v, w)
    solver.nut()
    xs, ys, xh, yh = [], [], [], []
    for snap in range(4):
        for _ in range(10):
            solver.dt(0.5)
            solver.step()
        x, y = solver.mlp_sample(100 + snap, 8192)
        xs.append(x)
        ys.append(y)
        x, y = solver.mlp_sample(900 + snap, 2048)
        xh.append(x)
        yh.append(y)
    xr, yr, xhr, yhr = torch.cat(xs), torch.cat(ys), torch.cat(xh), torch.cat(yh)
    torch.cuda.synchronize()
    xn = xr.cpu().numpy().astype(np.float64)
    lo, hi = xn.min(axis=0), xn.max(axis=0)
    # an input constant over the grid up to rounding (Delta on a uniform grid) gets a unit
    # span: a span of rounding size would turn last-bit differences into O(1) inputs
    hi = np.where(hi - lo > 1e-9 * np.maximum(1.0, np.abs(hi)), hi, lo + 1.0)
    x = torch.empty_like(xr)
    xhn = torch.empty_like(xhr)
    les.les_mlp_normalize(solver.stream.cuda_stream, xr.data_ptr(), xr.shape[0], lo, hi, x.data_ptr())
    les.les_mlp_normalize(solver.stream.cuda_stream, xhr.data_ptr(), xhr.shape[0], lo, hi, xhn.data_ptr())
    mlp = les.Mlp(OM.flatten(OM.init_params(3)), stream=solver.stream)
    for it in range(800):
        mlp.train_step(x, yr, 3e-3 if it < 500 else 1e-3)
    pred_d = mlp.forward(xhn)
    solver.synchronize()
    pred = np.maximum(pred_d.cpu().numpy(), 0.0)
    yt = yhr.cpu().numpy()
    c0 = yr.cpu().numpy().mean()
    mse_mlp = np.mean((pred - yt) ** 2)
    mse_const = np.mean((c0 - yt) ** 2)
    say(f"duct targets mean {yt.mean():.3e} std {yt.std():.3e}; held-out MSE learned {mse_mlp:.3e}, "
        f"best constant {mse_const:.3e}, ratio {mse_mlp / mse_const:.3f}")
    assert mse_const > 0.0 and mse_mlp < 0.9 * mse_const
    # the trained network drives the duct: bound to an MLP context on the same state
    cfg_m = make_pair(nx=64, ny=32, nz=32, lx=4.0, ly=2.0, lz=2.0, zbc=ZBC_WALLMODEL, nu=5e-5, sgs=SGS_MLP,
                      ybc=YBC_WALL, ubulk=1.0, h_wm=0.1)[2]
    sm = les.Solver(cfg_m)
    fu, fv, fw, _ = solver.fields()
    sm.set_state(fu, fv, fw)
    sm.mlp_bind(mlp, lo, hi)
    sm.nut()
    for _ in range(5):
        sm.dt(0.5)
        sm.step()
    d, status = sm.diag()
    say(f"  learned duct: 5 steps, max div {d.max_div:.2e}, ubulk {d.ubulk!r}, flagged {d.mlp_flagged}")
    assert status == 0 and abs(d.ubulk - 1.0) < 1e-12 and d.max_div < 1e-10
    assert d.mlp_flagged < 0.1 * g.nx * g.ny * g.nz
    sm.close()
    solver.close()
