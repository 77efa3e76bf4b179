"""GPU tests of the learned closure (network kernels on the matrix cores) against the oracle.

Tolerances.  The oracle emulates the kernels' bfloat16 rounding points (weights and the
inputs of the two 64-wide products, and dz2/dz1 in the backward pass) in float64; the
kernels accumulate in float32 in an unspecified order and use float32 exp.  Differences are
therefore float32 roundoff (~1e-6 of the output scale) except where a value lies within
float32 roundoff of a bfloat16 rounding boundary: then the two sides round it to adjacent
bfloat16 values (relative step 2^-8) and that sample's output moves by up to ~1e-3 of the
scale.  The tests bound the median difference at float32 level and the maximum at the
single-flip level.
"""
import numpy as np
import pytest

from oracle import mlp as OM, sgs as OS, bc as OBC
from oracle import substep as S
from oracle.case import ZBC_WALLMODEL, SGS_DSM, SGS_MLP
from tests.cases import make_pair, initial_fields, say

pytestmark = pytest.mark.gpu
TWO_PI = 2 * np.pi


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2411_09364_amd import les
    return les, torch


def _data(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-0.1, 1.1, (n, 7))
    t = 0.02 + 0.01 * np.sin(3 * x[:, 5]) + 0.005 * x[:, 0] - 0.003 * x[:, 2] * x[:, 6]
    return x, t


@pytest.mark.parametrize("n", [64, 1000, 4133])
def test_forward_matches_oracle(env, n):
    les, torch = env
    p = OM.init_params(11)
    x, _ = _data(n, 3)
    x32 = x.astype(np.float32)
    ref, _ = OM.forward(p, x32.astype(np.float64), emulate_bf16=True)
    mlp = les.Mlp(OM.flatten(p))
    xd = torch.as_tensor(x32).cuda()
    yd = mlp.forward(xd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy().astype(np.float64)
    d = np.abs(y - ref)
    scale = np.max(np.abs(ref))
    say(f"forward n={n}: median {np.median(d) / scale:.2e} max {d.max() / scale:.2e}")
    assert np.median(d) <= 2e-6 * scale
    assert d.max() <= 2e-3 * scale


def test_gradient_matches_oracle(env):
    les, torch = env
    n = 3000
    p = OM.init_params(12)
    x, t = _data(n, 4)
    x32, t32 = x.astype(np.float32), t.astype(np.float32)
    loss_ref, g_ref = OM.loss_and_grad(p, x32.astype(np.float64), t32.astype(np.float64), emulate_bf16=True)
    mlp = les.Mlp(OM.flatten(p))
    g, loss = mlp.gradient(torch.as_tensor(x32).cuda(), torch.as_tensor(t32).cuda())
    torch.cuda.synchronize()
    g = OM.unflatten(g.cpu().numpy().astype(np.float64))
    assert abs(loss.item() - loss_ref) <= 1e-5 * loss_ref
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        err = np.linalg.norm(g[k] - g_ref[k]) / np.linalg.norm(g_ref[k])
        say(f"grad {k}: rel norm err {err:.2e}")
        assert err < 2e-3, (k, err)
    # the float64 oracle gradient without bf16 emulation is pinned by finite differences;
    # the kernels' gradient points the same way (cosine similarity)
    _, g64 = OM.loss_and_grad(p, x32.astype(np.float64), t32.astype(np.float64), emulate_bf16=False)
    a, b = OM.flatten(g), OM.flatten(g64)
    assert a @ b / (np.linalg.norm(a) * np.linalg.norm(b)) > 0.999


def test_gradient_is_deterministic(env):
    les, torch = env
    p = OM.init_params(13)
    x, t = _data(5000, 5)
    mlp = les.Mlp(OM.flatten(p))
    xd, td = torch.as_tensor(x.astype(np.float32)).cuda(), torch.as_tensor(t.astype(np.float32)).cuda()
    g1 = mlp.gradient(xd, td)[0].clone()
    g2 = mlp.gradient(xd, td)[0].clone()
    torch.cuda.synchronize()
    assert torch.equal(g1, g2)


def test_adam_matches_oracle(env):
    les, torch = env
    rng = np.random.Generator(np.random.PCG64(9))
    p = OM.init_params(14)
    g = OM.unflatten(rng.standard_normal(OM.NPARAM) * 1e-2)
    m = rng.standard_normal(OM.NPARAM) * 1e-3
    v = np.abs(rng.standard_normal(OM.NPARAM)) * 1e-5
    p1, m1, v1 = OM.adam_step(p, g, m, v, 3, lr=1e-3)
    mlp = les.Mlp(OM.flatten(p))
    mlp.m.copy_(torch.as_tensor(m.astype(np.float32)))
    mlp.v.copy_(torch.as_tensor(v.astype(np.float32)))
    gd = torch.as_tensor(OM.flatten(g).astype(np.float32)).cuda()
    torch.cuda.synchronize()
    les.les_mlp_adam(mlp.stream.cuda_stream, mlp.params.data_ptr(), gd.data_ptr(), mlp.m.data_ptr(),
                     mlp.v.data_ptr(), 3, 1e-3)
    torch.cuda.synchronize()
    assert np.allclose(mlp.params.cpu().numpy(), OM.flatten(p1), rtol=2e-6, atol=2e-7)
    assert np.allclose(mlp.m.cpu().numpy(), m1, rtol=1e-5, atol=1e-9)


def test_training_on_gpu_reduces_loss(env):
    les, torch = env
    x, t = _data(8192, 6)
    mlp = les.Mlp(OM.flatten(OM.init_params(15)))
    xd, td = torch.as_tensor(x.astype(np.float32)).cuda(), torch.as_tensor(t.astype(np.float32)).cuda()
    l0 = None
    for it in range(300):
        loss = mlp.train_step(xd, td, 2e-3)
        if it == 0:
            torch.cuda.synchronize()
            l0 = loss.item()
    torch.cuda.synchronize()
    say(f"training loss {l0:.3e} -> {loss.item():.3e}")
    assert loss.item() < 0.05 * l0


def _channel(env, sgs):
    les, torch = env
    case, g, cfg = make_pair(nx=48, ny=24, nz=16, lx=TWO_PI, ly=np.pi, lz=2.0, zbc=ZBC_WALLMODEL, beta=1.5,
                             nu=5e-5, sgs=sgs, ubulk=1.0)
    return case, g, cfg


def _splitmix64(z):
    M = (1 << 64) - 1
    z = (z + 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def test_sample_matches_oracle_features(env):
    les, torch = env
    case, g, cfg = _channel(env, SGS_DSM)
    u, v, w = initial_fields(case, g, 8, "channel")
    st = S.initial_state(case, g, u, v, w)
    solver = les.Solver(cfg)
    solver.set_state(u, v, w)
    solver.nut()
    n, seed = 500, 12345
    x, y = solver.mlp_sample(seed, n)
    x, y = x.cpu().numpy().astype(np.float64), y.cpu().numpy().astype(np.float64)
    s6 = OS.model_strain(case, g, st.u, st.v, st.w)
    feats = OM.raw_features(case, g, st.u, st.v, st.w, s6, OS.friction_velocity(st.tau))
    ncell = g.nz * g.ny * g.nx
    for s in range(n):
        e = _splitmix64(seed ^ _splitmix64(s)) % ncell
        k, r = divmod(e, g.ny * g.nx)
        j, i = divmod(r, g.nx)
        ref = feats[k, j, i]
        assert np.allclose(x[s], ref, rtol=1e-5, atol=1e-6 * (1 + np.abs(ref).max())), (s, x[s], ref)
        assert abs(y[s] - st.cs[k]) <= 1e-6 * max(abs(st.cs[k]), 1e-12)
    solver.close()


@pytest.mark.parametrize("narrow", [False, True])
def test_fused_inference_matches_oracle(env, narrow):
    """les_nut with the learned closure against oracle.mlp.mlp_eddy_viscosity; with narrow
    ranges many points fall back to the dynamic coefficient of their plane."""
    les, torch = env
    case_d, g, _ = _channel(env, SGS_DSM)
    _, _, cfg_m = _channel(env, SGS_MLP)
    u, v, w = initial_fields(case_d, g, 9, "channel")
    st = S.initial_state(case_d, g, u, v, w)
    ut = OS.friction_velocity(st.tau)
    s6 = OS.model_strain(case_d, g, st.u, st.v, st.w)
    f = OM.raw_features(case_d, g, st.u, st.v, st.w, s6, ut).reshape(-1, 7)
    lo, hi = f.min(axis=0), f.max(axis=0)
    if narrow:
        hi[5] = np.median(f[:, 5])       # the upper half of y+ falls back
    hi = np.where(hi > lo, hi, lo + 1.0)
    p = OM.init_params(21)
    p["b3"][:] = 0.03                    # mostly positive output
    ref, flags = OM.mlp_eddy_viscosity(case_d, g, st.u, st.v, st.w, p, lo, hi, st.cs, ut, emulate_bf16=True)
    solver = les.Solver(cfg_m)
    solver.set_state(u, v, w)
    mlp = les.Mlp(OM.flatten(p), stream=solver.stream)
    solver.mlp_bind(mlp, lo, hi)
    solver.nut()
    nut = solver.eddy_viscosity()[1:g.nz + 1]
    d, stat = solver.diag()
    scale = np.max(np.abs(ref))
    diff = np.abs(nut - ref)
    say(f"fused inference narrow={narrow}: flagged {int(flags.sum())} (gpu {d.mlp_flagged}), "
        f"median {np.median(diff) / scale:.2e} max {diff.max() / scale:.2e}")
    assert d.mlp_flagged == int(flags.sum())
    assert np.median(diff) <= 2e-6 * scale
    assert diff.max() <= 2e-3 * scale
    if narrow:
        assert np.array_equal(nut[flags] == ref[flags], np.ones(int(flags.sum()), bool)) or \
            np.max(np.abs(nut[flags] - ref[flags])) <= 1e-12 * scale
    solver.close()


def test_fallback_takes_the_current_coefficients(env):
    """The fallback of a flagged cell is the dynamic coefficient of the state being evaluated
    (R27), also in the first evaluation that flags anything after evaluations that flagged
    nothing.  The y+ range is set so that its extreme values of the initial state sit just
    inside the 5 % margin: the first evaluation flags no cell, and as the friction velocities
    change over the substeps cells at one end leave the range.  After every substep the
    library's eddy viscosity is compared with the oracle's learned closure evaluated on the
    library's own state, whose fallback is the oracle's dynamic coefficient of that state."""
    from tests.cases import CS_ROUNDING_K, UNIT_ROUNDOFF
    from oracle.ops import strain_magnitude
    les, torch = env
    case_d, g, _ = _channel(env, SGS_DSM)
    _, _, cfg_m = _channel(env, SGS_MLP)
    u, v, w = initial_fields(case_d, g, 9, "channel")
    st = S.initial_state(case_d, g, u, v, w)
    ut0 = OS.friction_velocity(st.tau)
    f = OM.raw_features(case_d, g, st.u, st.v, st.w, OS.model_strain(case_d, g, st.u, st.v, st.w), ut0)
    f = f.reshape(-1, 7)
    lo, hi = f.min(axis=0), f.max(axis=0)
    hi = np.where(hi > lo, hi, lo + 1.0)
    a, b, e = lo[5], hi[5], 1e-9
    span = (b - a) / (1.1 - 2 * e)
    lo[5] = a + span * (0.05 - e)
    hi[5] = lo[5] + span
    p = OM.init_params(21)
    p["b3"][:] = 0.03
    solver = les.Solver(cfg_m)
    solver.set_state(u, v, w)
    mlp = les.Mlp(OM.flatten(p), stream=solver.stream)
    solver.mlp_bind(mlp, lo, hi)
    solver.nut()
    n = g.nz
    I = slice(1, n + 1)
    counts = []
    for sub in range(7):
        if sub > 0:
            if (sub - 1) % 3 == 0:
                solver.dt(0.5)
            solver.substep((sub - 1) % 3)
        gu, gv, gw, _ = solver.fields()
        tau = solver.wall_stress()
        ut = OS.friction_velocity(tuple(tau[q] for q in range(4)))
        cs, _, _, _ = OS.dynamic_coefficient(case_d, g, gu, gv, gw)
        ref, flags = OM.mlp_eddy_viscosity(case_d, g, gu, gv, gw, p, lo, hi, cs, ut, emulate_bf16=True)
        nut = solver.eddy_viscosity()[I]
        d, _ = solver.diag()
        scale = np.max(np.abs(ref))
        diff = np.abs(nut - ref)
        counts.append(int(flags.sum()))
        say(f"substep {sub}: flagged {counts[-1]} (gpu {d.mlp_flagged}), median {np.median(diff) / scale:.2e} "
            f"max {diff.max() / scale:.2e}")
        assert d.mlp_flagged == counts[-1]
        assert np.median(diff) <= 2e-6 * scale
        assert diff.max() <= 2e-3 * scale
        if counts[-1]:
            # flagged cells: the dynamic coefficient of this state, within its rounding bound
            rs = OS.coefficient_rounding_scale(case_d, g, gu, gv, gw)
            smag = strain_magnitude(OS.model_strain(case_d, g, gu, gv, gw))
            allow = 1e-12 * scale + CS_ROUNDING_K * UNIT_ROUNDOFF * (rs * g.delta() ** 2)[:, None, None] * smag
            assert np.all(diff[flags] <= allow[flags]), float(np.max(diff[flags] / allow[flags]))
        if sub > 0 and counts[-1] and counts[-2] == 0:
            break
    assert counts[0] == 0
    assert any(c > 0 for c in counts[1:]), counts
    solver.close()


def test_learned_closure_gains_over_constant_coefficient(env):
    """Train on dynamic-model coefficients produced by the GPU solver itself (channel, dynamic
    Smagorinsky + wall model + CN-z, six snapshots); on held-out cells of the same snapshots
    the network's error against the dynamic coefficient must be well below that of the best
    constant coefficient (the static model without the dynamic procedure, c = mean target)."""
    les, torch = env
    case, g, cfg = make_pair(nx=64, ny=32, nz=48, lx=TWO_PI, ly=np.pi, lz=2.0, zbc=ZBC_WALLMODEL, beta=1.5,
                             nu=5e-5, sgs=SGS_DSM, implicit_z=True, ubulk=1.0)
    u, v, w = initial_fields(case, g, 2, "channel")
    solver = les.Solver(cfg)
    solver.set_state(u, v, w)
    solver.nut()
    xs, ys, xh, yh = [], [], [], []
    for snap in range(6):
        for _ in range(10):
            solver.dt(0.5)
            solver.step()
        x, y = solver.mlp_sample(1000 + snap, 8192)
        xs.append(x)
        ys.append(y)
        x, y = solver.mlp_sample(5000 + snap, 2048)      # held-out cells, same state
        xh.append(x)
        yh.append(y)
    xr, yr, xhr, yhr = torch.cat(xs), torch.cat(ys), torch.cat(xh), torch.cat(yh)
    torch.cuda.synchronize()
    xn = xr.cpu().numpy().astype(np.float64)
    lo, hi = xn.min(axis=0), xn.max(axis=0)
    hi = np.where(hi > lo, hi, lo + 1.0)
    x = torch.empty_like(xr)
    xhn = torch.empty_like(xhr)
    les.les_mlp_normalize(solver.stream.cuda_stream, xr.data_ptr(), xr.shape[0], lo, hi, x.data_ptr())
    les.les_mlp_normalize(solver.stream.cuda_stream, xhr.data_ptr(), xhr.shape[0], lo, hi, xhn.data_ptr())
    mlp = les.Mlp(OM.flatten(OM.init_params(3)), stream=solver.stream)
    for it in range(800):
        mlp.train_step(x, yr, 3e-3 if it < 500 else 1e-3)
    pred_d = mlp.forward(xhn)
    solver.synchronize()                                  # forward ran on the library stream
    pred = np.maximum(pred_d.cpu().numpy(), 0.0)
    yt = yhr.cpu().numpy()
    c0 = yr.cpu().numpy().mean()
    mse_mlp = np.mean((pred - yt) ** 2)
    mse_const = np.mean((c0 - yt) ** 2)
    say(f"targets mean {yt.mean():.3e} std {yt.std():.3e}; held-out MSE learned {mse_mlp:.3e}, "
        f"best constant {mse_const:.3e}, ratio {mse_mlp / mse_const:.3f}")
    assert mse_mlp < 0.8 * mse_const
    solver.close()
