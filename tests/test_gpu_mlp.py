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


U32 = 2.0 ** -24   # unit roundoff of float32


def _bf16_margin(v):
    """Distance of each value from the nearest bfloat16 rounding boundary (the midpoint
    between the two bfloat16 values that bracket it): a perturbation smaller than this
    cannot change the value's round-to-nearest bfloat16."""
    a = np.abs(np.asarray(v, dtype=np.float64))
    bits = a.astype(np.float32).view(np.uint32)
    lower = (bits & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
    mid = (((bits & np.uint32(0xFFFF0000)) + np.uint32(0x8000)).view(np.float32)).astype(np.float64)
    upper_mid = 2.0 * lower - mid   # midpoint below the lower bfloat16 value
    return np.minimum(np.abs(a - mid), np.abs(a - upper_mid))


def _d2silu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 - s) * (2.0 + z * (1.0 - 2.0 * s))


def _gradient_error_model(p, x, t, n=None):
    """First-order bounds on the float32 error of every intermediate of the kernels' forward
    and backward pass, from the float64 oracle values with bfloat16 emulation.  The products
    of bfloat16 operands are exact in float32, so a matrix-core accumulation of K products
    plus a bias errs by at most (K + 2) u32 times the sum of the magnitudes; SiLU and its
    derivative take exp2 and rcp of about 1 ulp each (a few u32 relative, plus the argument's
    rounding, |z| u32), and inherit the error of their argument through their derivative.
    Returns the oracle gradient, per-entry error bounds of the accumulated gradient and the
    per-sample mask of samples whose bfloat16 roundings (h1, dz2, dz1) are decided the same
    way on both sides (every rounded value farther from a rounding boundary than twice its
    error bound).  n: the batch size of the mean (default: the number of samples); a power of
    two scales dy exactly, so that a sample's roundings do not depend on which other samples
    share its batch."""
    r = OM.bf16
    n = x.shape[0] if n is None else n
    W1, W2 = r(p["W1"]), r(p["W2"])
    w3, b1, b2, b3 = p["W3"][0], p["b1"], p["b2"], p["b3"][0]
    xb = r(x)
    z1 = xb @ W1.T + b1
    E_z1 = 9 * U32 * (np.abs(xb) @ np.abs(W1).T + np.abs(b1))
    h1 = OM.silu(z1)
    E_h1 = np.abs(OM.dsilu(z1)) * E_z1 + (8 + np.abs(z1)) * U32 * np.abs(h1)
    h1b = r(h1)
    z2 = h1b @ W2.T + b2
    E_z2 = 66 * U32 * (np.abs(h1b) @ np.abs(W2).T + np.abs(b2))
    h2 = OM.silu(z2)
    E_h2 = np.abs(OM.dsilu(z2)) * E_z2 + (8 + np.abs(z2)) * U32 * np.abs(h2)
    y = h2 @ w3 + b3
    E_y = E_h2 @ np.abs(w3) + 70 * U32 * (np.abs(h2) @ np.abs(w3) + abs(b3))
    e = y - t
    E_e = E_y + U32 * (np.abs(y) + np.abs(t))
    dy = 2.0 * e / n
    E_dy = 2.0 * E_e / n + 3 * U32 * np.abs(dy)
    ds2 = OM.dsilu(z2)
    E_ds2 = np.abs(_d2silu(z2)) * E_z2 + (10 + 2 * np.abs(z2)) * U32 * np.abs(ds2) + 4 * U32 * np.abs(z2) * U32
    dz2 = (dy[:, None] * w3[None, :]) * ds2
    E_dz2 = np.abs(w3)[None, :] * (E_dy[:, None] * np.abs(ds2) + np.abs(dy)[:, None] * E_ds2) + 3 * U32 * np.abs(dz2)
    dz2b = r(dz2)
    dh1 = dz2b @ W2
    E_dh1 = 66 * U32 * (np.abs(dz2b) @ np.abs(W2))
    ds1 = OM.dsilu(z1)
    E_ds1 = np.abs(_d2silu(z1)) * E_z1 + (10 + 2 * np.abs(z1)) * U32 * np.abs(ds1)
    dz1 = dh1 * ds1
    E_dz1 = E_dh1 * np.abs(ds1) + np.abs(dh1) * E_ds1 + 2 * U32 * np.abs(dz1)
    dz1b = r(dz1)
    ok = np.ones(x.shape[0], dtype=bool)
    for v, E in ((h1, E_h1), (dz2, E_dz2), (dz1, E_dz1)):
        ok &= np.all(_bf16_margin(v) > 2.0 * E, axis=1)
    g = {"W1": dz1b.T @ xb, "b1": dz1.sum(0), "W2": dz2b.T @ h1b, "b2": dz2.sum(0),
         "W3": (dy @ h2)[None, :], "b3": np.array([dy.sum()])}
    # accumulated sums: depth d of the kernel's summation tree (16-sample matrix-core steps over
    # 4 sample blocks and the block's chunks, 4 waves, the blocks in order) bounds their
    # rounding by d u32 times the sum of the magnitudes of the terms
    nblk = min(max((n + 255) // 256, 1), 1024)
    d = 64 + (n + 256 * nblk - 1) // (256 * nblk) + 4 + nblk + 4
    bound = {
        "W1": d * U32 * (np.abs(dz1b).T @ np.abs(xb)),
        "W2": d * U32 * (np.abs(dz2b).T @ np.abs(h1b)),
        "b1": E_dz1.sum(0) + d * U32 * np.abs(dz1).sum(0),
        "b2": E_dz2.sum(0) + d * U32 * np.abs(dz2).sum(0),
        "W3": ((E_dy @ np.abs(h2)) + (np.abs(dy) @ E_h2) + (d + 1) * U32 * (np.abs(dy) @ np.abs(h2)))[None, :],
        "b3": np.array([E_dy.sum() + d * U32 * np.abs(dy).sum()]),
    }
    loss = np.mean(e * e)
    loss_bound = (2.0 * np.abs(e) @ E_e + d * U32 * np.sum(e * e)) / n + U32 * loss
    return g, bound, ok, loss, loss_bound


def _grad_case(kind):
    """Parameters, inputs and targets of the element-wise gradient test.  "positive": weights,
    biases and inputs of one sign, so that no accumulation cancels and the error bounds are
    those of the roundings themselves (about 1e-5 of each entry); targets t = y (1 - xi), xi in
    [0.5, 1.5], so that every error y - t is positive and the sums over samples do not cancel
    either.  "general": the usual signed initialisation and inputs, targets on both sides of
    the output; cancellation makes the bounds looser and leaves fewer samples unambiguous."""
    rng = np.random.Generator(np.random.PCG64(41))
    p = OM.init_params(12)
    if kind == "positive":
        for k in ("W1", "W2", "W3"):
            p[k] = np.abs(p[k])
        p["b1"][:] = 0.1
        p["b2"][:] = 0.1
        x = rng.uniform(0.0, 1.0, (8000, 7))
    else:
        x = rng.uniform(-0.1, 1.1, (300000, 7))
    x = x.astype(np.float32).astype(np.float64)
    y0, _ = OM.forward(p, x, emulate_bf16=True)
    if kind == "positive":
        t = y0 * (1.0 - rng.uniform(0.5, 1.5, size=y0.shape))
    else:
        t = y0 + 20.0 * np.max(np.abs(y0)) * rng.choice([-1.0, 1.0], size=y0.shape) * rng.uniform(0.5, 1.5, size=y0.shape)
    return p, x, t.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("kind", ["positive", "general"])
def test_gradient_matches_oracle_elementwise(env, kind):
    """Every gradient entry and the loss within twice their propagated float32 error bounds of
    the oracle (bfloat16 emulation; both sides err by at most the bound), on the samples whose
    bfloat16 roundings are unambiguous."""
    les, torch = env
    p, x, t = _grad_case(kind)
    n = 2048   # a power of two: dy = 2 (y - t) / n scales every sample's values exactly
    _, _, ok, _, _ = _gradient_error_model(p, x, t, n)
    sel = np.flatnonzero(ok)
    say(f"elementwise gradient ({kind}): {sel.size} of {x.shape[0]} samples with unambiguous bf16 roundings")
    assert sel.size >= n
    xs, ts = x[sel[:n]], t[sel[:n]]
    g_ref, bound, ok2, loss_ref, loss_bound = _gradient_error_model(p, xs, ts)
    assert np.all(ok2)
    mlp = les.Mlp(OM.flatten(p))
    g, loss = mlp.gradient(torch.as_tensor(xs.astype(np.float32)).cuda(), torch.as_tensor(ts.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    g = OM.unflatten(g.cpu().numpy().astype(np.float64))
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        diff = np.abs(g[k] - g_ref[k])
        mag = np.maximum(np.abs(g_ref[k]), 1e-300)
        say(f"grad {k}: worst diff/bound {np.max(diff / (2.0 * bound[k] + 1e-300)):.3f}, rel diff median "
            f"{np.median(diff / mag):.2e} max {np.max(diff / mag):.2e}, bound/|g| median {np.median(bound[k] / mag):.2e}")
        assert np.all(diff <= 2.0 * bound[k]), k
    assert abs(loss.item() - loss_ref) <= 2.0 * loss_bound
    # the float64 oracle gradient without bf16 emulation is pinned by finite differences;
    # the kernels' gradient points the same way (cosine similarity)
    _, g64 = OM.loss_and_grad(p, xs, ts, emulate_bf16=False)
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
    from tests.dsm_bound import nut_difference_bound
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
            bound, _, _ = nut_difference_bound(case_d, g, gu, gv, gw)
            allow = 1e-12 * scale + bound
            assert np.all(diff[flags] <= allow[flags]), float(np.max(diff[flags] / allow[flags]))
        if sub > 0 and counts[-1] and counts[-2] == 0:
            break
    assert counts[0] == 0
    assert any(c > 0 for c in counts[1:]), counts
    solver.close()


def test_learned_closure_gains_over_constant_coefficient(env):
    """Train on dynamic-model coefficients produced by the GPU solver itself (channel, dynamic
    Smagorinsky + wall model + CN-z, six snapshots 10 steps apart) and test on two later
    snapshots (30 and 40 steps after the last training one): the network's error against the
    dynamic coefficient there must be well below that of the best constant coefficient (the
    static model without the dynamic procedure, c = mean training target).  Then a posteriori:
    from the last state, the learned closure and the dynamic model advance 40 steps with the
    same time step; the learned run stays finite and divergence-free and its plane-mean u
    profile stays within 1 % (the Eq. error measure of Sec. 4.3, over 0.1 h to h) of the
    dynamic model's.  (The bench's default line compares the closures, and static
    Smagorinsky + van Driest, over one flow-through of a developed channel.)"""
    les, torch = env
    common = dict(nx=64, ny=32, nz=48, lx=TWO_PI, ly=np.pi, lz=2.0, zbc=ZBC_WALLMODEL, beta=1.5, nu=5e-5,
                  implicit_z=True, ubulk=1.0)
    case, g, cfg = make_pair(sgs=SGS_DSM, **common)
    u, v, w = initial_fields(case, g, 2, "channel")
    solver = les.Solver(cfg)
    solver.set_state(u, v, w)
    solver.nut()

    def advance(n):
        for _ in range(n):
            solver.dt(0.5)
            solver.step()

    xs, ys, xh, yh = [], [], [], []
    for snap in range(6):
        advance(10)
        x, y = solver.mlp_sample(1000 + snap, 8192)
        xs.append(x)
        ys.append(y)
    for snap, gap in enumerate((30, 10)):                # held-out snapshots, later in time
        advance(gap)
        x, y = solver.mlp_sample(5000 + snap, 4096)
        xh.append(x)
        yh.append(y)
    xr, yr, xhr, yhr = torch.cat(xs), torch.cat(ys), torch.cat(xh), torch.cat(yh)
    torch.cuda.synchronize()
    xn = xr.cpu().numpy().astype(np.float64)
    lo, hi = xn.min(axis=0), xn.max(axis=0)
    span = np.where(hi > lo, hi - lo, 1.0)
    lo, hi = lo - 0.25 * span, hi + 0.25 * span          # later states may leave the sampled range
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
    say(f"held-out (later) targets mean {yt.mean():.3e} std {yt.std():.3e}; MSE learned {mse_mlp:.3e}, "
        f"best constant {mse_const:.3e}, ratio {mse_mlp / mse_const:.3f}")
    assert mse_mlp < 0.8 * mse_const

    # a posteriori, from the same state with the same time step
    _, _, cfg_l = make_pair(sgs=SGS_MLP, **common)
    learned = les.Solver(cfg_l)
    fu, fv, fw, fp = solver.fields()
    learned.set_state(fu, fv, fw, fp)
    learned.mlp_bind(mlp, lo, hi)
    learned.nut()
    dt0 = solver.dt(0.5)
    for s in (solver, learned):
        s.set_dt(dt0)
        for _ in range(40):
            s.step()
    # plane-mean u, the two halves averaged, from the wall to the centre (h = lz / 2 = 1)
    zf, zc = solver.zgrid()
    half = g.nz // 2
    zl = np.append(zc[1:half + 1], 1.0)

    def sym(p):
        return np.append(0.5 * (p[:half] + p[::-1][:half]), 0.5 * (p[half - 1] + p[half]))

    prof = [sym(s.fields()[0][1:g.nz + 1].mean(axis=(1, 2))) for s in (solver, learned)]
    err = les.les_profile_error(zl, prof[1], prof[0], 0.1, 1.0)
    d, status = learned.diag()
    say(f"a posteriori, 40 steps: Eq. error of the learned closure's mean u against the dynamic model "
        f"{err:.3e}; learned max|div| {d.max_div:.2e}, fallback points {d.mlp_flagged}")
    assert status == 0 and d.nonfinite == 0 and d.max_div < 1e-10
    assert err < 1e-2
    learned.close()
    solver.close()
