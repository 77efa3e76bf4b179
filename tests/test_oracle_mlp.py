"""Pins of the oracle's learned-closure network: backpropagation against central finite
differences, Adam against its closed form on one step, bf16 rounding on exact cases."""
import numpy as np
import pytest

from oracle import mlp


def _data(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(0, 1, (n, 7))
    t = 0.02 + 0.01 * np.sin(3 * x[:, 5]) + 0.005 * x[:, 0]
    return x, t


def test_parameter_count():
    assert mlp.NPARAM == 7 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4737


def test_backprop_matches_finite_differences():
    p = mlp.init_params(3)
    x, t = _data(40, 1)
    _, g = mlp.loss_and_grad(p, x, t)
    vec = mlp.flatten(p)
    gvec = mlp.flatten(g)
    rng = np.random.Generator(np.random.PCG64(2))
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [mlp.NPARAM - 1, 0, 7 * 64 + 3]])
    for i in idx:
        h = 1e-6 * max(1.0, abs(vec[i]))
        vp, vm = vec.copy(), vec.copy()
        vp[i] += h
        vm[i] -= h
        lp, _ = mlp.loss_and_grad(mlp.unflatten(vp), x, t)
        lm, _ = mlp.loss_and_grad(mlp.unflatten(vm), x, t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gvec[i]) <= 1e-7 * max(abs(fd), 1e-4 * np.abs(gvec).max()), (i, fd, gvec[i])


def test_adam_first_step_is_sign_times_lr():
    """On the first step m_hat = g and v_hat = g^2, so the update is -lr g/(|g| + eps)."""
    p = mlp.init_params(4)
    x, t = _data(16, 2)
    _, g = mlp.loss_and_grad(p, x, t)
    z = np.zeros(mlp.NPARAM)
    p1, m, v = mlp.adam_step(p, g, z, z, 1, lr=1e-3)
    gv = mlp.flatten(g)
    expect = mlp.flatten(p) - 1e-3 * gv / (np.abs(gv) + 1e-8)
    assert np.allclose(mlp.flatten(p1), expect, rtol=1e-14, atol=1e-18)


def test_bf16_rounding_exact_cases():
    one = 1.0
    ulp = 2.0 ** -7                     # bf16 spacing just above 1
    assert mlp.bf16(one) == one
    assert mlp.bf16(one + ulp / 2) == one              # tie to even (1.0 has even mantissa)
    assert mlp.bf16(one + 3 * ulp / 2) == one + 2 * ulp  # tie to even upwards
    assert mlp.bf16(one + 0.51 * ulp) == one + ulp
    assert mlp.bf16(-2.0 - 0.49 * 2 * ulp) == -2.0
    big = mlp.bf16(3.0e38)
    assert abs(big / 3.0e38 - 1.0) <= 2.0 ** -8
    assert (np.float32(big).view(np.uint32) & 0xFFFF) == 0     # low 16 bits cleared


def test_training_reduces_loss():
    p = mlp.init_params(5)
    x, t = _data(256, 3)
    m = v = np.zeros(mlp.NPARAM)
    l0, _ = mlp.loss_and_grad(p, x, t)
    for it in range(1, 101):
        l, g = mlp.loss_and_grad(p, x, t)
        p, m, v = mlp.adam_step(p, g, m, v, it, lr=2e-3)
    l1, _ = mlp.loss_and_grad(p, x, t)
    assert l1 < 0.1 * l0
