"""The allocation-free gradient entry point (partials in the library's static device array)
against the workspace entry point: two calls in a row, the second with fewer samples, each
bitwise equal to les_mlp_grad on the same inputs (same kernels, same grid, same summation
order); sizes beyond the array's limit are refused with a message."""
import numpy as np
import pytest

from tests.cases import say

pytestmark = pytest.mark.gpu


def _inputs(torch, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-0.1, 1.1, (n, 7)).astype(np.float32)
    t = (0.02 + 0.01 * np.sin(3 * x[:, 5]) + 0.005 * x[:, 0]).astype(np.float32)
    return torch.as_tensor(x).cuda(), torch.as_tensor(t).cuda()


def _params(torch, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = np.concatenate([rng.uniform(-0.6, 0.6, 448), np.zeros(64), rng.uniform(-0.15, 0.15, 4096),
                        rng.uniform(-0.05, 0.05, 64), rng.uniform(-0.2, 0.2, 64), [0.01]]).astype(np.float32)
    assert p.size == 4737
    return torch.as_tensor(p).cuda()


def test_grad_noalloc_matches_workspace_entry_point():
    import torch
    from paper_2411_09364_amd import les
    assert torch.cuda.is_available()
    stream = torch.cuda.current_stream().cuda_stream
    params = _params(torch, 3)
    for n, seed in ((les.MLP_NOALLOC_MAX_SAMPLES, 21), (9001, 22)):
        say(f"no-alloc gradient: n={n}")
        x, t = _inputs(torch, n, seed)
        ws = torch.empty(les.les_mlp_workspace_bytes(n) // 4, dtype=torch.float32, device="cuda")
        g_ref = torch.empty(4737, dtype=torch.float32, device="cuda")
        l_ref = torch.empty(1, dtype=torch.float32, device="cuda")
        g = torch.full((4737,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        les.les_mlp_grad(stream, params.data_ptr(), x.data_ptr(), t.data_ptr(), n, ws.data_ptr(), g_ref.data_ptr(),
                         l_ref.data_ptr())
        les.les_mlp_grad_noalloc(stream, params.data_ptr(), x.data_ptr(), t.data_ptr(), n, g.data_ptr(),
                                 loss.data_ptr())
        torch.cuda.synchronize()
        a, b = g.cpu().numpy(), g_ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), np.max(np.abs(a - b))
        assert np.array_equal(loss.cpu().numpy().view(np.uint32), l_ref.cpu().numpy().view(np.uint32))
        assert float(np.abs(b).max()) > 0.0


def test_grad_noalloc_rejects_sizes_beyond_the_limit():
    import torch
    from paper_2411_09364_amd import les
    stream = torch.cuda.current_stream().cuda_stream
    params = _params(torch, 4)
    n = les.MLP_NOALLOC_MAX_SAMPLES + 1
    x, t = _inputs(torch, n, 23)
    g = torch.empty(4737, dtype=torch.float32, device="cuda")
    with pytest.raises(les.LesError) as e:
        les.les_mlp_grad_noalloc(stream, params.data_ptr(), x.data_ptr(), t.data_ptr(), n, g.data_ptr(), 0)
    assert "exceeds LES_MLP_NOALLOC_MAX_SAMPLES" in str(e.value)
