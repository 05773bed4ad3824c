"""GPU: the indicator gradient entry point that allocates nothing (lxw_indicator_grad_noalloc, for
callers that cannot allocate device memory) against lxw_indicator_grad, whose kernels it shares:
two calls in a row, the second with fewer samples (the fixed workspace keeps the first call's
partials), both bit for bit equal to the allocating entry point, plus the size limit."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    from paper_1601_08145_amd import lxw
    return lxw


def _data(n, seed):
    g = np.random.default_rng(seed)
    X = g.uniform(-1, 1, (n, 48)).astype(np.float32)
    y = (g.uniform(0, 1, n) < 0.3).astype(np.float32)
    return X, y


def test_grad_noalloc_equals_grad(L):
    from paper_1601_08145_amd import inputs as I
    ind = L.Indicator(I.mlp_init(3))
    for n, seed in [(5000, 1), (300, 2), (L.IND_NOALLOC_MAX, 3), (1, 4)]:
        print(f"[gpu] grad_noalloc n={n}", flush=True)
        X, y = _data(n, seed)
        ref, ref_loss = ind.grad(X, y, 1.5, 0.7)
        Xd = torch.from_numpy(X).cuda()
        yd = torch.from_numpy(y).cuda()
        g = torch.full((L.NPARAM,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        ind.grad_noalloc(Xd, yd, g, loss, 1.5, 0.7)
        ind.stream.synchronize()
        gh = g.cpu().numpy()
        assert np.array_equal(gh, ref), (n, np.max(np.abs(gh - ref)))
        assert float(loss.cpu()[0]) == np.float32(ref_loss)
    # without a loss output
    X, y = _data(200, 5)
    ref, _ = ind.grad(X, y)
    g = torch.zeros(L.NPARAM, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    ind.grad_noalloc(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), g)
    ind.stream.synchronize()
    assert np.array_equal(g.cpu().numpy(), ref)


def test_grad_noalloc_rejects_sizes_beyond_its_workspace(L):
    from paper_1601_08145_amd import inputs as I
    ind = L.Indicator(I.mlp_init(0))
    n = L.IND_NOALLOC_MAX + 1
    Xd = torch.zeros((n, 48), dtype=torch.float32, device="cuda")
    yd = torch.zeros(n, dtype=torch.float32, device="cuda")
    g = torch.zeros(L.NPARAM, dtype=torch.float32, device="cuda")
    with pytest.raises(L.LxwError) as ei:
        ind.grad_noalloc(Xd, yd, g)
    assert ei.value.code == -1 and "8192" in ei.value.msg
