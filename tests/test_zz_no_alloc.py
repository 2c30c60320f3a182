"""lst_mlp_backward_noalloc (the backward pass with the library's fixed
workspace, for callers that cannot allocate) against lst_mlp_backward with a
caller workspace: the same kernels on the same inputs, so gradients and loss
must be equal bit for bit.  Two calls in a row, the second with fewer rows,
so that words left in the fixed array by the first call cannot leak into the
second; then the row limit is refused before anything is launched."""
import numpy as np
import pytest
import torch

from oracle import mlp as M
from synth import weights as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _inputs(ctx, rng, n):
    F = (rng.normal(0, 1, (n, 40)) * 10.0 ** rng.integers(-2, 2, 40)).astype(np.float32)
    mean = F.mean(axis=0).astype(np.float32)
    istd = (1.0 / np.maximum(F.std(axis=0), 1e-6)).astype(np.float32)
    x = torch.empty((n, 64), dtype=torch.int16, device=DEV)
    ctx.mlp_prepare(torch.from_numpy(F).to(DEV), torch.from_numpy(mean).to(DEV),
                    torch.from_numpy(istd).to(DEV), x)
    P = torch.from_numpy(W.random_params(rng, bias=0.2)).to(DEV)
    y = torch.from_numpy(rng.integers(0, 2, n).astype(np.uint8)).to(DEV)
    lg = torch.empty(n, dtype=torch.float32, device=DEV)
    h1 = torch.empty((n, 64), dtype=torch.int16, device=DEV)
    h2 = torch.empty((n, 64), dtype=torch.float32, device=DEV)
    ctx.mlp_forward(P, x, lg, h1, h2)
    return P, x, y, lg, h1, h2


def test_backward_without_allocation_equals_workspace_call():
    import paper_2209_13711_amd as lst
    from synth import geometry as G
    from synth import params as PR
    geo = G.get("barrel_toy")
    ctx = lst.Context(PR.make(), geo.f32, geo.i32, device=0)
    rng = np.random.default_rng(42)
    for n in (8192, 1237):
        print(f"case noalloc backward n={n}", flush=True)
        P, x, y, lg, h1, h2 = _inputs(ctx, rng, n)
        work = torch.empty(ctx.mlp_workspace_bytes(n), dtype=torch.uint8, device=DEV)
        g_ref = torch.full((M.N_PARAM,), float("nan"), dtype=torch.float32, device=DEV)
        l_ref = torch.full((1,), float("nan"), dtype=torch.float32, device=DEV)
        ctx.mlp_backward(P, x, y, lg, h1, h2, work, g_ref, l_ref)
        g = torch.full_like(g_ref, float("nan"))
        l = torch.full_like(l_ref, float("nan"))
        ctx.mlp_backward_noalloc(P, x, y, lg, h1, h2, g, l)
        torch.cuda.synchronize()
        a, b = g.cpu().numpy(), g_ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), n
        assert l.item() == l_ref.item() and np.isfinite(l.item())
    # more rows than the fixed workspace holds: refused, outputs untouched
    n = 8193
    P, x, y, lg, h1, h2 = _inputs(ctx, rng, n)
    g = torch.full((M.N_PARAM,), 7.0, dtype=torch.float32, device=DEV)
    l = torch.full((1,), 7.0, dtype=torch.float32, device=DEV)
    with pytest.raises(lst.LSTError) as ei:
        ctx.mlp_backward_noalloc(P, x, y, lg, h1, h2, g, l)
    assert ei.value.code == lst.LST_E_CAPACITY
    torch.cuda.synchronize()
    assert bool((g == 7.0).all()) and l.item() == 7.0
