"""erf_mlp_loss_grad_noalloc (include/erf_mlp.h), the allocation-free variant
of erf_mlp_loss_grad for callers that cannot allocate, against the allocating
call through the C-ABI.  Both run the same kernels with the same split of the
long reductions, so the gradient and the loss agree bit for bit (stronger than
the FP32 accumulation bound the gradient parity tests use).  Two calls in a
row, the second on a smaller batch, show that nothing left in the shared
scratch by one call leaks into the next."""
import sys

import numpy as np
import pytest

from paper_2412_04395_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_loss_grad_noalloc_matches_the_allocating_call():
    import torch
    from paper_2412_04395_amd import erf

    cfg = W.les_mlp(nx=16, ny=16, nz=8, dz=W.uniform_dz(8, 40.0))  # the context only holds the network
    s = erf.Solver(cfg)
    p = np.random.default_rng(23).normal(0.0, 0.1, erf.MLP_NPARAMS).astype(np.float32)
    s.mlp_set_weights(p)
    gen = torch.Generator(device="cuda").manual_seed(23)
    sizes = (8192, 3001)  # the maximum batch, then a smaller ragged one
    batches, refs = [], []
    for n in sizes:
        x = torch.randn((n, 10), generator=gen, device="cuda", dtype=torch.float32)
        t = torch.randn((n, 9), generator=gen, device="cuda", dtype=torch.float32)
        loss_ref, g_ref = s.mlp_loss_grad(x, t)
        batches.append((x, t))
        refs.append((loss_ref, g_ref.clone()))
    torch.cuda.synchronize()
    for (x, t), (loss_ref, g_ref) in zip(batches, refs):
        n = x.shape[0]
        _say("noalloc loss_grad batch", n)
        g = torch.full((erf.MLP_NPARAMS,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        s.mlp_loss_grad_noalloc(x, t, g, loss)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(g).all())
        assert torch.equal(g, g_ref), float((g - g_ref).abs().max())
        assert loss.item() == loss_ref
    # beyond the maximum batch: a clear error before anything is launched
    n_big = erf.MLP_NOALLOC_MAX_BATCH + 1
    xb = torch.zeros((n_big, 10), dtype=torch.float32, device="cuda")
    tb = torch.zeros((n_big, 9), dtype=torch.float32, device="cuda")
    with pytest.raises(erf.ErfError) as ei:
        s.mlp_loss_grad_noalloc(xb, tb)
    assert ei.value.status == erf.ERF_E_ARG
    assert "ERF_MLP_NOALLOC_MAX_BATCH" in str(ei.value)
    s.close()
