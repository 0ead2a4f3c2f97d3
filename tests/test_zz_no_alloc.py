"""The allocation-free gradient entry point against the trainer's gradient:
same kernels, same fixed-order reductions, so bit-identical, on two calls in
a row (the second with a smaller batch), and its size check."""
import numpy as np
import pytest
import torch

from paper_2105_00448_amd import hca

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def test_gradient_noalloc_equals_trainer_gradient():
    rng = np.random.default_rng(77)
    n = 3000
    X = (rng.standard_normal((n, 6)) * 2 + 1).astype(np.float32)
    Y = rng.standard_normal((n, 3)).astype(np.float32)
    Xd = torch.tensor(X, device=DEV)
    Yd = torch.tensor(Y, device=DEV)
    tr = hca.Trainer(Xd, Yd, seed=5)
    tr.train(20, batch=256, lr=1e-3)          # parameters away from the initial ones
    theta = torch.tensor(tr.params(), device=DEV)
    Xs = torch.empty((n, 6), device=DEV)
    Ys = torch.empty((n, 3), device=DEV)
    tr.data(Xs, Ys)
    stream = torch.cuda.current_stream().cuda_stream
    for batch in (1024, 192):
        print(f"\n[noalloc] batch {batch}", flush=True)
        idx = torch.tensor(rng.integers(0, n, batch).astype(np.int32), device=DEV)
        g_ref = torch.empty(hca.MLP_NPARAM, device=DEV)
        loss_ref = tr.gradient(idx, g_ref)
        g = torch.full((hca.MLP_NPARAM,), float("nan"), device=DEV)
        loss = torch.full((1,), float("nan"), device=DEV)
        hca.mlp_gradient_noalloc(theta, Xs, Ys, idx, g, loss, stream=stream)
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref), batch
        assert loss.item() == loss_ref, (loss.item(), loss_ref)
    # sizes beyond the static scratch, and batches that are not multiples of 64
    g = torch.empty(hca.MLP_NPARAM, device=DEV)
    big = torch.zeros(4096 + 64, dtype=torch.int32, device=DEV)
    for b in (4096 + 64, 100, 0):
        st = hca.lib().hca_mlp_gradient_noalloc(theta.data_ptr(), Xs.data_ptr(), Ys.data_ptr(), n,
                                                big.data_ptr(), b, g.data_ptr(), None, None)
        assert st == hca.E_RANGE, (b, st)
    tr.close()
