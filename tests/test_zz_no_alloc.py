"""The allocation-free loss (mdfnn_mse_noalloc) against mdfnn_mse with a
caller-owned scratch buffer: the same loss and gradient, bit for bit, on two
calls in a row, the second with fewer pixels (the static scratch keeps the
first call's partial sums, which the second must not pick up)."""
import sys

import numpy as np
import pytest
import torch

from paper_2108_08591_amd import nn

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _inputs(P, C, seed):
    g = torch.Generator().manual_seed(seed)
    y = torch.randn(P, C, generator=g, dtype=torch.float32)
    t = torch.randn(P, C, generator=g, dtype=torch.float32)
    wt = (torch.rand(P, generator=g) > 0.2).to(torch.float32)
    return y.to(DEV), t.to(DEV), wt.to(DEV)


def test_noalloc_loss_equals_scratch_loss_on_two_calls():
    for P, C, seed in ((256 * 300 + 77, 7, 1), (1000, 7, 2)):
        print(f"[no-alloc] mse P={P} C={C}", flush=True)
        sys.stdout.flush()
        y, t, wt = _inputs(P, C, seed)
        dy_a = torch.empty_like(y)
        dy_b = torch.full_like(y, float("nan"))
        loss_a = torch.zeros(1, device=DEV)
        loss_b = torch.full((1,), float("nan"), device=DEV)
        scratch = torch.empty(nn.loss_scratch_bytes(P), dtype=torch.uint8, device=DEV)
        nn.mse(y, t, wt, dy_a, loss_a, scratch)
        nn.mse_noalloc(y, t, wt, dy_b, loss_b)
        torch.cuda.synchronize()
        assert torch.equal(loss_a, loss_b)
        assert torch.equal(dy_a, dy_b)
        # and the loss is the weighted mean square error in FP64 to FP32 rounding
        yd, td, wd = y.double().cpu(), t.double().cpu(), wt.double().cpu()
        ref = float(((yd - td) ** 2 * wd[:, None]).sum() / (wd.sum() * C))
        assert abs(float(loss_b) / ref - 1) < 1e-5
