"""fipt_render_loss_noalloc (the render loss with its partial sums in the
library's static per-GPU array) against fipt_render_loss, through the C ABI:
two calls in a row, the second on fewer points, each bitwise equal to the
plain call on the same inputs (same kernels, same grid, same summation
order), and the loss also within 1e-6 of the oracle's float64 loss."""
import numpy as np
import pytest
import torch

import synth
from oracle import render as orr
from paper_2304_05669_amd import fipt

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
SIG32 = tuple(float(s) for s in np.asarray(synth.SIGMA_GRID, np.float32))


def _inputs(n, seed):
    shade = synth.random_shading(n, len(SIG32), seed=seed)
    mat = synth.random_materials(n, seed=seed + 1)
    obs = synth.random_observations(n, seed=seed + 2)
    return shade, mat, obs


def _both(shade, mat, obs, tonemap):
    S, M, O = (torch.from_numpy(a).to(DEV) for a in (shade, mat, obs))
    n = M.shape[1]
    ref_buf, ref_grad, ref_lr = fipt.fipt_render_loss(S, M, O, SIG32, tonemap=tonemap, want_lr=True)
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    grad = torch.full((5, n), float("nan"), dtype=torch.float32, device=DEV)
    lr = torch.full((3, n), float("nan"), dtype=torch.float32, device=DEV)
    fipt.fipt_render_loss_noalloc(S, M, O, SIG32, loss, grad, lr, tonemap=tonemap)
    torch.cuda.synchronize()
    return (ref_buf[0].item(), ref_grad.cpu().numpy(), ref_lr.cpu().numpy(), loss.item(),
            grad.cpu().numpy(), lr.cpu().numpy())


@pytest.mark.parametrize("tonemap", [fipt.TONEMAP_NONE, fipt.TONEMAP_LOG_SRGB])
def test_noalloc_equals_plain_call_twice_shrinking(tonemap):
    # the first call fills all 2048 partial slots (more than 2048 x 256
    # points), the second uses 4 of them: stale slots must not leak in
    for n, seed in ((600_001, 11), (1_000, 21)):
        shade, mat, obs = _inputs(n, seed)
        l_ref, g_ref, lr_ref, l, g, lr = _both(shade, mat, obs, tonemap)
        assert l == l_ref, (n, l, l_ref)
        np.testing.assert_array_equal(g, g_ref)
        np.testing.assert_array_equal(lr, lr_ref)
        want, _, _ = orr.loss_and_grad(shade, mat, obs, SIG32, tone=tonemap)
        assert abs(l - want) <= 1e-6 * abs(want), (n, l, want)


def test_noalloc_loss_only_and_one_point():
    shade, mat, obs = _inputs(1, 5)
    S, M, O = (torch.from_numpy(a).to(DEV) for a in (shade, mat, obs))
    loss = torch.zeros((1,), dtype=torch.float64, device=DEV)
    fipt.fipt_render_loss_noalloc(S, M, O, SIG32, loss)
    ref, _, _ = fipt.fipt_render_loss(S, M, O, SIG32, want_grad=False)
    torch.cuda.synchronize()
    assert loss.item() == ref[0].item()
    with pytest.raises(ValueError):
        fipt.fipt_render_loss_noalloc(S, M, O, SIG32, torch.zeros((2,), dtype=torch.float64, device=DEV))
