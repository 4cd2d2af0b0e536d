"""The streaming bandwidth probe (fipt_hbm_stream) moves the right data:
copy and triad are exact, including a ragged length (a tail of fewer than
four floats) and one float."""
import pytest
import torch

from paper_2304_05669_amd import fipt

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


@pytest.mark.parametrize("n", [1, 3, 1024, 1_000_003])
def test_copy_and_triad_exact(n):
    g = torch.Generator().manual_seed(n)
    a = torch.randn(n, generator=g).to(DEV)
    b = torch.randn(n, generator=g).to(DEV)
    c = torch.full((n,), float("nan"), device=DEV)
    fipt.fipt_hbm_stream(0, a, c)
    torch.cuda.synchronize()
    assert torch.equal(c, a)
    fipt.fipt_hbm_stream(1, a, c, b, s=0.5)
    torch.cuda.synchronize()
    # a + 0.5 b: one rounding in either order of evaluation (0.5 b is exact)
    assert torch.equal(c, a + 0.5 * b)
