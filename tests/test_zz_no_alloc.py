"""The no-allocation product entry point (mmot_marginal_product_noalloc) against
the plan's product, which runs the same kernels with a plan-owned workspace:
two calls in a row on the shared per-GPU workspace, the second smaller, each
bit-for-bit equal to the plan's result (same kernel, same inputs)."""
import numpy as np
import pytest

from gpu_util import say, to_dev
from paper_2405_19246_amd import inputs

pytestmark = pytest.mark.gpu


def _rand_potentials(l, N, seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(l, N)) * 3.0
    if N > 2:
        a[0, 1] = -np.inf
    return a


@pytest.mark.parametrize("l,N1,N2,prec", [(4, 700, 300, 0), (3, 2000, 64, 1), (6, 150, 37, 0), (8, 200, 90, 0),
                                          (10, 30, 11, 1)])
def test_noalloc_product_matches_plan_on_two_calls(l, N1, N2, prec):
    import torch
    from paper_2405_19246_amd import mmot
    for N in (N1, N2):
        h, eps = inputs.grid_step(N), 0.05
        a = to_dev(_rand_potentials(l, N, 100 * l + N))
        plan = mmot.Plan(l, N, h, eps, precision=prec)
        for j in (0, l - 1):
            say("noalloc product l=%d N=%d j=%d prec=%d" % (l, N, j, prec))
            ref = plan.marginal_product(j, a).cpu().numpy()
            out = torch.full((N,), float("nan"), dtype=torch.float64, device=a.device)
            mmot.marginal_product_noalloc(l, N, h, eps, j, a, out, precision=prec)
            got = out.cpu().numpy()
            assert np.array_equal(got, ref), (l, N, j, np.nanmax(np.abs(got - ref)))
        plan.close()


def test_noalloc_rejects_a_problem_beyond_its_workspace():
    import torch
    from paper_2405_19246_amd import mmot
    l, N = 10, 200000
    a = torch.zeros((l, N), dtype=torch.float64, device="cuda:0")
    out = torch.zeros(N, dtype=torch.float64, device="cuda:0")
    with pytest.raises(mmot.MmotError) as e:
        mmot.marginal_product_noalloc(l, N, 1.0 / (N - 1), 0.01, 0, a, out)
    assert e.value.code == mmot.ERR_INVALID
