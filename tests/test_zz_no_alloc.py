"""poisson_solve_static (the allocation-free variant of poisson_solve) against poisson_solve.

Both run the same kernels on the same inputs, so the results must agree bitwise; two calls
in a row, the second on a smaller box, show that the static scratch carries nothing from
one call into the next.  A box larger than the static array is refused before any launch.
"""
import numpy as np
import pytest
import torch

from paper_1705_01423_amd import _lib
from paper_1705_01423_amd._lib import PsError
from gpu_util import banner, grids

pytestmark = pytest.mark.gpu


def _rhs(plan, seed):
    rng = np.random.default_rng(seed)
    return torch.as_tensor(rng.standard_normal(plan.centre_shape)).to("cuda")


@pytest.mark.parametrize("prec", ["fp64", "fp32_refined"])
def test_static_matches_plan_workspace(prec):
    for shape, seed in (((96, 64, 48), 1), ((24, 12, 10), 2)):
        banner(f"static scratch {prec} {shape}")
        _, plan = grids(*shape, 2.0, 1.5, precision=prec)
        f = _rhs(plan, seed)
        ref, info_ref = plan.solve(f)
        got = torch.full_like(f, float("nan"))
        got, info = plan.solve_static(f, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), shape
        assert info["iterations"] == info_ref["iterations"]
        assert info["compat_defect"] == info_ref["compat_defect"]
        # the plan's own workspace is still in use afterwards
        again, _ = plan.solve(f)
        assert torch.equal(again, ref)


def test_static_refuses_large_box():
    _, plan = grids(512, 512, 384, 2.0, 2.0)
    assert plan.workspace_bytes() > 256 << 20
    f = torch.zeros(plan.centre_shape, dtype=torch.float64, device="cuda")
    with pytest.raises(PsError) as e:
        plan.solve_static(f)
    assert e.value.status == _lib.PS_EINVAL
    assert "static" in str(e.value)
