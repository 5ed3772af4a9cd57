"""pm_quality_noalloc, the entry point that allocates nothing, called through
the C ABI and compared with pm_quality on the same handles: two calls in a
row, the second on a smaller mesh, then the same handle after coarsening has
shrunk it; and device memory is unchanged across repeated calls."""
import numpy as np
import pytest

from paper_1505_04694_amd import inputs, pmesh

pytestmark = pytest.mark.gpu


def same_as_pm_quality(gm):
    import torch
    V, _ = gm.sizes()
    Q1, m1, gx1, gd1 = pmesh.pm_quality(gm.h, grad=True)
    gx2 = torch.full((V, 2), float("nan"), dtype=torch.float64, device="cuda")
    gd2 = torch.full((V, 3), float("nan"), dtype=torch.float64, device="cuda")
    Q2, m2 = pmesh.pm_quality_noalloc(gm.h, gx2, gd2)
    # the same reduction over the same data: equal to the last bit
    assert Q2 == Q1 and m2 == m1, (Q1, Q2, m1, m2)
    assert torch.equal(gx1, gx2) and torch.equal(gd1, gd2)
    # without gradient outputs
    assert pmesh.pm_quality_noalloc(gm.h) == (Q1, m1)
    return Q1


def test_noalloc_quality_equals_pm_quality_on_two_calls_the_second_smaller():
    big = pmesh.Mesh.from_input(inputs.config2(1025), seed=1)
    small = pmesh.Mesh.from_input(inputs.config2(33), seed=1)
    # the first call fills all 2048 partial sums, the second only a few
    assert big.sizes()[1] > 256 * 2048 and small.sizes()[1] < 256 * 16
    same_as_pm_quality(big)
    same_as_pm_quality(small)
    big.coarsen()
    same_as_pm_quality(big)


def test_noalloc_quality_leaves_device_memory_unchanged():
    import torch
    gm = pmesh.Mesh.from_input(inputs.config2(129), seed=1)
    V, _ = gm.sizes()
    gx = torch.empty((V, 2), dtype=torch.float64, device="cuda")
    gd = torch.empty((V, 3), dtype=torch.float64, device="cuda")
    pmesh.pm_quality_noalloc(gm.h, gx, gd)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(5):
        pmesh.pm_quality_noalloc(gm.h, gx, gd)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
