"""hrc_forward_static (the forward on the library's own static device scratch,
for callers that cannot allocate) through the C ABI: bitwise equal to
hrc_forward with the same flags on two calls in a row, the second on a smaller
grid (the scratch keeps the first call's contents), and the size limit."""
import numpy as np
import pytest
import torch

from scenes import config2, scene_like_512

pytestmark = pytest.mark.gpu

from gpu_common import log, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_02041_amd import Context
    return Context(0)


def _both(ctx, eps, sig, flags):
    e, s = to_dev(eps), to_dev(sig)
    want = ctx.hrc_forward(e, s, flags=flags)
    got = torch.full_like(e, float("nan"))
    ctx.hrc_forward_static(e, s, got, flags=flags)
    torch.cuda.synchronize()
    return got, want


@pytest.mark.parametrize("flags", [0, 0x2, 0x4, 0x10],
                         ids=["plain", "blur", "half-intervals", "one-quadrant-at-a-time"])
def test_forward_static_matches_forward(ctx, flags):
    big = config2()  # 512^2, the largest grid the scratch holds
    small = scene_like_512(64, 61, 3, 4)
    for name, sc in (("512^2", big), ("64^2 after 512^2", small)):
        log(f"hrc_forward_static {name}, flags {flags:#x}")
        got, want = _both(ctx, sc.eps, sc.sigma, flags)
        assert torch.equal(got, want), name


def test_forward_static_limits(ctx):
    from paper_2505_02041_amd._lib import (HRC_ERR_TOO_LARGE, HRC_ERR_UNSUPPORTED, HRCError)
    z = torch.zeros((1024, 1024), device="cuda")
    with pytest.raises(HRCError) as e:
        ctx.hrc_forward_static(z, z, torch.empty_like(z))
    assert e.value.status == HRC_ERR_TOO_LARGE
    z = torch.zeros((64, 64), device="cuda")
    with pytest.raises(HRCError) as e:
        ctx.hrc_forward_static(z, z, torch.empty_like(z), flags=0x1)
    assert e.value.status == HRC_ERR_UNSUPPORTED
    # the smallest grid, after the limits were hit
    sc = scene_like_512(8, 62, 1, 1)
    got, want = _both(ctx, sc.eps, sc.sigma, 0)
    assert torch.equal(got, want)
