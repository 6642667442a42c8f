"""The Python binding's argument checks (a tensor of the wrong shape, dtype,
layout or device is refused before anything reaches the C ABI) and its
per-stream workspaces (two streams never share one)."""
import pytest
import torch

from scenes import scene_like_512

pytestmark = pytest.mark.gpu

from gpu_common import to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_02041_amd import Context
    return Context(0)


def test_wrong_shapes_are_refused(ctx):
    e = torch.zeros((32, 32), device="cuda")
    small = torch.zeros((16, 16), device="cuda")
    with pytest.raises(ValueError):
        ctx.hrc_forward(e, e, out=small)
    with pytest.raises(ValueError):
        ctx.hrc_forward(e, small)
    with pytest.raises(ValueError):
        ctx.hrc_backward(e, e, small)
    with pytest.raises(ValueError):
        ctx.hrc_backward(e, small, e)
    with pytest.raises(ValueError):
        ctx.hrc_multibounce_forward(e, e, small, 2)
    with pytest.raises(ValueError):
        ctx.hrc_multibounce_backward(e, e, e, 2, small)
    with pytest.raises(ValueError):
        ctx.hrc_forward(e, e, out=torch.zeros((32, 32), device="cuda", dtype=torch.float64))
    with pytest.raises(ValueError):
        ctx.hrc_forward(e, torch.zeros((32, 64), device="cuda")[:, ::2])  # not contiguous
    with pytest.raises(ValueError):
        ctx.hrc_forward(e, e.cpu())


def test_streams_have_their_own_workspaces(ctx):
    sc_a = scene_like_512(256, 81, 8, 16)
    sc_b = scene_like_512(256, 82, 8, 16)
    ea, sa, eb, sb = to_dev(sc_a.eps), to_dev(sc_a.sigma), to_dev(sc_b.eps), to_dev(sc_b.sigma)
    want_a = ctx.hrc_forward(ea, sa).clone()
    want_b = ctx.hrc_forward(eb, sb).clone()
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for _ in range(3):
        with torch.cuda.stream(s1):
            fa = ctx.hrc_forward(ea, sa)
        with torch.cuda.stream(s2):
            fb = ctx.hrc_forward(eb, sb)
        outs.append((fa, fb))
    torch.cuda.synchronize()
    for fa, fb in outs:
        assert torch.equal(fa, want_a) and torch.equal(fb, want_b)
    keys = [k for k in ctx._ws if k[:3] == (8, False, 0)]
    assert len({k[3] for k in keys}) >= 3  # the default stream, s1 and s2
