"""GPU parity of the RGB solve (hrc_forward_rgb / hrc_backward_rgb: three
emission channels over one attenuation, sharing every transmittance and its
adjoint) through the C ABI: each channel's fluence and d emission bitwise equal
to the one-channel calls, d sigma against the sum of three oracle reverses, up
to the 1024x1024 benchmark scene, the reserve-space pair, and autograd."""
import numpy as np
import pytest
import torch

from oracle import blur as oracle_blur
from oracle import hrc as oracle
from oracle import hrc_vjp
from scenes import config3, scene_like_512

pytestmark = pytest.mark.gpu

from gpu_common import (assert_forward_close, assert_grad_close, assert_half_close,  # noqa: E402
                        assert_half_grad, log, to_dev)


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_02041_amd import Context
    return Context(0)


def _rgb_scene(S, seed):
    """Three emission channels over one attenuation: the channels are the
    scene's emission, a second seeded scene's emission, and their mix."""
    if S >= 128:
        a = scene_like_512(S, seed, max(2, S // 32), max(4, S // 16))
        b = scene_like_512(S, seed + 1, max(2, S // 32), 2)
        eps = np.stack([a.eps, b.eps, 0.5 * a.eps + 0.25 * b.eps]).astype(np.float32)
        return eps, a.sigma
    rng = np.random.default_rng(seed)
    eps = (rng.uniform(0, 3, (3, S, S)) * (rng.random((3, S, S)) < 0.3)).astype(np.float32)
    sig = rng.uniform(0, 1.5, (S, S)).astype(np.float32)
    return eps, sig


@pytest.mark.parametrize("S", [8, 16, 64, 256])
@pytest.mark.parametrize("flags", [0, 0x2], ids=["plain", "blur"])
def test_rgb_forward_equals_one_channel_calls(ctx, S, flags):
    log(f"rgb forward S={S} flags {flags:#x}")
    eps, sig = _rgb_scene(S, 10 + S)
    e, s = to_dev(eps), to_dev(sig)
    F = ctx.hrc_forward_rgb(e, s, flags=flags)
    for c in range(3):
        assert torch.equal(F[c], ctx.hrc_forward(e[c].contiguous(), s, flags=flags)), c


@pytest.mark.parametrize("S", [8, 64, 256])
def test_rgb_forward_matches_oracle(ctx, S):
    log(f"rgb forward vs oracle S={S}")
    eps, sig = _rgb_scene(S, 20 + S)
    F = ctx.hrc_forward_rgb(to_dev(eps), to_dev(sig)).cpu().numpy()
    for c in range(3):
        assert_forward_close(F[c], oracle.fluence(eps[c], sig), f"rgb channel {c} S={S}")


def test_rgb_forward_benchmark_scene_matches_oracle(ctx):
    """The 1024x1024 benchmark scene's attenuation with three emission channels
    (its own emission, a shifted copy, a scaled copy) against three oracle
    solves."""
    log("rgb forward 1024 vs oracle")
    sc = config3()
    eps = np.stack([sc.eps, np.roll(sc.eps, 37, axis=1), 0.3 * sc.eps]).astype(np.float32)
    F = ctx.hrc_forward_rgb(to_dev(eps), to_dev(sc.sigma)).cpu().numpy()
    for c in range(3):
        assert_forward_close(F[c], oracle.fluence(eps[c], sc.sigma), f"rgb 1024 channel {c}")
    ctx.release_workspaces()


@pytest.mark.parametrize("S,flags", [(8, 0), (64, 0), (256, 0), (64, 0x2)])
def test_rgb_backward(ctx, S, flags):
    """d emission per channel bitwise equal to the one-channel reverse (its
    radiance adjoints never meet the transmittance adjoints); d sigma, which the
    RGB reverse gathers over the channels inside, close to the sum of the three
    one-channel d sigma; both against the oracle's reverse."""
    log(f"rgb backward S={S} flags {flags:#x}")
    eps, sig = _rgb_scene(S, 30 + S)
    dF = np.random.default_rng(S).normal(size=(3, S, S)).astype(np.float32)
    e, s, g = to_dev(eps), to_dev(sig), to_dev(dF)
    ge, gs = ctx.hrc_backward_rgb(e, s, g, flags=flags)
    parts = [ctx.hrc_backward(e[c].contiguous(), s, g[c].contiguous(), flags=flags)
             for c in range(3)]
    for c in range(3):
        assert torch.equal(ge[c], parts[c][0]), c
    assert_grad_close(gs.cpu().numpy(), ((parts[0][1] + parts[1][1]) + parts[2][1]).cpu().numpy(),
                      f"rgb d sigma vs three one-channel reverses S={S}")
    ge, gs = ge.cpu().numpy(), gs.cpu().numpy()
    rs = np.zeros((S, S))
    for c in range(3):
        d = dF[c] if not flags else oracle_blur.cross_blur_vjp(dF[c], sig)
        re, rsc = hrc_vjp.fluence_vjp(eps[c], sig, d)
        assert_grad_close(ge[c], re, f"rgb d eps channel {c} S={S}")
        rs += rsc
    assert_grad_close(gs, rs, f"rgb d sigma S={S}")


def test_rgb_backward_benchmark_scene(ctx):
    """The 1024x1024 benchmark scene's medium with three emission channels:
    d emission per channel bitwise equal to the one-channel reverse and, like
    d sigma, within the gradient tolerance of three oracle reverses."""
    log("rgb backward 1024 vs oracle reverse")
    sc = config3()
    eps = np.stack([sc.eps, np.roll(sc.eps, 37, axis=1), 0.3 * sc.eps]).astype(np.float32)
    dF = np.random.default_rng(11).normal(size=(3, 1024, 1024)).astype(np.float32)
    e, s, g = to_dev(eps), to_dev(sc.sigma), to_dev(dF)
    ge, gs = ctx.hrc_backward_rgb(e, s, g)
    for c in range(3):
        gc = ctx.hrc_backward(e[c].contiguous(), s, g[c].contiguous())[0]
        assert torch.equal(ge[c], gc), c
    torch.cuda.synchronize()
    ge, gs = ge.cpu().numpy(), gs.cpu().numpy()
    ctx.release_workspaces()
    rs = np.zeros((1024, 1024))
    for c in range(3):
        re, rsc = hrc_vjp.fluence_vjp(eps[c], sc.sigma, dF[c])
        assert_grad_close(ge[c], re, f"rgb 1024 d eps channel {c}")
        rs += rsc
    assert_grad_close(gs, rs, "rgb 1024 d sigma")


def test_rgb_largest_grid_equals_one_channel_calls(ctx):
    """At 4096x4096, the largest grid, where the element offsets into the
    channel planes and the interval levels are largest: each channel's fluence
    and d emission bitwise those of the one-channel calls, d sigma within the
    gradient tolerance of the sum of the three one-channel d sigma."""
    S = 4096
    log("rgb forward and backward S=4096 vs one-channel calls")
    g = torch.Generator(device="cuda").manual_seed(S)
    sig = torch.rand((S, S), device="cuda", generator=g) * 0.5
    eps = torch.rand((3, S, S), device="cuda", generator=g) * (
        torch.rand((3, S, S), device="cuda", generator=g) < 0.05)
    dF = torch.randn((3, S, S), device="cuda", generator=g)
    F = ctx.hrc_forward_rgb(eps, sig)
    for c in range(3):
        assert torch.equal(F[c], ctx.hrc_forward(eps[c].contiguous(), sig)), c
    del F
    ge, gs = ctx.hrc_backward_rgb(eps, sig, dF)
    gs_sum = torch.zeros_like(sig)
    for c in range(3):
        pe, ps = ctx.hrc_backward(eps[c].contiguous(), sig, dF[c].contiguous())
        assert torch.equal(ge[c], pe), c
        gs_sum += ps
    torch.cuda.synchronize()
    assert_grad_close(gs.cpu().numpy(), gs_sum.cpu().numpy(), "rgb d sigma S=4096")
    del ge, gs, gs_sum
    ctx.release_workspaces()


@pytest.mark.parametrize("S,flags", [(8, 0), (64, 0x2), (256, 0), (1024, 0)])
def test_rgb_kept_forward_and_reused_backward(ctx, S, flags):
    """The reserve-space pair for RGB: the kept forward's fluence and the
    reused reverse's gradients bitwise those of the plain RGB calls, twice."""
    from paper_2505_02041_amd import _lib
    log(f"rgb keep/reuse S={S} flags {flags:#x}")
    eps, sig = _rgb_scene(S, 60 + S)
    e, s = to_dev(eps), to_dev(sig)
    res = ctx.reserve_rgb(S.bit_length() - 1)
    Fk = ctx.hrc_forward_rgb(e, s, flags=flags | _lib.HRC_FLAG_KEEP_PYRAMID, reserve=res)
    F = ctx.hrc_forward_rgb(e, s, flags=flags)
    assert torch.equal(Fk, F)
    for seed in (1, 2):
        g = to_dev(np.random.default_rng(seed).normal(size=(3, S, S)).astype(np.float32))
        gk = ctx.hrc_backward_rgb(e, s, g, flags=flags | _lib.HRC_FLAG_REUSE_PYRAMID, reserve=res)
        gp = ctx.hrc_backward_rgb(e, s, g, flags=flags)
        assert torch.equal(gk[0], gp[0]) and torch.equal(gk[1], gp[1])
    del res
    ctx.release_workspaces()


def test_rgb_autograd(ctx):
    from paper_2505_02041_amd import fluence_rgb
    eps, sig = _rgb_scene(32, 40)
    e = to_dev(eps).requires_grad_(True)
    s = to_dev(sig).requires_grad_(True)
    g = torch.randn((3, 32, 32), device="cuda")
    for keep in (True, False):
        e.grad = s.grad = None
        F = fluence_rgb(e, s, keep=keep)
        F.backward(g)
        ge, gs = ctx.hrc_backward_rgb(to_dev(eps), to_dev(sig), g)
        assert torch.equal(e.grad, ge) and torch.equal(s.grad, gs)
        assert torch.equal(F.detach(), ctx.hrc_forward_rgb(to_dev(eps), to_dev(sig)))


@pytest.mark.parametrize("S", [8, 64, 256])
def test_rgb_half_storage(ctx, S):
    """The paper's storage (16-bit RGB intervals): each channel bitwise equal to
    the one-channel 16-bit forward (the same values rounded at the same points)
    and within the derived bound N 2^-11 of the oracle."""
    log(f"rgb 16-bit forward S={S}")
    eps, sig = _rgb_scene(S, 50 + S)
    e, s = to_dev(eps), to_dev(sig)
    F = ctx.hrc_forward_rgb(e, s, flags=0x4)
    N = S.bit_length() - 1
    for c in range(3):
        assert torch.equal(F[c], ctx.hrc_forward(e[c].contiguous(), s, flags=0x4)), c
        assert_half_close(F[c].cpu().numpy(), oracle.fluence(eps[c], sig), N,
                          f"rgb 16-bit channel {c} S={S}")


def test_rgb_half_storage_benchmark_scene(ctx):
    log("rgb 16-bit forward 1024 vs oracle")
    sc = config3()
    eps = np.stack([sc.eps, np.roll(sc.eps, 37, axis=1), 0.3 * sc.eps]).astype(np.float32)
    F = ctx.hrc_forward_rgb(to_dev(eps), to_dev(sc.sigma), flags=0x4).cpu().numpy()
    for c in range(3):
        assert_half_close(F[c], oracle.fluence(eps[c], sc.sigma), 10, f"rgb 16-bit 1024 ch {c}")
    ctx.release_workspaces()


@pytest.mark.parametrize("S", [64, 256, 1024])
def test_rgb_half_backward(ctx, S):
    """The RGB reverse with the paper's 16-bit storage: d emission per channel
    bitwise equal to the one-channel 16-bit reverse (the same values rounded at
    the same points); both gradients within N 2^-11 times the gradient of
    abs(dLoss/dF) of three oracle reverses, as the one-channel 16-bit reverse;
    the reserve-space pair bitwise equal to the plain call."""
    from paper_2505_02041_amd import _lib
    log(f"rgb 16-bit reverse S={S}")
    H = _lib.HRC_FLAG_HALF_INTERVALS
    if S == 1024:
        sc = config3()
        eps = np.stack([sc.eps, np.roll(sc.eps, 37, axis=1), 0.3 * sc.eps]).astype(np.float32)
        sig = sc.sigma
    else:
        eps, sig = _rgb_scene(S, 80 + S)
    N = S.bit_length() - 1
    dF = np.random.default_rng(S + 3).normal(size=(3, S, S)).astype(np.float32)
    e, s, g = to_dev(eps), to_dev(sig), to_dev(dF)
    ge, gs = ctx.hrc_backward_rgb(e, s, g, flags=H)
    for c in range(3):
        assert torch.equal(ge[c], ctx.hrc_backward(e[c].contiguous(), s, g[c].contiguous(),
                                                   flags=H)[0]), c
    res = ctx.reserve_rgb(N, H)
    ctx.hrc_forward_rgb(e, s, flags=H | _lib.HRC_FLAG_KEEP_PYRAMID, reserve=res)
    gk = ctx.hrc_backward_rgb(e, s, g, flags=H | _lib.HRC_FLAG_REUSE_PYRAMID, reserve=res)
    assert torch.equal(gk[0], ge) and torch.equal(gk[1], gs)
    torch.cuda.synchronize()
    ge, gs = ge.cpu().numpy(), gs.cpu().numpy()
    del res
    ctx.release_workspaces()
    rs = np.zeros((S, S))
    as_ = np.zeros((S, S))
    for c in range(3):
        re, rsc = hrc_vjp.fluence_vjp(eps[c], sig, dF[c])
        ae, asc = hrc_vjp.fluence_vjp(eps[c], sig, np.abs(dF[c]))
        assert_half_grad(ge[c], re, ae, N, f"rgb 16-bit d eps channel {c} S={S}")
        rs += rsc
        as_ += asc
    assert_half_grad(gs, rs, as_, N, f"rgb 16-bit d sigma S={S}")


def test_rgb_rejects_bad_arguments(ctx):
    from paper_2505_02041_amd._lib import HRCError
    z = torch.zeros((3, 16, 16), device="cuda")
    s = torch.zeros((16, 16), device="cuda")
    with pytest.raises(HRCError):
        ctx.hrc_forward_rgb(z, s, flags=0x10)  # no quadrant grouping for RGB
    with pytest.raises(HRCError):
        ctx.hrc_backward_rgb(z, s, z, flags=0x10)  # no quadrant grouping for RGB
    with pytest.raises(ValueError):
        ctx.hrc_forward_rgb(z[:2].contiguous(), s)
