"""GPU parity of the cross blur of Eq. 21 (HRC_FLAG_BLUR) through the C ABI:
the blurred fluence against the oracle's blur of the oracle's fluence, and the
backward with the blur's transpose against the oracle's reverse pass.  The
scenes have opacity jumps (opaque boxes, random per-pixel attenuation), so
neighbours are ignored along their edges."""
import numpy as np
import pytest
import torch

from oracle import blur as oracle_blur
from oracle import hrc as oracle
from oracle import hrc_vjp
from scenes import config2, config3, scene_like_512

pytestmark = pytest.mark.gpu

from gpu_common import assert_forward_close, assert_grad_close, log, to_dev  # noqa: E402

BLUR = 0x2


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_02041_amd import Context
    return Context(0)


def _random_scene(S, seed):
    rng = np.random.default_rng(seed)
    eps = (rng.uniform(0, 3, (S, S)) * (rng.random((S, S)) < 0.3)).astype(np.float32)
    sig = rng.uniform(0, 1.5, (S, S)).astype(np.float32)
    return eps, sig


def _scenes():
    out = [("random8", *_random_scene(8, 11)), ("random64", *_random_scene(64, 12))]
    sc = scene_like_512(128, 13, 6, 10)
    out.append(("boxes128", sc.eps, sc.sigma))
    sc = scene_like_512(256, 14, 12, 20)
    out.append(("boxes256", sc.eps, sc.sigma))
    sc = config2()
    out.append(("config512", sc.eps, sc.sigma))
    return out


@pytest.mark.parametrize("case", [0, 1, 2], ids=["random8", "random64", "boxes128"])
def test_blurred_forward_matches_oracle(ctx, case):
    name, eps, sig = _scenes()[case]
    log(f"blurred forward {name}")
    F = ctx.hrc_forward(to_dev(eps), to_dev(sig), flags=BLUR)
    torch.cuda.synchronize()
    want = oracle_blur.cross_blur(oracle.fluence(eps, sig), sig)
    assert_forward_close(F.cpu().numpy(), want, f"blurred {name}")
    # the blur changes the fluence, and some neighbours are ignored
    assert not np.allclose(want, oracle.fluence(eps, sig))
    assert not oracle_blur.kept_neighbours(sig)[:, 1:-1, 1:-1].all()


def test_unblurred_forward_unchanged_by_the_flag_bit(ctx):
    _, eps, sig = _scenes()[1]
    a = ctx.hrc_forward(to_dev(eps), to_dev(sig))
    b = ctx.hrc_forward(to_dev(eps), to_dev(sig), flags=BLUR)
    torch.cuda.synchronize()
    assert not torch.equal(a, b)
    want = oracle_blur.cross_blur(a.cpu().numpy().astype(np.float64), sig)
    assert_forward_close(b.cpu().numpy(), want, "blur of the GPU's own fluence")


@pytest.mark.parametrize("case", [0, 1, 2, 3, 4],
                         ids=["random8", "random64", "boxes128", "boxes256", "config512"])
def test_blurred_backward_matches_oracle(ctx, case):
    name, eps, sig = _scenes()[case]
    log(f"blurred backward {name}")
    S = eps.shape[0]
    dF = np.random.default_rng(300 + case).normal(size=(S, S)).astype(np.float32)
    ge, gs = ctx.hrc_backward(to_dev(eps), to_dev(sig), to_dev(dF), flags=BLUR)
    torch.cuda.synchronize()
    re, rs = hrc_vjp.fluence_vjp(eps, sig, oracle_blur.cross_blur_vjp(dF, sig))
    assert_grad_close(ge.cpu().numpy(), re, f"d eps blurred {name}")
    assert_grad_close(gs.cpu().numpy(), rs, f"d sigma blurred {name}")


def test_blurred_autograd_equals_backward(ctx):
    from paper_2505_02041_amd import fluence
    _, eps, sig = _scenes()[1]
    e = to_dev(eps).requires_grad_(True)
    s = to_dev(sig).requires_grad_(True)
    F = fluence(e, s, blur=True)
    g = torch.randn_like(F)
    F.backward(g)
    ge, gs = ctx.hrc_backward(to_dev(eps), to_dev(sig), g, flags=BLUR)
    torch.cuda.synchronize()
    assert torch.equal(e.grad, ge) and torch.equal(s.grad, gs)
    assert torch.equal(F.detach(), ctx.hrc_forward(to_dev(eps), to_dev(sig), flags=BLUR))


def test_blurred_forward_benchmark_scene_1024(ctx):
    """The 1024x1024 benchmark scene (opaque boxes, sigma-100 lines, fog), blurred."""
    log("blurred forward 1024 benchmark scene")
    sc = config3()
    F = ctx.hrc_forward(to_dev(sc.eps), to_dev(sc.sigma), flags=BLUR)
    torch.cuda.synchronize()
    want = oracle_blur.cross_blur(oracle.fluence(sc.eps, sc.sigma), sc.sigma)
    assert_forward_close(F.cpu().numpy(), want, "blurred 1024")
