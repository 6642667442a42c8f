"""GPU parity of environment lighting (hrc_set_environment: light from beyond
the grid) through the C ABI, against the oracle's forward and reverse passes,
and the closed form F = 2 pi E for a uniform map in vacuum."""
import math

import numpy as np
import pytest
import torch

from oracle import hrc as oracle
from oracle import hrc_vjp
from scenes import config2, scene_like_512

pytestmark = pytest.mark.gpu

from gpu_common import assert_forward_close, assert_grad_close, log, to_dev  # noqa: E402


@pytest.fixture()
def ctx():
    from paper_2505_02041_amd import Context
    c = Context(0)
    yield c
    c.set_environment(None)


def _env(K, seed):
    return np.random.default_rng(seed).uniform(0.2, 2.0, K).astype(np.float32)


def _random_scene(S, seed):
    rng = np.random.default_rng(seed)
    eps = (rng.uniform(0, 3, (S, S)) * (rng.random((S, S)) < 0.3)).astype(np.float32)
    sig = rng.uniform(0, 1.5, (S, S)).astype(np.float32)
    return eps, sig


@pytest.mark.parametrize("S", [8, 256])
def test_uniform_environment_in_vacuum(ctx, S):
    log(f"uniform environment S={S}")
    ctx.set_environment([1.5])
    z = torch.zeros((S, S), device="cuda")
    F = ctx.hrc_forward(z, z).cpu().numpy().astype(np.float64)
    assert np.allclose(F, 2 * math.pi * 1.5, rtol=2e-6, atol=0)


@pytest.mark.parametrize("S,K", [(8, 4), (16, 2), (64, 16), (128, 61)])
def test_environment_forward_matches_oracle(ctx, S, K):
    log(f"environment forward S={S} K={K}")
    if S == 128:
        sc = scene_like_512(S, 21, 6, 10)
        eps, sig = sc.eps, sc.sigma
    else:
        eps, sig = _random_scene(S, 30 + S)
    env = _env(K, S)
    ctx.set_environment(env)
    F = ctx.hrc_forward(to_dev(eps), to_dev(sig))
    torch.cuda.synchronize()
    want = oracle.fluence(eps, sig, environment=env.astype(np.float64))
    assert_forward_close(F.cpu().numpy(), want, f"environment S={S}")


@pytest.mark.parametrize("S", [8, 64, 256, 512])
def test_environment_backward_matches_oracle(ctx, S):
    """Up to the 512x512 configuration's scene (opaque boxes and fog), whose
    upper levels (N = 9) read the map through every off-grid lookup of the
    merge-down and interval adjoints."""
    log(f"environment backward S={S}")
    if S == 512:
        sc = config2()
        eps, sig = sc.eps, sc.sigma
    elif S == 256:
        sc = scene_like_512(S, 41, 12, 20)
        eps, sig = sc.eps, sc.sigma
    else:
        eps, sig = _random_scene(S, 40 + S)
    env = _env(12 if S < 256 else 64, 7 + S)
    dF = np.random.default_rng(S).normal(size=(S, S)).astype(np.float32)
    ctx.set_environment(env)
    ge, gs = ctx.hrc_backward(to_dev(eps), to_dev(sig), to_dev(dF))
    torch.cuda.synchronize()
    re, rs = hrc_vjp.fluence_vjp(eps, sig, dF, environment=env.astype(np.float64))
    assert_grad_close(ge.cpu().numpy(), re, f"d eps environment S={S}")
    assert_grad_close(gs.cpu().numpy(), rs, f"d sigma environment S={S}")


def test_quadrant_groupings_with_environment_are_bitwise_equal(ctx):
    eps, sig = _random_scene(64, 5)
    ctx.set_environment(_env(9, 1))
    e, s = to_dev(eps), to_dev(sig)
    outs = [ctx.hrc_forward(e, s, flags=f) for f in (0x10, 0x20, 0x30)]
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_removing_the_environment_restores_the_plain_result(ctx):
    eps, sig = _random_scene(32, 6)
    e, s = to_dev(eps), to_dev(sig)
    plain = ctx.hrc_forward(e, s).clone()
    ctx.set_environment(_env(5, 2))
    lit = ctx.hrc_forward(e, s).clone()
    ctx.set_environment(None)
    again = ctx.hrc_forward(e, s)
    torch.cuda.synchronize()
    assert not torch.equal(plain, lit)
    assert torch.equal(plain, again)


def test_environment_with_blur_and_profile(ctx):
    from oracle import blur as oracle_blur
    eps, sig = _random_scene(32, 8)
    env = _env(7, 3)
    ctx.set_environment(env)
    e, s = to_dev(eps), to_dev(sig)
    F = ctx.hrc_forward(e, s, flags=0x2)
    torch.cuda.synchronize()
    want = oracle_blur.cross_blur(oracle.fluence(eps, sig, environment=env.astype(np.float64)), sig)
    assert_forward_close(F.cpu().numpy(), want, "environment + blur")
    _, Fp = ctx.hrc_profile_solve(e, s, return_outputs=True)
    assert torch.equal(Fp, ctx.hrc_forward(e, s))


def test_environment_rejects_bad_radiance(ctx):
    from paper_2505_02041_amd._lib import HRCError
    with pytest.raises(HRCError):
        ctx.set_environment([1.0, float("nan")])
