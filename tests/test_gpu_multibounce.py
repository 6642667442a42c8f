"""GPU parity of several diffuse bounces (hrc_multibounce_forward / _backward)
against the oracle's bounces and their reverse pass, the thick-medium closed
form, and the single-bounce and zero-albedo special cases."""
import math

import numpy as np
import pytest
import torch

from oracle import multibounce as oracle_mb
from scenes import scene_like_512

pytestmark = pytest.mark.gpu

from gpu_common import assert_forward_close, assert_grad_close, log, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_02041_amd import Context
    return Context(0)


def _scene(S, seed):
    rng = np.random.default_rng(seed)
    eps = (rng.uniform(0, 3, (S, S)) * (rng.random((S, S)) < 0.3)).astype(np.float32)
    sig = rng.uniform(0, 1.5, (S, S)).astype(np.float32)
    alb = rng.uniform(0, 0.9, (S, S)).astype(np.float32)
    return eps, sig, alb


@pytest.mark.parametrize("S,K", [(8, 2), (64, 3), (128, 4), (1024, 3)])
def test_multibounce_forward_matches_oracle(ctx, S, K):
    log(f"multibounce forward S={S} K={K}")
    if S >= 128:
        sc = scene_like_512(S, 51, max(6, S // 16), max(10, S // 8))
        eps, sig = sc.eps, sc.sigma
        alb = np.full((S, S), 0.7, np.float32)
    else:
        eps, sig, alb = _scene(S, S + K)
    F = ctx.hrc_multibounce_forward(to_dev(eps), to_dev(sig), to_dev(alb), K)
    torch.cuda.synchronize()
    assert_forward_close(F.cpu().numpy(), oracle_mb.fluence(eps, sig, alb, K),
                         f"bounces S={S} K={K}")


@pytest.mark.parametrize("S,K", [(8, 1), (16, 3), (64, 2), (256, 3), (512, 2)])
def test_multibounce_backward_matches_oracle(ctx, S, K):
    log(f"multibounce backward S={S} K={K}")
    if S == 512:
        sc = scene_like_512(S, 52, 32, 64)
        eps, sig = sc.eps, sc.sigma
        alb = np.random.default_rng(9).uniform(0, 0.9, (S, S)).astype(np.float32)
    else:
        eps, sig, alb = _scene(S, 100 + S + K)
    dF = np.random.default_rng(S).normal(size=(S, S)).astype(np.float32)
    ge, gs, ga = ctx.hrc_multibounce_backward(to_dev(eps), to_dev(sig), to_dev(alb), K,
                                              to_dev(dF))
    torch.cuda.synchronize()
    re, rs, ra = oracle_mb.fluence_vjp(eps, sig, alb, K, dF)
    assert_grad_close(ge.cpu().numpy(), re, f"d eps bounces S={S} K={K}")
    assert_grad_close(gs.cpu().numpy(), rs, f"d sigma bounces S={S} K={K}")
    if K > 1:
        assert_grad_close(ga.cpu().numpy(), ra, f"d albedo bounces S={S} K={K}")
    else:
        assert torch.count_nonzero(ga) == 0


def test_one_bounce_and_zero_albedo_are_the_single_solve(ctx):
    eps, sig, alb = _scene(32, 7)
    e, s = to_dev(eps), to_dev(sig)
    single = ctx.hrc_forward(e, s)
    one = ctx.hrc_multibounce_forward(e, s, to_dev(alb), 1)
    dark = ctx.hrc_multibounce_forward(e, s, torch.zeros_like(e), 4)
    torch.cuda.synchronize()
    assert torch.equal(single, one) and torch.equal(single, dark)


def test_thick_medium_geometric_series(ctx):
    S = 64
    eps0, sig, a, K = 0.7, 3.0, 0.6, 5
    F = ctx.hrc_multibounce_forward(torch.full((S, S), eps0, device="cuda"),
                                    torch.full((S, S), sig, device="cuda"),
                                    torch.full((S, S), a, device="cuda"), K)
    want = 2 * math.pi * eps0 / sig * sum(a ** j for j in range(K))
    centre = F[24:40, 24:40].cpu().numpy().astype(np.float64)
    assert np.allclose(centre, want, rtol=1e-4)


def test_multibounce_autograd_equals_backward(ctx):
    from paper_2505_02041_amd import fluence_multibounce
    eps, sig, alb = _scene(32, 9)
    e = to_dev(eps).requires_grad_(True)
    s = to_dev(sig).requires_grad_(True)
    a = to_dev(alb).requires_grad_(True)
    F = fluence_multibounce(e, s, a, 3)
    g = torch.randn_like(F)
    F.backward(g)
    ge, gs, ga = ctx.hrc_multibounce_backward(to_dev(eps), to_dev(sig), to_dev(alb), 3, g)
    torch.cuda.synchronize()
    assert torch.equal(e.grad, ge) and torch.equal(s.grad, gs) and torch.equal(a.grad, ga)
