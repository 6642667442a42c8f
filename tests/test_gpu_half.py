"""The 16-bit interval storage (HRC_FLAG_HALF_INTERVALS, the storage of
Section 5) against the FP64 oracle: the forward within the bound derived from
the arithmetic (tests/gpu_common.py, pinned on the oracle's own steps in
tests/test_oracle_half_storage.py), and the reverse with its recomputed
forward stored so, within the bound on each gradient term."""
import numpy as np
import pytest
import torch

from oracle import hrc as oracle
from scenes import config1, config2, config3

pytestmark = pytest.mark.gpu

from gpu_common import assert_forward_close, assert_half_close, assert_half_grad, log, to_dev  # noqa: E402

HALF = 0x4


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_02041_amd import Context
    return Context(0)


def _run(ctx, eps, sig, flags=HALF):
    F = ctx.hrc_forward(to_dev(eps), to_dev(sig), flags=flags)
    torch.cuda.synchronize()
    return F.cpu().numpy()


def _random_scene(S, seed):
    rng = np.random.default_rng(seed)
    eps = (rng.uniform(0, 3, (S, S)) * (rng.random((S, S)) < 0.2)).astype(np.float32)
    sig = rng.uniform(0, 2, (S, S)).astype(np.float32)
    return eps, sig


@pytest.mark.parametrize("S", [8, 16, 64, 256])
def test_half_random_scenes(ctx, S):
    log(f"half intervals, random S={S}")
    eps, sig = _random_scene(S, 300 + S)
    N = S.bit_length() - 1
    assert_half_close(_run(ctx, eps, sig), oracle.fluence(eps, sig), N, f"S={S}")


@pytest.mark.parametrize("which", ["64", "512", "1024"])
def test_half_benchmark_configurations(ctx, which):
    """The three forward configurations, every pixel; the stored levels do
    round (the result is not the FP32 one)."""
    log(f"half intervals, configuration {which}")
    sc = {"64": config1, "512": config2, "1024": config3}[which]()
    N = sc.eps.shape[0].bit_length() - 1
    Fh = _run(ctx, sc.eps, sc.sigma)
    worst = assert_half_close(Fh, oracle.fluence(sc.eps, sc.sigma), N, which)
    log(f"  worst relative error (|F| > 1e-3 max): {worst:.2e}")
    assert not np.array_equal(Fh, _run(ctx, sc.eps, sc.sigma, 0))


def test_half_max_size_against_fp32(ctx):
    """S = 4096 (the largest size), against the FP32 path (itself within 1e-4
    of the oracle at every tested size)."""
    log("half intervals, 4096 vs FP32")
    from scenes import scene_like_512
    sc = scene_like_512(4096, 7, 128, 256)
    assert_half_close(_run(ctx, sc.eps, sc.sigma), _run(ctx, sc.eps, sc.sigma, 0), 12, "4096")
    ctx.release_workspaces()


def test_half_groupings_and_repeat_are_bitwise_equal(ctx):
    log("half intervals, quadrant groupings")
    eps, sig = _random_scene(128, 77)
    ref = _run(ctx, eps, sig)
    for g in (0x10, 0x20, 0x30):
        assert np.array_equal(_run(ctx, eps, sig, HALF | g), ref), hex(g)
    assert np.array_equal(_run(ctx, eps, sig), ref)


def test_half_with_environment_and_blur(ctx):
    """The other forward options combine with the storage: environment light
    (vs the oracle with the same map) and the cross blur (vs the FP32 blur)."""
    log("half intervals, environment and blur")
    eps, sig = _random_scene(64, 91)
    env = [float(np.float32(0.5 + 0.25 * np.cos(2 * np.pi * k / 16))) for k in range(16)]
    ctx.set_environment(env)
    try:
        assert_half_close(_run(ctx, eps, sig), oracle.fluence(eps, sig, environment=env), 6, "env")
    finally:
        ctx.set_environment(None)
    assert_half_close(_run(ctx, eps, sig, HALF | 0x2), _run(ctx, eps, sig, 0x2), 6, "blur")


def test_fp32_path_unchanged_by_the_option(ctx):
    """The FP32 forward still meets its 1e-4 bar on the same scene."""
    eps, sig = _random_scene(64, 12)
    assert_forward_close(_run(ctx, eps, sig, 0), oracle.fluence(eps, sig), "fp32")


# ---- the reverse with the 16-bit storage ------------------------------------

@pytest.mark.parametrize("case", ["random8", "random64", "config1", "random256", "config3"])
def test_half_backward_within_derived_bound(ctx, case):
    """hrc_backward with HRC_FLAG_HALF_INTERVALS against the oracle's FP64
    reverse pass, up to the 1024x1024 benchmark scene."""
    from oracle import hrc_vjp
    log(f"16-bit reverse {case}")
    if case == "config1":
        sc = config1()
        eps, sig = sc.eps, sc.sigma
    elif case == "config3":
        sc = config3()
        eps, sig = sc.eps, sc.sigma
    else:
        S = int(case[len("random"):])
        eps, sig = _random_scene(S, 70 + S)
    S = eps.shape[0]
    N = S.bit_length() - 1
    dF = np.random.default_rng(S + 1).normal(size=(S, S)).astype(np.float32)
    ge, gs = ctx.hrc_backward(to_dev(eps), to_dev(sig), to_dev(dF), flags=HALF)
    torch.cuda.synchronize()
    re, rs = hrc_vjp.fluence_vjp(eps, sig, dF)
    ae, as_ = hrc_vjp.fluence_vjp(eps, sig, np.abs(dF))
    assert_half_grad(ge.cpu().numpy(), re, ae, N, f"d eps {case}")
    assert_half_grad(gs.cpu().numpy(), rs, as_, N, f"d sigma {case}")
    # the storage does round (the check is not vacuous)
    ge32, _ = ctx.hrc_backward(to_dev(eps), to_dev(sig), to_dev(dF))
    assert not torch.equal(ge, ge32) or S <= 8
    ctx.release_workspaces()
