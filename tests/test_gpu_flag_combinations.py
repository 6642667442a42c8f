"""Every combination of the forward's options (and of the reverse's) on small ragged grids, each
against the FP64 oracle: quadrant grouping, cross blur, environment light and
16-bit interval storage (tolerances from tests/gpu_common.py)."""
import itertools

import numpy as np
import pytest
import torch

from oracle import blur as oracle_blur
from oracle import hrc as oracle

pytestmark = pytest.mark.gpu

from gpu_common import assert_forward_close, assert_half_close, log, to_dev  # noqa: E402

BLUR, HALF = 0x2, 0x4
GROUPS = (0, 0x10, 0x20)


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_02041_amd import Context
    return Context(0)


def _scene(S, seed):
    rng = np.random.default_rng(seed)
    eps = (rng.uniform(0, 4, (S, S)) * (rng.random((S, S)) < 0.15)).astype(np.float32)
    sig = (rng.uniform(0, 3, (S, S)) * (rng.random((S, S)) < 0.6)).astype(np.float32)
    return eps, sig


ENV = [float(np.float32(0.3 + 0.2 * np.sin(2 * np.pi * k / 24))) for k in range(24)]


@pytest.mark.parametrize("S", [8, 32, 128])
def test_forward_option_combinations(ctx, S):
    eps, sig = _scene(S, 500 + S)
    N = S.bit_length() - 1
    refs = {}
    for env in (False, True):
        base = oracle.fluence(eps, sig, environment=ENV if env else None)
        refs[(env, False)] = base
        refs[(env, True)] = oracle_blur.cross_blur(base, sig)
    for group, blur, half, env in itertools.product(GROUPS, (0, BLUR), (0, HALF), (False, True)):
        flags = group | blur | half
        log(f"S={S} flags={flags:#x} env={env}")
        ctx.set_environment(ENV if env else None)
        F = ctx.hrc_forward(to_dev(eps), to_dev(sig), flags=flags)
        torch.cuda.synchronize()
        got = F.cpu().numpy()
        want = refs[(env, bool(blur))]
        what = f"S={S} flags={flags:#x} env={env}"
        if half:
            assert_half_close(got, want, N, what)
        else:
            assert_forward_close(got, want, what)
    ctx.set_environment(None)


@pytest.mark.parametrize("S", [8, 32])
def test_backward_option_combinations(ctx, S):
    """The reverse with the blur's transpose and with environment light, alone
    and together, against the oracle's reverse pass."""
    from gpu_common import assert_grad_close
    from oracle import hrc_vjp
    eps, sig = _scene(S, 700 + S)
    dF = np.random.default_rng(S).normal(size=(S, S)).astype(np.float32)
    for blur, env in itertools.product((0, BLUR), (False, True)):
        what = f"S={S} blur={bool(blur)} env={env}"
        log(f"backward {what}")
        ctx.set_environment(ENV if env else None)
        ge, gs = ctx.hrc_backward(to_dev(eps), to_dev(sig), to_dev(dF), flags=blur)
        torch.cuda.synchronize()
        dG = oracle_blur.cross_blur_vjp(dF, sig) if blur else dF
        re, rs = hrc_vjp.fluence_vjp(eps, sig, dG, environment=np.asarray(ENV) if env else None)
        assert_grad_close(ge.cpu().numpy(), re, f"d eps {what}")
        assert_grad_close(gs.cpu().numpy(), rs, f"d sigma {what}")
    ctx.set_environment(None)
