"""hrc_profile_solve: the timed solve runs the passes of Algorithm 1 (and its
reverse) in order, every pass has a positive kernel duration, and its results
are bitwise those of hrc_forward / hrc_backward."""
import numpy as np
import pytest
import torch

from scenes import scene_like_512

pytestmark = pytest.mark.gpu

from gpu_common import log, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_02041_amd import Context
    return Context(0)


def _forward_order(N):
    return ([("seed", -1)] + [("merge_up", n) for n in range(3, N)] +
            [("merge_down", n) for n in range(N - 1, 1, -1)] + [("tail", -1)])


@pytest.mark.parametrize("S", [8, 128, 512])
def test_profile_forward(ctx, S):
    log(f"profile forward S={S}")
    N = S.bit_length() - 1
    sc = scene_like_512(S, 41, 4, 6)
    e, s = to_dev(sc.eps), to_dev(sc.sigma)
    passes, F = ctx.hrc_profile_solve(e, s, return_outputs=True)
    assert [(p, n) for p, n, _ in passes] == _forward_order(N)
    assert all(ms > 0 for _, _, ms in passes)
    assert torch.equal(F, ctx.hrc_forward(e, s))


@pytest.mark.parametrize("S", [8, 256])
def test_profile_backward(ctx, S):
    log(f"profile backward S={S}")
    N = S.bit_length() - 1
    sc = scene_like_512(S, 43, 4, 6)
    e, s = to_dev(sc.eps), to_dev(sc.sigma)
    g = to_dev(np.random.default_rng(5).normal(size=(S, S)))
    passes, (ge, gs) = ctx.hrc_profile_solve(e, s, g, return_outputs=True)
    names = [p for p, _, _ in passes]
    # the recomputed forward (down to R_1, no gather), then the reverse
    fwd = _forward_order(N)[:-1] + [("merge_down", 1)]
    assert [(p, n) for p, n, _ in passes[:len(fwd)]] == fwd
    rev = names[len(fwd):]
    assert rev[0] == "gather_adj" and rev[-1] == "seed_adj"
    assert rev.count("merge_down_adj") == N - 1 and rev.count("interval_adj") == N + 1
    assert all(ms > 0 for _, _, ms in passes)
    ge2, gs2 = ctx.hrc_backward(e, s, g)
    assert torch.equal(ge, ge2) and torch.equal(gs, gs2)
