"""The batched launch (persistent kernel, plus the larger scenes as kernels of
their own where the autotuner picks that): bitwise equal to single-scene calls,
replayed several times, with mixed sizes and forward-only scenes."""
import numpy as np
import pytest
import torch

from scenes import config5, scene_like_512

pytestmark = pytest.mark.gpu

from gpu_common import log, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_02041_amd import Context
    return Context(0)


def _make(scenes, with_grad):
    out = []
    for i, sc in enumerate(scenes):
        S = sc.eps.shape[0]
        d = {"emission": to_dev(sc.eps), "sigma_t": to_dev(sc.sigma),
             "fluence": torch.full((S, S), float("nan"), device="cuda")}
        if with_grad(i):
            rng = np.random.default_rng(900 + i)
            d["grad_fluence"] = to_dev(rng.normal(size=(S, S)))
            d["grad_emission"] = torch.full((S, S), float("nan"), device="cuda")
            d["grad_sigma_t"] = torch.full((S, S), float("nan"), device="cuda")
        out.append(d)
    return out


def _check_against_single(ctx, items):
    for i, d in enumerate(items):
        F = ctx.hrc_forward(d["emission"], d["sigma_t"])
        assert torch.equal(F, d["fluence"]), f"scene {i} fluence"
        if "grad_fluence" in d:
            ge, gs = ctx.hrc_backward(d["emission"], d["sigma_t"], d["grad_fluence"])
            assert torch.equal(ge, d["grad_emission"]), f"scene {i} d eps"
            assert torch.equal(gs, d["grad_sigma_t"]), f"scene {i} d sigma"


@pytest.mark.parametrize("flags", [0, 0x100, 0x200, 0x400],
                         ids=["autotuned", "full", "dense", "persistent-only"])
def test_batch_small_mixed_sizes(ctx, flags):
    from paper_2505_02041_amd import Batch
    log(f"batch small mixed, flags {flags:#x}")
    scenes = [scene_like_512(S, 70 + i, 3, 4) for i, S in enumerate([8, 64, 32, 128, 16, 256])]
    items = _make(scenes, lambda i: i % 2 == 0)
    b = Batch(items, ctx, flags=flags)
    want = {0x100: 0, 0x200: 1}.get(flags)
    if want is not None:
        assert b.describe()["variant"] == want
    if flags & 0x400:
        assert b.describe()["direct_scenes"] == 0
    log(f"  autotuned: {b.describe()}")
    for rep in range(3):
        for d in items:
            d["fluence"].fill_(float("nan"))
            if "grad_fluence" in d:
                d["grad_emission"].fill_(float("nan"))
                d["grad_sigma_t"].fill_(float("nan"))
        b.launch()
        torch.cuda.synchronize()
        _check_against_single(ctx, items)
    del b


@pytest.mark.parametrize("flags", [0, 0x500, 0x600],
                         ids=["autotuned", "full-persistent", "dense-persistent"])
def test_batch_benchmark_workload_subset(ctx, flags):
    """16 scenes of the 64-scene batch workload (sizes 128..1024), fwd + bwd."""
    from paper_2505_02041_amd import Batch
    log(f"batch 16 scenes of the batch workload, flags {flags:#x}")
    scenes = config5()[:16]
    items = _make(scenes, lambda i: True)
    b = Batch(items, ctx, flags=flags)
    log(f"  autotuned: {b.describe()}")
    if flags & 0x400:
        assert b.describe()["direct_scenes"] == 0
    b.launch()
    torch.cuda.synchronize()
    _check_against_single(ctx, items)
    ctx.release_workspaces()
    del b
