"""The batched launch (persistent kernel with one queue per XCD, plus the
larger scenes as kernels of their own where the autotuner picks that): bitwise
equal to single-scene calls, replayed several times, with mixed sizes and
forward-only scenes; the whole 64-scene batch workload against the single-scene
calls and, for its scenes up to 256^2 and two of 512^2, against the oracle; and
the failure path of the dependency waits, forced from the host."""
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest
import torch

from oracle import hrc as oracle
from oracle import hrc_vjp
from scenes import config5, scene_like_512

pytestmark = pytest.mark.gpu

from gpu_common import assert_forward_close, assert_grad_close, log, to_dev  # noqa: E402


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
    want = {0x100: 0, 0x200: 1}.get(flags)  # parity of the variant: register budget
    if want is not None:
        assert b.describe()["variant"] % 2 == want
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
        b.status()
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
    b.status()
    _check_against_single(ctx, items)
    ctx.release_workspaces()
    del b


def _oracle_one(args):
    eps, sig, dF = args
    F = oracle.fluence(eps, sig)
    ge, gs = hrc_vjp.fluence_vjp(eps, sig, dF)
    return F, ge, gs


@pytest.mark.parametrize("flags", [0, 0x400], ids=["autotuned", "persistent-only"])
def test_batch_workload_64_scenes(ctx, flags):
    """The 64-scene batch workload (sizes drawn from 128^2..1024^2, forward and
    backward for every scene): every scene bitwise equal to its single-scene
    calls, the scheduler's status clean after two launches, and the batch's
    own outputs for the scenes up to 256^2 and two of the 512^2 scenes against
    the oracle's forward and reverse passes."""
    from paper_2505_02041_amd import Batch
    log(f"batch: the 64-scene workload, flags {flags:#x}")
    scenes = config5()
    assert len(scenes) == 64
    items = _make(scenes, lambda i: True)
    b = Batch(items, ctx, flags=flags)
    d = b.describe()
    log(f"  autotuned: {d}")
    if flags & 0x400:
        assert d["direct_scenes"] == 0
    for _ in range(2):
        b.launch()
    b.status()
    small = [i for i, sc in enumerate(scenes) if sc.eps.shape[0] <= 256]
    small += [i for i, sc in enumerate(scenes) if sc.eps.shape[0] == 512][:2]
    got = {i: (items[i]["fluence"].cpu().numpy(), items[i]["grad_emission"].cpu().numpy(),
               items[i]["grad_sigma_t"].cpu().numpy()) for i in small}
    _check_against_single(ctx, items)
    ctx.release_workspaces()
    del b
    log(f"  oracle on {len(small)} scenes")
    jobs = [(scenes[i].eps, scenes[i].sigma, items[i]["grad_fluence"].cpu().numpy())
            for i in small]
    workers = max(1, min(16, os.cpu_count() or 1))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        refs = list(ex.map(_oracle_one, jobs))
    for i, (F, ge, gs) in zip(small, refs):
        S = scenes[i].eps.shape[0]
        assert_forward_close(got[i][0], F, f"batch scene {i} ({S}^2) fluence")
        assert_grad_close(got[i][1], ge, f"batch scene {i} ({S}^2) d eps")
        assert_grad_close(got[i][2], gs, f"batch scene {i} ({S}^2) d sigma")


def test_batch_wait_failure_is_reported(ctx):
    """A dependency wait that gives up is reported by hrc_batch_status, forced
    from the host: every wait asks for one group more than its step holds and
    gives up after a few polls, so every kernel still runs to its end.  With
    normal waits restored the next launch is clean and bitwise correct."""
    from paper_2505_02041_amd import Batch
    from paper_2505_02041_amd._lib import HRC_ERR_TIMEOUT, HRCError
    log("batch: forced wait failure")
    scenes = [scene_like_512(S, 90 + i, 3, 4) for i, S in enumerate([32, 64, 128, 64])]
    items = _make(scenes, lambda i: i != 1)
    b = Batch(items, ctx, flags=0x400)
    b.status()
    b.debug_waits(16)
    b.launch()
    with pytest.raises(HRCError) as e:
        b.status()
    assert e.value.status == HRC_ERR_TIMEOUT
    b.status()  # the report was cleared
    b.debug_waits(0)
    for d in items:
        d["fluence"].fill_(float("nan"))
    b.launch()
    b.status()
    _check_against_single(ctx, items)
    del b
