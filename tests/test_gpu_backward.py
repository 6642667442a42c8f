"""GPU parity of the reverse pass (hrc_backward through the C ABI): against the
oracle's reverse pass element by element, against FP64 central differences of
the oracle's forward pass, and through torch.autograd."""
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest
import torch

from oracle import hrc as oracle
from oracle import hrc_vjp
from scenes import config1, config3, config4, scene_like_512

pytestmark = pytest.mark.gpu

from gpu_common import assert_grad_close, log, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    from paper_2505_02041_amd import Context
    return Context(0)


def _random_scene(S, seed):
    rng = np.random.default_rng(seed)
    eps = (rng.uniform(0, 3, (S, S)) * (rng.random((S, S)) < 0.3)).astype(np.float32)
    sig = rng.uniform(0, 1.5, (S, S)).astype(np.float32)
    dF = rng.normal(size=(S, S)).astype(np.float32)
    return eps, sig, dF


def _bwd(ctx, eps, sig, dF):
    ge, gs = ctx.hrc_backward(to_dev(eps), to_dev(sig), to_dev(dF))
    torch.cuda.synchronize()
    return ge.cpu().numpy(), gs.cpu().numpy()


@pytest.mark.parametrize("S", [8, 16, 32, 64, 128])
def test_backward_matches_oracle_reverse(ctx, S):
    log(f"backward random S={S}")
    eps, sig, dF = _random_scene(S, 200 + S)
    ge, gs = _bwd(ctx, eps, sig, dF)
    re, rs = hrc_vjp.fluence_vjp(eps, sig, dF)
    assert_grad_close(ge, re, f"d eps S={S}")
    assert_grad_close(gs, rs, f"d sigma S={S}")


def test_backward_benchmark_scene_matches_oracle_reverse(ctx):
    """The 1024x1024 benchmark scene (opaque boxes, sigma-100 lines, fog, 128
    disks), seeded normal dLoss/dF: d eps and d sigma from the HIP adjoint
    element by element against the oracle's FP64 reverse pass, the transposes
    of Eq. 7-8 and Eq. 14-20 at every level up to N = 10."""
    log("backward 1024x1024 benchmark scene vs oracle reverse")
    sc = config3()
    dF = np.random.default_rng(1024).normal(size=(1024, 1024)).astype(np.float32)
    ge, gs = _bwd(ctx, sc.eps, sc.sigma, dF)
    log("  oracle reverse (about 20 s on one host core)")
    re, rs = hrc_vjp.fluence_vjp(sc.eps, sc.sigma, dF)
    assert_grad_close(ge, re, "d eps 1024")
    assert_grad_close(gs, rs, "d sigma 1024")
    ctx.release_workspaces()


def test_backward_2048_matches_oracle_reverse(ctx):
    """2048x2048 (N = 11) with the benchmark scene's recipe scaled with the
    area, through the reuse pair (kept forward, reused reverse): d eps and
    d sigma element by element against the oracle's reverse (about a minute
    on one host core)."""
    from paper_2505_02041_amd import _lib
    log("backward 2048x2048 vs oracle reverse")
    S = 2048
    sc = scene_like_512(S, 32, 512, 1024, 128)
    dF = np.random.default_rng(7).normal(size=(S, S)).astype(np.float32)
    e, s, g = to_dev(sc.eps), to_dev(sc.sigma), to_dev(dF)
    res = ctx.reserve(11)
    ctx.hrc_forward(e, s, flags=_lib.HRC_FLAG_KEEP_PYRAMID, reserve=res)
    ge, gs = ctx.hrc_backward(e, s, g, flags=_lib.HRC_FLAG_REUSE_PYRAMID, reserve=res)
    torch.cuda.synchronize()
    ge, gs = ge.cpu().numpy(), gs.cpu().numpy()
    del res, e, s, g
    ctx.release_workspaces()
    re, rs = hrc_vjp.fluence_vjp(sc.eps, sc.sigma, dF)
    assert_grad_close(ge, re, "d eps 2048")
    assert_grad_close(gs, rs, "d sigma 2048")


def test_backward_config1(ctx):
    sc = config1()
    dF = np.random.default_rng(1).random((64, 64)).astype(np.float32)
    ge, gs = _bwd(ctx, sc.eps, sc.sigma, dF)
    re, rs = hrc_vjp.fluence_vjp(sc.eps, sc.sigma, dF)
    assert_grad_close(ge, re, "d eps 64")
    assert_grad_close(gs, rs, "d sigma 64")


def _mse_target():
    hidden = config4()
    return oracle.fluence(hidden.eps, hidden.sigma)


def _start_scene():
    S = 256
    rng = np.random.default_rng(44)
    eps = rng.uniform(0.05, 2.0, (S, S)).astype(np.float32) * (rng.random((S, S)) < 0.1)
    sig = rng.uniform(0.0, 1.0, (S, S)).astype(np.float32)
    return eps, sig


def test_backward_config4_matches_oracle_reverse(ctx):
    """256x256 differentiable workload: Loss = mean((F - F_target)^2)."""
    log("backward 256x256 vs oracle reverse")
    Ft = _mse_target()
    eps, sig = _start_scene()
    F = oracle.fluence(eps, sig)
    dF = (2 * (F - Ft) / F.size).astype(np.float32)
    ge, gs = _bwd(ctx, eps, sig, dF)
    re, rs = hrc_vjp.fluence_vjp(eps, sig, dF)
    assert_grad_close(ge, re, "d eps 256")
    assert_grad_close(gs, rs, "d sigma 256")


_FD = {}


def _fd_one(args):
    field, r, c = args
    eps, sig, Ft = _FD["eps"], _FD["sig"], _FD["Ft"]
    x = [eps.astype(np.float64).copy(), sig.astype(np.float64).copy()]
    h = 1e-4 * max(1.0, abs(x[field][r, c]))
    x[field][r, c] += h
    lp = np.mean((oracle.fluence(*x) - Ft) ** 2)
    x[field][r, c] -= 2 * h
    lm = np.mean((oracle.fluence(*x) - Ft) ** 2)
    return (lp - lm) / (2 * h)


def test_backward_config4_central_differences(ctx):
    """dLoss/d eps and dLoss/d sigma from the HIP adjoint against FP64 central
    differences of the oracle's forward pass at 64 seeded pixels (seed 40)."""
    log("backward 256x256 vs central differences")
    Ft = _mse_target()
    eps, sig = _start_scene()
    e_t, s_t = to_dev(eps).requires_grad_(), to_dev(sig).requires_grad_()
    from paper_2505_02041_amd import fluence
    F = fluence(e_t, s_t)
    loss = torch.mean((F.double() - torch.from_numpy(Ft).cuda()) ** 2)
    loss.backward()
    ge, gs = e_t.grad.cpu().numpy(), s_t.grad.cpu().numpy()
    pix = np.random.default_rng(40).integers(0, 256, (64, 2))
    _FD.update(eps=eps, sig=sig, Ft=Ft)
    jobs = [(f, int(r), int(c)) for r, c in pix for f in (0, 1)]
    workers = max(1, min(16, os.cpu_count() or 1))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        fds = list(ex.map(_fd_one, jobs))
    gmax_e, gmax_s = np.abs(ge).max(), np.abs(gs).max()
    for (f, r, c), fd in zip(jobs, fds):
        g = ge[r, c] if f == 0 else gs[r, c]
        scale = gmax_e if f == 0 else gmax_s
        assert abs(g - fd) <= 1e-3 * abs(fd) + 1e-4 * scale, (f, r, c, g, fd)


def test_autograd_function_matches_direct_calls(ctx):
    from paper_2505_02041_amd import fluence
    eps, sig, dF = _random_scene(64, 7)
    e_t, s_t = to_dev(eps).requires_grad_(), to_dev(sig).requires_grad_()
    F = fluence(e_t, s_t)
    F.backward(to_dev(dF))
    F2 = ctx.hrc_forward(to_dev(eps), to_dev(sig))
    ge, gs = ctx.hrc_backward(to_dev(eps), to_dev(sig), to_dev(dF))
    assert torch.equal(F.detach(), F2)
    assert torch.equal(e_t.grad, ge) and torch.equal(s_t.grad, gs)


@pytest.mark.parametrize("S,flags,env", [(8, 0, False), (64, 0x2, False), (64, 0x4, False),
                                          (256, 0x6, False), (128, 0, True), (1024, 0, False)],
                         ids=["8", "64-blur", "64-half", "256-blur-half", "128-env", "1024"])
def test_kept_forward_and_reused_backward_equal_the_plain_calls(ctx, S, flags, env):
    """HRC_FLAG_KEEP_PYRAMID / HRC_FLAG_REUSE_PYRAMID: the kept forward's
    fluence and the reused reverse's gradients are bitwise those of the plain
    calls; a second reverse on the same reserve (another dLoss/dF) too, since a
    reverse leaves the kept levels intact."""
    from paper_2505_02041_amd import _lib
    log(f"keep/reuse S={S} flags {flags:#x} env {env}")
    if S == 1024:
        sc = config3()
        eps, sig = sc.eps, sc.sigma
        dF = np.random.default_rng(5).normal(size=(S, S)).astype(np.float32)
    else:
        eps, sig, dF = _random_scene(S, 40 + S)
    dF2 = np.random.default_rng(S + 1).normal(size=(S, S)).astype(np.float32)
    if env:
        ctx.set_environment([0.5 + 0.25 * k for k in range(12)])
    try:
        e, s, g, g2 = to_dev(eps), to_dev(sig), to_dev(dF), to_dev(dF2)
        res = ctx.reserve(int(np.log2(S)), flags)
        Fk = ctx.hrc_forward(e, s, flags=flags | _lib.HRC_FLAG_KEEP_PYRAMID, reserve=res)
        gk = ctx.hrc_backward(e, s, g, flags=flags | _lib.HRC_FLAG_REUSE_PYRAMID, reserve=res)
        gk2 = ctx.hrc_backward(e, s, g2, flags=flags | _lib.HRC_FLAG_REUSE_PYRAMID, reserve=res)
        F = ctx.hrc_forward(e, s, flags=flags)
        gp = ctx.hrc_backward(e, s, g, flags=flags)
        gp2 = ctx.hrc_backward(e, s, g2, flags=flags)
        torch.cuda.synchronize()
    finally:
        if env:
            ctx.set_environment(None)
    assert torch.equal(Fk, F)
    for a, b in zip(gk + gk2, gp + gp2):
        assert torch.equal(a, b)


def test_autograd_without_keep_equals_with_keep(ctx):
    from paper_2505_02041_amd import fluence
    eps, sig, dF = _random_scene(128, 9)
    grads = []
    for keep in (True, False):
        e_t, s_t = to_dev(eps).requires_grad_(), to_dev(sig).requires_grad_()
        F = fluence(e_t, s_t, keep=keep)
        F.backward(to_dev(dF))
        grads.append((F.detach(), e_t.grad, s_t.grad))
    for a, b in zip(*grads):
        assert torch.equal(a, b)


def test_backward_signs(ctx):
    """With dF >= 0 the emission gradient is >= 0 and the attenuation gradient
    is <= 0 (every term of F grows with emission and shrinks with attenuation)."""
    sc = config1()
    dF = np.random.default_rng(3).random((64, 64)).astype(np.float32)
    ge, gs = _bwd(ctx, sc.eps, sc.sigma, dF)
    assert (ge >= 0).all() and (gs <= 0).all()


def test_backward_is_deterministic(ctx):
    eps, sig, dF = _random_scene(128, 8)
    a = _bwd(ctx, eps, sig, dF)
    b = _bwd(ctx, eps, sig, dF)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_adam_recovers_scene(ctx):
    """200 Adam steps (lr 0.3) on softplus-parameterised emission and attenuation
    from a uniform start (0.1, 0.1) reduce the MSE to the hidden scene's fluence
    by more than 250x (measured 3782 -> 5.96, i.e. 635x; the fields themselves
    are not identifiable from the fluence alone)."""
    log("adam 200 steps 256x256")
    from paper_2505_02041_amd import fluence
    hidden = config4()
    with torch.no_grad():
        Ft = fluence(to_dev(hidden.eps), to_dev(hidden.sigma))
    inv = float(np.log(np.expm1(0.1)))
    pe = torch.full((256, 256), inv, device="cuda", requires_grad=True)
    ps = torch.full((256, 256), inv, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([pe, ps], lr=0.3)
    losses = []
    for _ in range(200):
        opt.zero_grad()
        F = fluence(torch.nn.functional.softplus(pe), torch.nn.functional.softplus(ps))
        loss = torch.mean((F - Ft) ** 2)
        loss.backward()
        opt.step()
        losses.append(loss.item())
    log(f"adam loss {losses[0]:.4g} -> {losses[-1]:.4g}")
    assert losses[-1] < 4e-3 * losses[0]


@pytest.mark.parametrize("S", [1024, 4096])
def test_backward_emission_adjoint_identity_at_full_size(ctx, S):
    """At the benchmark size and the largest supported size: F is linear in the
    emission for a fixed attenuation, so the emission gradient is the
    transpose of the forward map itself and <dF, F(e')> = <d eps, e'> for any
    probe e' (a property the oracle cannot reach at these sizes)."""
    log(f"backward adjoint identity S={S}")
    g = torch.Generator(device="cuda").manual_seed(S)
    sig = torch.rand((S, S), device="cuda", generator=g) * 0.3
    sig[S // 4:S // 4 + 16, S // 8:S // 2] = 50.0   # an opaque bar
    eps = torch.rand((S, S), device="cuda", generator=g) * (
        torch.rand((S, S), device="cuda", generator=g) < 0.05)
    probe = torch.rand((S, S), device="cuda", generator=g)
    dF = torch.randn((S, S), device="cuda", generator=g)
    ge, _ = ctx.hrc_backward(eps, sig, dF)
    Fp = ctx.hrc_forward(probe, sig)
    torch.cuda.synchronize()
    lhs = float((dF.double() * Fp.double()).sum())
    rhs = float((ge.double() * probe.double()).sum())
    assert lhs == pytest.approx(rhs, rel=2e-4), (lhs, rhs)
    ctx.release_workspaces()
