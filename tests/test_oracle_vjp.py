"""Pins of the oracle's reverse pass: FP64 central differences of the forward
pass, and the sign structure of the derivatives."""
import numpy as np
import pytest

from oracle import hrc, hrc_vjp
from scenes import config1


def _scene(S, seed):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(0, 3, (S, S)) * (rng.random((S, S)) < 0.3)
    sig = rng.uniform(0, 1.5, (S, S))
    return eps, sig


@pytest.mark.parametrize("S,seed_levels", [(16, 3), (32, 3), (16, 5)])
def test_vjp_matches_central_differences(S, seed_levels):
    """Loss = mean((F - F_t)^2); compare dLoss/d eps and dLoss/d sigma of the
    reverse pass with FP64 central differences at 16 seeded pixels each."""
    eps, sig = _scene(S, 11)
    rng = np.random.default_rng(12)
    Ft = hrc.fluence(*_scene(S, 13), seed_levels=seed_levels)

    def loss(e, s):
        F = hrc.fluence(e, s, seed_levels=seed_levels)
        return np.mean((F - Ft) ** 2)

    F = hrc.fluence(eps, sig, seed_levels=seed_levels)
    dF = 2 * (F - Ft) / F.size
    dE, dS = hrc_vjp.fluence_vjp(eps, sig, dF, seed_levels=seed_levels)
    pix = rng.integers(0, S, (16, 2))
    for r, c in pix:
        for field, grad in ((0, dE), (1, dS)):
            x = [eps.copy(), sig.copy()]
            h = 1e-5 * max(1.0, abs(x[field][r, c]))
            x[field][r, c] += h
            lp = loss(*x)
            x[field][r, c] -= 2 * h
            lm = loss(*x)
            fd = (lp - lm) / (2 * h)
            assert grad[r, c] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(grad).max())


def test_vjp_is_transpose_of_forward_in_emission():
    """F is linear in eps at fixed sigma, so <dF, F(e)> = <J^T dF, e> exactly."""
    eps, sig = _scene(32, 21)
    rng = np.random.default_rng(22)
    dF = rng.normal(size=eps.shape)
    dE, _ = hrc_vjp.fluence_vjp(eps, sig, dF)
    lhs = np.sum(dF * hrc.fluence(eps, sig))
    rhs = np.sum(dE * eps)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_vjp_signs_monotonicity():
    """Every term of F is a non-negative product, increasing in emission and
    decreasing in attenuation: with dF >= 0, d eps >= 0 and d sigma <= 0."""
    sc = config1()
    dF = np.random.default_rng(3).random((64, 64))
    dE, dS = hrc_vjp.fluence_vjp(sc.eps, sc.sigma, dF)
    assert np.all(dE >= 0)
    assert np.all(dS <= 1e-15)
    assert dE.max() > 0 and dS.min() < 0


def test_cell_gradient_small_tau_branch():
    """The series branch of phi' agrees with central differences near tau = 0."""
    for sig in (0.0, 1e-6, 3e-3, 2e-2):
        for ell in (0.5, 1.0, np.sqrt(2)):
            de, dsL, dsT = hrc_vjp.cell_interval_grad(2.0, sig, ell)
            h = 1e-7
            Lp, Tp = hrc.cell_interval(2.0, sig + h, ell)
            Lm, Tm = hrc.cell_interval(2.0, max(sig - h, 0.0), ell)
            hh = (sig + h) - max(sig - h, 0.0)
            assert float(dsL) == pytest.approx(float(Lp - Lm) / hh, rel=1e-5)
            assert float(dsT) == pytest.approx(float(Tp - Tm) / hh, rel=1e-5)
            assert float(de) == pytest.approx(float(hrc.cell_interval(1.0, sig, ell)[0]), rel=1e-15)
