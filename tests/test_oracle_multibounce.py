"""Pins of the multi-bounce oracle (fluence fed back as an in-scattering
source, Section 4.2)."""
import math

import numpy as np
import pytest

from oracle import hrc
from oracle import multibounce


def _scene(S, seed):
    rng = np.random.default_rng(seed)
    eps = rng.random((S, S)) * (rng.random((S, S)) < 0.2)
    sig = rng.random((S, S)) * 2
    alb = rng.random((S, S))
    return eps, sig, alb


def test_one_bounce_is_algorithm_1():
    eps, sig, alb = _scene(16, 1)
    assert np.array_equal(multibounce.fluence(eps, sig, alb, 1), hrc.fluence(eps, sig))


def test_zero_albedo_adds_nothing():
    eps, sig, _ = _scene(16, 2)
    assert np.array_equal(multibounce.fluence(eps, sig, np.zeros((16, 16)), 4),
                          hrc.fluence(eps, sig))


def test_thick_uniform_medium_geometric_series():
    """Deep inside an optically thick uniform medium each bounce gives
    F = 2 pi eps / sigma_t, so K bounces give (2 pi eps_0 / sigma_t) sum a^j."""
    S = 32
    eps0, sig, a = 0.7, 3.0, 0.6
    E = np.full((S, S), eps0)
    Sg = np.full((S, S), sig)
    A = np.full((S, S), a)
    for K in (1, 2, 4):
        F = multibounce.fluence(E, Sg, A, K)
        want = 2 * math.pi * eps0 / sig * sum(a ** j for j in range(K))
        assert F[14:18, 14:18] == pytest.approx(np.full((4, 4), want), rel=1e-9)


def test_scattering_only_lights_the_medium():
    """A light in vacuum with a scattering slab: the second bounce brightens the
    pixels near the slab and leaves a pixel in vacuum behind an opaque wall
    unaffected by the wall's albedo when the wall does not scatter."""
    S = 16
    eps = np.zeros((S, S)); eps[8, 2] = 5.0
    sig = np.zeros((S, S)); sig[4:12, 10:12] = 1.0
    alb = np.zeros((S, S)); alb[4:12, 10:12] = 0.9
    F1 = multibounce.fluence(eps, sig, alb, 1)
    F2 = multibounce.fluence(eps, sig, alb, 2)
    assert (F2 >= F1 - 1e-12).all()
    assert F2[8, 9] > F1[8, 9] * 1.001


def test_reverse_pass_central_differences():
    rng = np.random.default_rng(3)
    S = 8
    eps, sig, alb = _scene(S, 4)
    dF = rng.normal(size=(S, S))
    K = 3
    de, ds, da = multibounce.fluence_vjp(eps, sig, alb, K, dF)
    h = 1e-6
    for (r, c) in ((0, 0), (2, 5), (6, 3), (7, 7)):
        for grad, which in ((de, 0), (ds, 1), (da, 2)):
            p = [eps.copy(), sig.copy(), alb.copy()]
            m = [eps.copy(), sig.copy(), alb.copy()]
            p[which][r, c] += h
            m[which][r, c] -= h
            fp = (multibounce.fluence(*p, K) * dF).sum()
            fm = (multibounce.fluence(*m, K) * dF).sum()
            assert grad[r, c] == pytest.approx((fp - fm) / (2 * h), rel=1e-6, abs=1e-8)
