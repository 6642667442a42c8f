"""Pins of the oracle's environment lighting (light from beyond the grid, the
footnote to Section 4.2: R_N looked up from the environment map in the cone's
direction, and so every angular fluence looked up outside the grid)."""
import math

import numpy as np
import pytest

from oracle import bruteforce
from oracle import hrc
from oracle import hrc_vjp


def test_uniform_environment_in_vacuum_is_2_pi_E():
    """Closed form: a uniform environment E seen through vacuum gives F = 2 pi E
    at every pixel, borders included (the cone angles of each level add up to
    the quadrant's pi/2)."""
    S = 16
    z = np.zeros((S, S))
    F = hrc.fluence(z, z, environment=[1.5])
    assert np.allclose(F, 2 * math.pi * 1.5, rtol=1e-13, atol=0)
    B = bruteforce.fluence(z, z, M=512, crop=(0, 3, 0, 3), environment=[1.5])
    assert np.allclose(B, 2 * math.pi * 1.5, rtol=1e-12)


def test_zero_environment_is_no_environment():
    rng = np.random.default_rng(1)
    S = 16
    eps = rng.random((S, S)) * (rng.random((S, S)) < 0.2)
    sig = rng.random((S, S))
    assert np.array_equal(hrc.fluence(eps, sig, environment=[0.0, 0.0, 0.0]),
                          hrc.fluence(eps, sig))


def test_linear_in_emission_and_environment():
    """For fixed attenuation F is linear in (emission, environment) jointly."""
    rng = np.random.default_rng(2)
    S = 16
    eps = rng.random((S, S)) * (rng.random((S, S)) < 0.2)
    sig = rng.random((S, S)) * 2
    env = rng.random(12)
    a = hrc.fluence(eps, sig, environment=env)
    b = hrc.fluence(eps, sig) + hrc.fluence(np.zeros((S, S)), sig, environment=env)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)


def test_direction_mapping_of_the_quadrants():
    """Four samples at angles 0, pi/2, pi, 3 pi/2 (nearest sample): only the cones
    around that direction see it, so in vacuum F = pi/2 E from one quadrant; a
    full-height opaque wall on that side blocks it, one on the other side does
    not."""
    S = 16
    z = np.zeros((S, S))
    for k, name in enumerate(("+x (increasing column)", "+y (increasing row)",
                              "-x", "-y")):
        env = np.zeros(4)
        env[k] = 2.0
        F = hrc.fluence(z, z, environment=env)
        assert np.allclose(F, math.pi / 2 * 2.0, rtol=1e-13), name
    env = np.array([2.0, 0.0, 0.0, 0.0])  # light from +x (large column)
    wall = np.zeros((S, S))
    wall[:, 12] = 60.0
    F = hrc.fluence(z, wall, environment=env)
    # right behind the wall every +x ray meets it inside the grid: dark (further
    # back, rays leave through the top and bottom edges first and see the
    # environment around the wall, which lies only inside the grid)
    assert np.abs(F[1:-1, 11]).max() < 1e-12
    assert np.allclose(F[:, 13:], math.pi, rtol=1e-13)  # in front: lit
    wall2 = np.zeros((S, S))
    wall2[:, 3] = 60.0                              # a wall on the far (-x) side
    F2 = hrc.fluence(z, wall2, environment=env)
    assert np.allclose(F2[:, 4:], math.pi, rtol=1e-13)


def test_opaque_enclosure_is_dark():
    S = 16
    sig = np.zeros((S, S))
    sig[4:12, 4] = sig[4:12, 11] = 60.0
    sig[4, 4:12] = sig[11, 4:12] = 60.0
    F = hrc.fluence(np.zeros((S, S)), sig, environment=[3.0])
    assert np.abs(F[5:11, 5:11]).max() < 1e-12
    assert F[0, 0] > 1.0


def test_environment_against_bruteforce_with_occluder():
    """A smooth environment (brighter towards +y) over fog with an opaque block:
    HRC against the brute-force march at the method's error level."""
    S = 32
    K = 64
    th = 2 * math.pi * np.arange(K) / K
    env = 1.0 + 0.8 * np.sin(th)
    sig = np.full((S, S), 0.02)
    sig[12:18, 10:22] = 50.0
    z = np.zeros((S, S))
    F = hrc.fluence(z, sig, environment=env)
    B = bruteforce.fluence(z, sig, M=4096, environment=env)
    mask = sig < 1
    err = np.abs(F - B)[mask] / B[mask]
    assert err.mean() < 0.025, err.mean()                               # measured 0.0207
    assert np.sqrt(np.mean((F - B)[mask] ** 2)) / B.max() < 0.022       # measured 0.0187


def test_environment_gradient_central_differences():
    """The reverse pass with an environment (a constant): FP64 central
    differences of the oracle's forward at a few entries."""
    rng = np.random.default_rng(3)
    S = 8
    eps = rng.random((S, S)) * 0.5
    sig = rng.random((S, S)) * 1.5
    env = rng.random(8) + 0.5
    dF = rng.normal(size=(S, S))
    dE, dS = hrc_vjp.fluence_vjp(eps, sig, dF, environment=env)
    h = 1e-6
    for (r, c) in ((0, 0), (3, 5), (7, 2), (4, 4)):
        for grad, field in ((dE, "eps"), (dS, "sig")):
            a = {"eps": eps.copy(), "sig": sig.copy()}
            b = {"eps": eps.copy(), "sig": sig.copy()}
            a[field][r, c] += h
            b[field][r, c] -= h
            fa = (hrc.fluence(a["eps"], a["sig"], environment=env) * dF).sum()
            fb = (hrc.fluence(b["eps"], b["sig"], environment=env) * dF).sum()
            assert grad[r, c] == pytest.approx((fa - fb) / (2 * h), rel=1e-6, abs=1e-8)


def test_halfway_directions_take_the_next_sample_counter_clockwise():
    """The tie-break of reading R15, fixed by hand: a direction exactly halfway
    between two samples of the map takes the next sample counter-clockwise
    (towards increasing angle).  Two samples [E0 at 0, E1 at pi]: the +y axis
    (pi/2) lies halfway and takes E1, the -y axis (-pi/2, i.e. 3 pi/2) takes E0
    (round half to even would give E0 and E0).  Four samples at 0, pi/2, pi,
    3 pi/2: pi/4 -> the one at pi/2, 3 pi/4 -> pi, -3 pi/4 -> 3 pi/2,
    -pi/4 -> 0."""
    two = [10.0, 20.0]
    assert hrc.environment_radiance(two, math.pi / 2) == 20.0
    assert hrc.environment_radiance(two, -math.pi / 2) == 10.0
    four = [1.0, 2.0, 3.0, 4.0]
    assert hrc.environment_radiance(four, math.pi / 4) == 2.0
    assert hrc.environment_radiance(four, 3 * math.pi / 4) == 3.0
    assert hrc.environment_radiance(four, -3 * math.pi / 4) == 4.0
    assert hrc.environment_radiance(four, -math.pi / 4) == 1.0
    # away from a tie the nearest sample wins on either side
    assert hrc.environment_radiance(two, math.pi / 2 - 1e-9) == 10.0
    assert hrc.environment_radiance(two, math.pi / 2 + 1e-9) == 20.0


def test_halfway_cone_reaches_the_gather_beyond_the_last_column():
    """The level-0 cone of the +y quadrant is centred on the +y axis, halfway
    between the two samples of [E0, E1]: its environment fluence is
    A_0(0) E1 = (pi/2) E1 (Eq. 13: A_0(0) = atan(1) - atan(-1)), and the -y
    quadrant's is (pi/2) E0.  The gather reads that fluence beyond the grid, so
    in the last frame column of the +y solve (the image's bottom row) the
    quadrant contributes exactly (pi/2) E1."""
    E0, E1 = 1.0, 3.0
    N = 3
    S = 1 << N
    env_py = hrc.environment_fluence([E0, E1], "+y", N)
    env_my = hrc.environment_fluence([E0, E1], "-y", N)
    assert env_py[0][0] == pytest.approx(math.pi / 2 * E1, rel=1e-15)
    assert env_my[0][0] == pytest.approx(math.pi / 2 * E0, rel=1e-15)
    z = np.zeros((S, S))
    Q = hrc.quadrant(z, z, env=env_py)
    assert np.allclose(Q[S - 1, :], math.pi / 2 * E1, rtol=1e-14, atol=0)
