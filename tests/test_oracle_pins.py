"""Pins of the FP64 oracle's forward pass against facts the paper and the
mathematics fix (not against the oracle itself)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import bruteforce, hrc
from scenes import config1

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng_scene(S, seed, sig_scale=1.0):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(0, 3, (S, S)) * (rng.random((S, S)) < 0.2)
    sig = rng.uniform(0, 2, (S, S)) * sig_scale
    return eps, sig


# ---------------------------------------------------------------- P1 ------
def test_fig2_worked_example():
    """Section 3, Fig. 2: two blocks of transmittance 0.5 give <2, 0.5> each and
    <3, 0.25> combined (Eq. 5-7)."""
    g = json.load(open(os.path.join(GOLDEN, "fig2_worked_example.json")))
    sig = math.log(2.0)            # exp(-sig * 1) = 0.5 over a unit chord
    eps = g["block"]["eps_over_sigma"] * sig
    near = hrc.cell_interval(eps, sig, 1.0)
    assert float(near[0]) == pytest.approx(g["near_block"]["L"], rel=1e-14)
    assert float(near[1]) == pytest.approx(g["near_block"]["T"], rel=1e-14)
    both = hrc.merge(near, near)
    assert float(both[0]) == pytest.approx(g["both_blocks"]["L"], rel=1e-14)
    assert float(both[1]) == pytest.approx(g["both_blocks"]["T"], rel=1e-14)
    # the same two blocks as a traced segment through two cells of a grid
    E = np.zeros((4, 4)); S_ = np.zeros((4, 4))
    E[1, 1] = E[2, 1] = eps
    S_[1, 1] = S_[2, 1] = sig
    L, T = hrc.trace(E, S_, (1.0, 1.5), (3.0, 1.5))
    assert L == pytest.approx(3.0, rel=1e-14) and T == pytest.approx(0.25, rel=1e-14)


def test_merge_not_commutative_but_associative():
    """Eq. 7 composes near first: it is associative (Eq. 5-6 split anywhere) but
    not commutative."""
    rng = np.random.default_rng(0)
    a, b, c = [(rng.random(), rng.random()) for _ in range(3)]
    left = hrc.merge(hrc.merge(a, b), c)
    right = hrc.merge(a, hrc.merge(b, c))
    assert np.allclose(left, right, rtol=1e-15, atol=0)
    assert not np.allclose(hrc.merge(a, b), hrc.merge(b, a))


def test_cell_integrator_closed_form_and_limits():
    """Eq. 2-4 for a uniform chord: L = eps*(1-exp(-sig*l))/sig, T = exp(-sig*l);
    sig -> 0 gives L = eps*l; integrating the ODE dL/dl = eps - sig*L numerically
    gives the same value."""
    for eps, sig, ell in [(2.0, 0.7, 1.3), (5.0, 1e-9, 2.0), (1.0, 0.0, 0.5), (3.0, 50.0, 1.0)]:
        L, T = hrc.cell_interval(eps, sig, ell)
        if sig > 0:
            assert float(L) == pytest.approx(-eps * math.expm1(-sig * ell) / sig, rel=1e-12)
        else:
            assert float(L) == pytest.approx(eps * ell, rel=1e-15)
        assert float(T) == pytest.approx(math.exp(-sig * ell), rel=1e-15)
        # midpoint-rule quadrature of Eq. 4 directly
        t = (np.arange(200000) + 0.5) * ell / 200000
        Lq = np.sum(np.exp(-sig * t) * eps) * ell / 200000
        assert float(L) == pytest.approx(Lq, rel=1e-8)


# ---------------------------------------------------------------- cones ---
@pytest.mark.parametrize("m", range(0, 9))
def test_cone_angles_partition_quadrant(m):
    """Eq. 13: the cones of a level tile [-pi/4, pi/4]; each is split exactly in
    two by the next level (j = 2i -+ 1/2)."""
    A = np.array([hrc.cone_angle(m, jj) for jj in range(2 ** m)])
    assert A.sum() == pytest.approx(math.pi / 2, rel=1e-14)
    assert np.all(A > 0)
    assert np.allclose(A, A[::-1], rtol=1e-14)          # mirror symmetric
    B = np.array([hrc.cone_angle(m + 1, jj) for jj in range(2 ** (m + 1))])
    assert np.allclose(A, B[0::2] + B[1::2], rtol=1e-13)
    # the widest cone is the central one: angles shrink towards the diagonals
    assert A[(2 ** m) // 2 - 1 if m else 0] == A.max()


# ---------------------------------------------------------------- P6 ------
# Cells crossed by Trace(P, P + v_n(k)) from a probe at a pixel centre, derived
# by hand from the geometry (Section 4.1, traced levels 0..2 of Section 4.2):
# (du, dw, chord length).  k > 2^(n-1) mirrors k' = 2^n - k in w.
r2, r5 = math.sqrt(2), math.sqrt(5)
HAND_STENCILS = {
    (0, 0): [(0, 0, r2 / 2), (1, -1, r2 / 2)],
    (1, 0): [(0, 0, r2 / 2), (1, -1, r2), (2, -2, r2 / 2)],
    (1, 1): [(0, 0, .5), (1, 0, 1.), (2, 0, .5)],
    (2, 0): [(0, 0, r2 / 2), (1, -1, r2), (2, -2, r2), (3, -3, r2), (4, -4, r2 / 2)],
    (2, 1): [(0, 0, r5 / 4), (1, 0, r5 / 4), (1, -1, r5 / 4), (2, -1, r5 / 2),
             (3, -1, r5 / 4), (3, -2, r5 / 4), (4, -2, r5 / 4)],
    (2, 2): [(0, 0, .5), (1, 0, 1.), (2, 0, 1.), (3, 0, 1.), (4, 0, .5)],
}


@pytest.mark.parametrize("n", [0, 1, 2])
def test_seed_stencils_match_hand_derivation(n):
    a = 2 ** n
    for k in range(a + 1):
        if (n, k) in HAND_STENCILS:
            want = HAND_STENCILS[(n, k)]
        else:
            want = [(du, -dw, l) for du, dw, l in HAND_STENCILS[(n, a - k)]]
        got = hrc.probe_offsets(n, k)
        assert [(u, w) for u, w, _ in got] == [(u, w) for u, w, _ in want]
        assert np.allclose([l for *_, l in got], [l for *_, l in want], rtol=1e-15)
        assert sum(l for *_, l in got) == pytest.approx(math.hypot(a, 2 * k - a), rel=1e-15)


def test_trace_matches_independent_grid_walk():
    """Eq. 9 by the oracle's rational segment cutting agrees with the C grid
    walk of the brute force (a separate implementation) for rays to the grid
    exit from pixel centres."""
    E, Sg = _rng_scene(16, 3)
    rng = np.random.default_rng(7)
    for _ in range(40):
        r, c = rng.integers(0, 16, 2)
        P = (c + 0.5, r + 0.5)
        dx, dy = rng.normal(size=2)
        nrm = math.hypot(dx, dy)
        dx, dy = dx / nrm, dy / nrm
        t = 100.0  # far beyond the grid: cells outside are vacuum
        Q = (P[0] + t * dx, P[1] + t * dy)
        # oracle frame here: first coordinate indexes axis 0 of E; use E.T so that
        # (x, y) = (column, row) as in the brute force
        L, _ = hrc.trace(E.T, Sg.T, P, Q)
        Lb = bruteforce.radiance(E, Sg, P[0], P[1], dx, dy)
        assert L == pytest.approx(Lb, rel=1e-10, abs=1e-12)


# ---------------------------------------------------------------- P2-P4 ---
def test_zero_emission_gives_zero_fluence():
    E, Sg = _rng_scene(32, 1)
    assert np.all(hrc.fluence(np.zeros_like(E), Sg) == 0.0)


def test_linearity_in_emission():
    E1, Sg = _rng_scene(32, 2)
    E2, _ = _rng_scene(32, 3)
    F = hrc.fluence(2.5 * E1 + 0.5 * E2, Sg)
    F12 = 2.5 * hrc.fluence(E1, Sg) + 0.5 * hrc.fluence(E2, Sg)
    assert np.allclose(F, F12, rtol=1e-12, atol=1e-12 * np.abs(F).max())


def test_vacuum_transmittance_is_one_everywhere():
    E, _ = _rng_scene(32, 4)
    T = hrc.build_pyramid(E, np.zeros_like(E))
    for TL, TT in T:
        assert np.all(TT == 1.0)


# ---------------------------------------------------------------- P5/P14 --
@pytest.mark.parametrize("S", [16, 32])
def test_even_split_directions_are_exact_traces(S):
    """Eq. 18 is exact: T_n(p, k) built by even splits only (k a multiple of
    2^(n-2), down to the traced level 2) equals Trace(p, p + v_n(k)) computed
    directly, including probes whose far half leaves the grid."""
    E, Sg = _rng_scene(S, 5, 0.5)
    T = hrc.build_pyramid(E, Sg, seed_levels=3)
    N = hrc.log2_size(S)
    rng = np.random.default_rng(1)
    for n in range(3, N + 1):
        a = 2 ** n
        for k in range(0, a + 1, a // 4):
            for _ in range(6):
                x = int(rng.integers(0, S // a))
                y = int(rng.integers(0, S))
                P = (x * a + 0.5, y + 0.5)
                L, Tr = hrc.trace(E, Sg, P, (P[0] + a, P[1] + 2 * k - a))
                assert T[n][0][x, k, y] == pytest.approx(L, rel=1e-12, abs=1e-14)
                assert T[n][1][x, k, y] == pytest.approx(Tr, rel=1e-12, abs=1e-300)


def test_pure_hrc_differs_only_in_odd_blends():
    """Tracing every level (no acceleration structure) changes only entries
    that contain an odd-direction blend (Eq. 19-20)."""
    E, Sg = _rng_scene(32, 6, 0.5)
    Ta = hrc.build_pyramid(E, Sg, seed_levels=3)
    Tp = hrc.build_pyramid(E, Sg, seed_levels=6)
    for n in range(3, 6):
        a = 2 ** n
        ks = list(range(0, a + 1, a // 4))
        assert np.allclose(Ta[n][0][:, ks], Tp[n][0][:, ks], rtol=1e-12, atol=1e-14)
        assert not np.allclose(Ta[n][0], Tp[n][0], rtol=1e-6)


def test_odd_blends_approximate_the_straight_trace():
    """The bent two-segment paths of Eq. 19 end where the straight ray ends, so
    their mean stays close to the exact trace (measured bound on a config-1
    scene; a wrong far offset roughly doubles the deviation)."""
    sc = config1()
    E = sc.eps.astype(float)
    Sg = sc.sigma.astype(float) * 0.2
    Ta = hrc.build_pyramid(E, Sg, 3)
    Tp = hrc.build_pyramid(E, Sg, 7)
    for n, bound in ((3, 0.09), (4, 0.11)):
        La, Lp = Ta[n][0][:, 1::2], Tp[n][0][:, 1::2]
        assert np.abs(La - Lp).mean() / np.abs(Lp).mean() < bound


# ---------------------------------------------------------------- P7 ------
@pytest.mark.parametrize("S", [8, 32, 64])
def test_opaque_unit_pyramid_angular_bookkeeping(S):
    """Inject T = <1, 0> everywhere: each half-cone then carries exactly its arc
    (Eq. 13-17), so R_n(p, ii) = A_n(ii) for x >= 1 and (1 - 2^(n-N)) A_n(ii) at
    x = 0 (R_N = 0); the gathered fluence is 2*pi inside, 3*pi/2 on an edge and
    pi at a corner (Algorithm 1, Lighting, offset x+1)."""
    N = hrc.log2_size(S)
    T = [(np.ones((S >> n, 2 ** n + 1, S)), np.zeros((S >> n, 2 ** n + 1, S)))
         for n in range(N + 1)]
    R = hrc.cascades_from_pyramid(T)
    for n in range(N):
        A = np.array([hrc.cone_angle(n, ii) for ii in range(2 ** n)])
        assert np.allclose(R[n][1:], A[None, :, None], rtol=1e-13, atol=0)
        assert np.allclose(R[n][0], (1 - 2.0 ** (n - N)) * A[:, None], rtol=1e-13)
    Q = hrc.gather(R[0])
    F = sum(hrc.from_frame(Q, d) for d in hrc.QUADRANTS)
    assert np.allclose(F[1:-1, 1:-1], 2 * math.pi, rtol=1e-13)
    assert np.allclose(F[0, 1:-1], 1.5 * math.pi, rtol=1e-13)
    assert np.allclose(F[1:-1, -1], 1.5 * math.pi, rtol=1e-13)
    assert F[0, 0] == pytest.approx(math.pi, rel=1e-13)
    assert F[-1, -1] == pytest.approx(math.pi, rel=1e-13)


# ---------------------------------------------------------------- P8 ------
@pytest.mark.parametrize("S", [32, 64])
def test_kirchhoff_isothermal_medium(S):
    """eps = sig * B everywhere: every interval has L = B (1 - T) (preserved by
    Eq. 7, by the averages of Eq. 15/20 and by Eq. 8), so F = B (2 pi - sum w T)
    <= 2 pi B, and F = 2 pi B where every path is optically thick (>= 40)."""
    sig = np.full((S, S), 5.0)
    B = 1.7
    F = hrc.fluence(sig * B, sig)
    assert np.all(F <= 2 * math.pi * B * (1 + 1e-12))
    assert np.allclose(F[8:-8, 8:-8], 2 * math.pi * B, rtol=1e-12)
    # and with a patchy medium (sig varies, eps/sig constant) the interval
    # identity still holds for every pyramid entry
    rng = np.random.default_rng(3)
    sig2 = rng.uniform(0.05, 3.0, (S, S))
    T = hrc.build_pyramid(sig2 * B, sig2)
    for TL, TT in T:
        assert np.allclose(TL, B * (1 - TT), rtol=1e-11, atol=1e-12)


# ---------------------------------------------------------------- P9 ------
def test_d4_equivariance():
    """The four quadrant solves are related by the symmetries of the square, so
    F commutes with transposes and flips of the scene."""
    E, Sg = _rng_scene(32, 8, 0.7)
    F = hrc.fluence(E, Sg)
    for g in (lambda a: a.T, lambda a: a[::-1], lambda a: a[:, ::-1],
              lambda a: np.rot90(a), lambda a: np.rot90(a, 2)):
        assert np.allclose(hrc.fluence(g(E), g(Sg)), g(F), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- P11 -----
@pytest.mark.parametrize("S", [8, 64, 1024])
def test_entry_counts(S):
    """Section 4.3: #R_n = X^2, #T_n = X^2 (1 + 2^-n), and 4*(#T_0+#T_1+#T_2)
    = 19 X^2 traced intervals per frame."""
    t, r = hrc.entry_counts(S)
    N = hrc.log2_size(S)
    assert all(v == S * S for v in r) and len(r) == N
    assert all(t[n] == S * S * (1 + 2.0 ** -n) for n in range(N + 1))
    assert 4 * sum(t[:3]) == 19 * S * S
    assert sum(t) == pytest.approx((N + 3 - 2.0 ** -N) * S * S)


def test_probe_centres_see_symmetric_quadrants():
    """Single emissive pixel in vacuum: the fluence is symmetric under the
    symmetries of the square that fix that pixel."""
    S = 33 - 1
    E = np.zeros((S, S)); E[16, 16] = 1.0
    F = hrc.fluence(E, np.zeros_like(E))
    assert np.allclose(F, F.T, rtol=1e-13, atol=1e-15)
