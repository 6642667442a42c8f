"""The tolerance of the 16-bit interval storage (HRC_FLAG_HALF_INTERVALS),
checked on the oracle's own steps.

Section 5 stores radiance and transmittance in 16-bit floats.  The kernels
store the interval levels that pass through memory, T_2 .. T_(N-1), as IEEE
half floats (T_0, T_1 and T_N never leave the chip in the forward), computing
everything else in FP32.  Every forward quantity is a sum or product of
non-negative values, so a relative rounding of at most u = 2^-11 at each of
the at most N - 2 stores on any path from the inputs changes the fluence by a
relative (N - 2) u to first order, below the N u the GPU test allows; values in
the half's subnormal range carry an absolute 2^-25 instead, which the test's
floor (relative to the largest fluence) covers.  This model rounds the oracle's
FP64 levels at the same points and checks that bound, so that the GPU test's
tolerance rests on more than the argument above."""
import sys

import numpy as np
import pytest

from oracle import hrc as O
from scenes import config1, scene_like_512

HALF_RTOL_PER_LEVEL = 2.0 ** -11
HALF_FLOOR = 1e-6


def _q16(a):
    return np.asarray(a, np.float64).astype(np.float16).astype(np.float64)


def _quadrant_half(E, Sg):
    """One quadrant with T_2 .. T_(N-1) rounded to half where they are stored;
    the merge down of levels 1 and 0 reads the unrounded T_0 .. T_2 (the
    kernels fold those on chip) and T_N is built from the rounded T_(N-1)."""
    S = E.shape[0]
    N = O.log2_size(S)
    T = [O.seed_level(E, Sg, n) for n in range(3)]
    Tq = [None, None, tuple(_q16(a) for a in T[2])]
    for n in range(3, N + 1):
        t = O.merge_up(Tq[n - 1], n)
        Tq.append(tuple(_q16(a) for a in t) if n < N else t)
    R = [None] * (N + 1)
    R[N] = np.zeros((1, 2 ** N, S))
    for n in range(N - 1, -1, -1):
        if n >= 2:
            R[n] = O.merge_down(R[n + 1], Tq[n], Tq[n + 1], n)
        else:
            R[n] = O.merge_down(R[n + 1], T[n], T[n + 1], n)
    return O.gather(R[0])


def _fluence_half(eps, sig):
    eps = np.asarray(eps, np.float64)
    sig = np.asarray(sig, np.float64)
    F = np.zeros(eps.shape)
    for d in O.QUADRANTS:
        F += O.from_frame(_quadrant_half(O.to_frame(eps, d), O.to_frame(sig, d)), d)
    return F


@pytest.mark.parametrize("which", ["64 disks3_boxes4", "256 like-512"])
def test_half_storage_stays_within_n_half_ulps(which):
    sc = config1() if which.startswith("64") else scene_like_512(256, 11, 8, 16)
    F = O.fluence(sc.eps, sc.sigma)
    Fh = _fluence_half(sc.eps, sc.sigma)
    N = O.log2_size(F.shape[0])
    err = np.abs(Fh - F)
    bound = N * HALF_RTOL_PER_LEVEL * np.abs(F) + HALF_FLOOR * np.abs(F).max()
    assert (err <= bound).all(), float(np.max(err / bound))
    # the storage does round (the check is not vacuous), and by more than FP32
    assert np.max(err / np.maximum(np.abs(F), 1e-300)) > 1e-5


def test_model_without_rounding_is_the_oracle(monkeypatch):
    """With the rounding taken out the model is the oracle's forward, bit for
    bit: it differs from it only where the kernels store a level."""
    monkeypatch.setattr(sys.modules[__name__], "_q16", lambda a: np.asarray(a, np.float64))
    sc = config1()
    assert np.array_equal(_fluence_half(sc.eps, sc.sigma), O.fluence(sc.eps, sc.sigma))


def _pyramid_half_reverse(E, Sg, seed_levels=3):
    """The reverse's recomputed pyramid as the kernels store it with 16-bit
    intervals: T_0 .. T_(N-1) rounded to half (traced levels rounded once,
    each merged level computed from the rounded one below and rounded), T_N
    built from the rounded T_(N-1) and never stored."""
    S = E.shape[0]
    N = O.log2_size(S)
    T = []
    for n in range(N + 1):
        t = O.seed_level(E, Sg, n) if n < seed_levels else O.merge_up(T[n - 1], n)
        T.append(tuple(_q16(a) for a in t) if n < N else t)
    return T


@pytest.mark.parametrize("which", ["64 disks3_boxes4", "128 like-512"])
def test_half_reverse_within_the_derived_bound(which, monkeypatch):
    """The reverse with the 16-bit pyramid stays within N 2^-11 times the
    gradient of abs(dLoss/dF), element by element, on the oracle's own steps:
    every gradient term is a fluence term with one factor differentiated, the
    terms of d eps are all >= 0 and those of d sigma all <= 0, and a term
    passes through at most N rounded values."""
    from oracle import hrc_vjp
    sc = config1() if which.startswith("64") else scene_like_512(128, 12, 4, 8)
    S = sc.eps.shape[0]
    N = O.log2_size(S)
    dF = np.random.default_rng(S).normal(size=(S, S))
    ge, gs = hrc_vjp.fluence_vjp(sc.eps, sc.sigma, dF)
    ae, as_ = hrc_vjp.fluence_vjp(sc.eps, sc.sigma, np.abs(dF))
    assert (ae >= 0).all() and (as_ <= 0).all()  # one sign per field
    monkeypatch.setattr(hrc_vjp, "build_pyramid", _pyramid_half_reverse)
    he, hs = hrc_vjp.fluence_vjp(sc.eps, sc.sigma, dF)
    for g16, g, ga, name in ((he, ge, ae, "d eps"), (hs, gs, as_, "d sigma")):
        err = np.abs(g16 - g)
        # Below 2^-14 half is subnormal: a stored value keeps an absolute
        # precision of 2^-24 there, not a relative one, and a term whose
        # factors underflow is lost whole.  Those terms are tiny beside the
        # largest gradient, hence the absolute term (the same the GPU tests
        # carry); where the gradient is not tiny the relative bound alone holds.
        bound = N * HALF_RTOL_PER_LEVEL * np.abs(ga) + 1e-4 * np.abs(ga).max()
        assert (err <= bound).all(), (name, float(np.max(err / bound)))
        big = np.abs(ga) >= 1e-3 * np.abs(ga).max()
        rel = err[big] / (N * HALF_RTOL_PER_LEVEL * np.abs(ga[big]))
        assert rel.max() <= 1.0, (name, float(rel.max()))
        # the storage does perturb the gradient (the check is not vacuous)
        assert rel.max() > 1e-3, (name, float(rel.max()))


def test_half_reverse_model_without_rounding_is_the_oracle(monkeypatch):
    from oracle import hrc_vjp
    sc = config1()
    dF = np.random.default_rng(3).normal(size=sc.eps.shape)
    want = hrc_vjp.fluence_vjp(sc.eps, sc.sigma, dF)
    monkeypatch.setattr(sys.modules[__name__], "_q16", lambda a: np.asarray(a, np.float64))
    monkeypatch.setattr(hrc_vjp, "build_pyramid", _pyramid_half_reverse)
    got = hrc_vjp.fluence_vjp(sc.eps, sc.sigma, dF)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
