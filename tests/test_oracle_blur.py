"""Pins of the cross-blur oracle (Eq. 21 with opacity rejection) and of its
adjoint, against facts that do not come from the oracle itself."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import blur

KERNEL = np.array([[0, 1, 0], [1, 4, 1], [0, 1, 0]], np.float64) / 8.0


def test_uniform_medium_interior_is_eq21_convolution():
    """Where all four neighbours are kept, the filter is Eq. 21 exactly: the
    interior matches a library convolution with (1/8)[0 1 0; 1 4 1; 0 1 0]."""
    rng = np.random.default_rng(1)
    F = rng.random((12, 12))
    sig = np.full((12, 12), 0.3)
    got = blur.cross_blur(F, sig)
    want = ndimage.convolve(F, KERNEL, mode="constant")
    assert np.allclose(got[1:-1, 1:-1], want[1:-1, 1:-1], rtol=0, atol=1e-15)


def test_border_renormalises_over_kept_neighbours():
    """A corner keeps two neighbours (4 F + F_a + F_b) / 6; an edge three."""
    F = np.arange(16, dtype=np.float64).reshape(4, 4)
    sig = np.zeros((4, 4))
    got = blur.cross_blur(F, sig)
    assert got[0, 0] == pytest.approx((4 * F[0, 0] + F[1, 0] + F[0, 1]) / 6)
    assert got[0, 2] == pytest.approx((4 * F[0, 2] + F[1, 2] + F[0, 1] + F[0, 3]) / 7)


def test_constant_field_is_unchanged():
    rng = np.random.default_rng(2)
    sig = rng.random((10, 10)) * rng.choice([0.0, 3.0], size=(10, 10))
    F = np.full((10, 10), 2.5)
    assert np.allclose(blur.cross_blur(F, sig), 2.5, rtol=0, atol=1e-15)


def test_checkerboard_averages_to_one_half():
    """The artifact the blur is for (Section 5.0.3): a 0/1 checkerboard in a
    uniform medium becomes 1/2 in the interior ((4*1 + 0)/8 and (0 + 4)/8)."""
    F = (np.indices((8, 8)).sum(0) % 2).astype(np.float64)
    got = blur.cross_blur(F, np.zeros((8, 8)))
    assert np.allclose(got[1:-1, 1:-1], 0.5, rtol=0, atol=1e-15)


def test_opaque_wall_blocks_the_filter():
    """Across a wall whose opacity differs by more than the threshold, nothing
    leaks: changing F on one side leaves the other side's output unchanged."""
    S = 10
    sig = np.zeros((S, S))
    sig[:, 5] = 50.0  # opacity ~1 against 0 on both sides
    rng = np.random.default_rng(3)
    F = rng.random((S, S))
    G = F.copy()
    G[:, 6:] += 10.0
    a, b = blur.cross_blur(F, sig), blur.cross_blur(G, sig)
    assert np.array_equal(a[:, :5], b[:, :5])
    # the wall pixels keep only their wall neighbours (vertical)
    r = 4
    assert a[r, 5] == pytest.approx((4 * F[r, 5] + F[r - 1, 5] + F[r + 1, 5]) / 6)


def test_threshold_edge_is_inclusive():
    """An opacity difference equal to the threshold keeps the neighbour; the
    next threshold below it drops it (both compared in FP32)."""
    sig = np.array([[0.0, 0.7]], np.float32)
    d = np.abs(blur.opacity(sig)[0, 1] - blur.opacity(sig)[0, 0])
    F = np.array([[1.0, 3.0]])
    got = blur.cross_blur(F, sig, threshold=float(d))
    assert got[0, 0] == pytest.approx((4 * 1.0 + 3.0) / 5)
    got = blur.cross_blur(F, sig, threshold=float(np.nextafter(d, np.float32(0))))
    assert got[0, 0] == pytest.approx(1.0)


def test_opacity_is_one_minus_transmittance():
    sig = np.array([0.0, 0.5, 3.0], np.float32)
    assert np.allclose(blur.opacity(sig), 1 - np.exp(-sig.astype(np.float64)), rtol=1e-6)


@pytest.mark.parametrize("seed", [4, 5])
def test_adjoint_dot_product(seed):
    """<blur(x), y> = <x, blur^T(y)> for random fields with rejections."""
    rng = np.random.default_rng(seed)
    S = 9
    sig = rng.random((S, S)) * rng.choice([0.0, 5.0], size=(S, S))
    x, y = rng.normal(size=(S, S)), rng.normal(size=(S, S))
    lhs = float((blur.cross_blur(x, sig) * y).sum())
    rhs = float((x * blur.cross_blur_vjp(y, sig)).sum())
    assert lhs == pytest.approx(rhs, rel=1e-13, abs=1e-13)


def test_adjoint_matches_explicit_matrix():
    """Column j of the filter matrix from unit inputs; its transpose applied to
    a unit output equals the VJP of that output."""
    rng = np.random.default_rng(6)
    S = 5
    sig = rng.random((S, S)) * rng.choice([0.0, 4.0], size=(S, S))
    M = np.zeros((S * S, S * S))
    for j in range(S * S):
        e = np.zeros(S * S)
        e[j] = 1.0
        M[:, j] = blur.cross_blur(e.reshape(S, S), sig).ravel()
    for i in (0, 7, 12, 24):
        e = np.zeros(S * S)
        e[i] = 1.0
        assert np.allclose(blur.cross_blur_vjp(e.reshape(S, S), sig).ravel(), M[i, :],
                           rtol=0, atol=1e-15)
