"""Helpers shared by the GPU tests: tolerances and tensor plumbing."""
import sys

import numpy as np
import torch

# Forward tolerance.  Every forward operation adds or multiplies non-negative
# numbers (L >= 0, T in [0, 1], arcs > 0, positive averaging weights), so the
# FP32 result has a componentwise relative error of about depth * 2^-24 with a
# depth of ~40 operations (~2.4e-6); 1e-4 leaves margin for the FP32
# exponentials of the traced cells.  The absolute floor covers transmittances
# that underflow FP32 (sigma = 100 lines give exp(-100 l)).
FWD_RTOL = 1e-4
FWD_FLOOR = 1e-7


def assert_forward_close(F_gpu, F_ref, what=""):
    F_gpu = np.asarray(F_gpu, dtype=np.float64)
    F_ref = np.asarray(F_ref, dtype=np.float64)
    assert F_gpu.shape == F_ref.shape
    bound = FWD_RTOL * np.abs(F_ref) + FWD_FLOOR * np.abs(F_ref).max()
    err = np.abs(F_gpu - F_ref)
    bad = err > bound
    if bad.any():
        i = np.unravel_index(np.argmax(err / np.maximum(bound, 1e-300)), err.shape)
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} outside tolerance; worst at {i}: "
                             f"gpu {F_gpu[i]!r} ref {F_ref[i]!r}")


# Forward tolerance with the 16-bit interval storage (HRC_FLAG_HALF_INTERVALS):
# each of the at most N - 2 stored levels on a path adds a relative rounding of
# at most 2^-11 to non-negative sums and products, so N * 2^-11 componentwise
# (plus FP32's 1e-4), with a floor for values in the half's subnormal range
# (absolute 2^-25 each).  tests/test_oracle_half_storage.py checks the bound on
# the oracle's steps rounded at the same points.
HALF_RTOL_PER_LEVEL = 2.0 ** -11
HALF_FLOOR = 1e-6


def assert_half_close(F_gpu, F_ref, N, what=""):
    F_gpu = np.asarray(F_gpu, dtype=np.float64)
    F_ref = np.asarray(F_ref, dtype=np.float64)
    assert F_gpu.shape == F_ref.shape
    rtol = N * HALF_RTOL_PER_LEVEL + FWD_RTOL
    bound = rtol * np.abs(F_ref) + HALF_FLOOR * np.abs(F_ref).max()
    err = np.abs(F_gpu - F_ref)
    bad = err > bound
    if bad.any():
        i = np.unravel_index(np.argmax(err / np.maximum(bound, 1e-300)), err.shape)
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} outside the 16-bit storage "
                             f"bound; worst at {i}: gpu {F_gpu[i]!r} ref {F_ref[i]!r}")
    return float(np.max(err / np.maximum(np.abs(F_ref), 1e-300) * (np.abs(F_ref) > 1e-3 * np.abs(F_ref).max())))


# Gradient tolerance: the reverse pass sums signed terms (the loss residual), so
# the bound is relative to the largest gradient, plus a relative check on the
# entries that carry most of the gradient.
GRAD_ATOL_REL = 1e-4
GRAD_RTOL_LARGE = 1e-3


def assert_grad_close(g_gpu, g_ref, what=""):
    g_gpu = np.asarray(g_gpu, dtype=np.float64)
    g_ref = np.asarray(g_ref, dtype=np.float64)
    gmax = np.abs(g_ref).max()
    err = np.abs(g_gpu - g_ref)
    assert err.max() <= GRAD_ATOL_REL * gmax, f"{what}: max err {err.max()} vs {gmax}"
    large = np.abs(g_ref) > 1e-2 * gmax
    rel = err[large] / np.abs(g_ref[large])
    assert rel.max() <= GRAD_RTOL_LARGE, f"{what}: max rel err on large entries {rel.max()}"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def assert_half_grad(g16, g_ref, g_abs, N, what):
    """Each gradient element within N 2^-11 times the same gradient taken with
    abs(dLoss/dF) (every term of a gradient is a fluence term with one factor
    differentiated: one sign per field, and at most N roundings on its path),
    plus the FP32 reverse's own tolerance."""
    g16 = np.asarray(g16, np.float64)
    err = np.abs(g16 - g_ref)
    bound = N * 2.0 ** -11 * np.abs(g_abs) + 1e-4 * np.abs(g_ref).max()
    bad = err > bound
    if bad.any():
        i = np.unravel_index(np.argmax(err / np.maximum(bound, 1e-300)), err.shape)
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} outside the 16-bit reverse "
                             f"bound; worst at {i}: gpu {g16[i]!r} ref {g_ref[i]!r} "
                             f"abs-gradient {g_abs[i]!r}")
