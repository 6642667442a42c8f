"""FP64 oracle of the cross blur that follows Algorithm 1 (Eq. 21), and of its
adjoint (test infrastructure only; see the package doc).

Eq. 21 filters the summed fluence with (1/8) [0 1 0; 1 4 1; 0 1 0] and ignores
the neighbours whose opacity differs significantly from the target's.  The
paper quantifies neither the opacity nor "significantly"; the readings here:

* the opacity of a pixel is that of one cell side of its medium,
  alpha = 1 - exp(-sigma_t);
* a neighbour is ignored when |alpha(neighbour) - alpha(target)| > threshold,
  threshold 0.5 by default, and so is a neighbour outside the grid;
* ignoring renormalises: out = (4 F(target) + sum of kept F(neighbour)) /
  (4 + number kept), which is Eq. 21 exactly where all four are kept and
  leaves a constant field unchanged everywhere.

The kept/ignored choice is piecewise constant in sigma_t, so the adjoint
carries no dLoss/d sigma_t term from the blur (its derivative is zero almost
everywhere); dLoss/dF is the transpose of the linear filter.

The choice is an integer outcome decided in floating point; it is taken in
FP32 (the kernel's precision, the paper fixing none), so that both sides keep
the same neighbours.  The averaging itself is FP64.
"""
from __future__ import annotations

import numpy as np

DEFAULT_THRESHOLD = 0.5
NEIGHBOURS = ((-1, 0), (1, 0), (0, -1), (0, 1))


def opacity(sigma):
    """alpha = 1 - exp(-sigma_t) of one unit cell side, in FP32 (the precision
    in which the kept neighbours are chosen)."""
    return -np.expm1(-np.asarray(sigma, np.float32))


def kept_neighbours(sigma, threshold: float = DEFAULT_THRESHOLD):
    """keep[i][r][c] for neighbour i of NEIGHBOURS: inside the grid and within
    ``threshold`` in opacity of pixel (r, c) (compared in FP32)."""
    a = opacity(sigma)
    thr = np.float32(threshold)
    S0, S1 = a.shape
    keep = np.zeros((4,) + a.shape, dtype=bool)
    for i, (dr, dc) in enumerate(NEIGHBOURS):
        for r in range(S0):
            for c in range(S1):
                rr, cc = r + dr, c + dc
                if 0 <= rr < S0 and 0 <= cc < S1:
                    keep[i, r, c] = np.abs(a[rr, cc] - a[r, c]) <= thr
    return keep


def cross_blur(F, sigma, threshold: float = DEFAULT_THRESHOLD):
    """Eq. 21 with opacity rejection and renormalisation (module doc)."""
    F = np.asarray(F, np.float64)
    keep = kept_neighbours(sigma, threshold)
    S0, S1 = F.shape
    out = np.empty_like(F)
    for r in range(S0):
        for c in range(S1):
            acc, wsum = 4.0 * F[r, c], 4.0
            for i, (dr, dc) in enumerate(NEIGHBOURS):
                if keep[i, r, c]:
                    acc += F[r + dr, c + dc]
                    wsum += 1.0
            out[r, c] = acc / wsum
    return out


def cross_blur_vjp(dOut, sigma, threshold: float = DEFAULT_THRESHOLD):
    """dLoss/dF given dLoss/d(cross_blur(F)): every output (r, c) sends its
    weight 4/(4+k) to F(r, c) and 1/(4+k) to each kept neighbour."""
    dOut = np.asarray(dOut, np.float64)
    keep = kept_neighbours(sigma, threshold)
    S0, S1 = dOut.shape
    dF = np.zeros_like(dOut)
    for r in range(S0):
        for c in range(S1):
            k = int(keep[:, r, c].sum())
            g = dOut[r, c] / (4.0 + k)
            dF[r, c] += 4.0 * g
            for i, (dr, dc) in enumerate(NEIGHBOURS):
                if keep[i, r, c]:
                    dF[r + dr, c + dc] += g
    return dF
