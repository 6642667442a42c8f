"""Closed-form fluences that pin the brute force of Eq. 1-3 (test infrastructure only).

* Vacuum (sigma = 0): L(p, w) = int eps(p + t w) dt, so by polar coordinates
  F(p) = int eps(x)/|x - p| dA.  For a uniform rectangle this integral has the
  closed form built from G(a, b) = a*asinh(b/a) + b*asinh(a/b), the integral of
  1/r over [0,a]x[0,b].
* Uniform medium (eps, sig constant on the grid, vacuum outside): a ray of
  in-grid length d carries (eps/sig)*(1 - exp(-sig*d)), so F(p) is a 1-D angle
  integral of that, done by adaptive quadrature between the corner angles.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate


def _G(a: float, b: float) -> float:
    if a == 0.0 or b == 0.0:
        return 0.0
    return a * math.asinh(b / a) + b * math.asinh(a / b)


def _H(a: float, b: float) -> float:
    """Signed integral of 1/r over the rectangle between the origin and (a, b)."""
    return math.copysign(1.0, a) * math.copysign(1.0, b) * _G(abs(a), abs(b))


def rect_inverse_distance(px, py, x0, x1, y0, y1) -> float:
    """int over [x0,x1]x[y0,y1] of 1/|x - p| dA."""
    ax0, ax1, ay0, ay1 = x0 - px, x1 - px, y0 - py, y1 - py
    return _H(ax1, ay1) - _H(ax0, ay1) - _H(ax1, ay0) + _H(ax0, ay0)


def vacuum_fluence(eps, r: int, c: int) -> float:
    """Exact F at the centre of pixel (r, c) of a scene with sigma = 0."""
    eps = np.asarray(eps, dtype=np.float64)
    px, py = c + 0.5, r + 0.5
    total = 0.0
    for (rr, cc) in zip(*np.nonzero(eps)):
        total += eps[rr, cc] * rect_inverse_distance(px, py, cc, cc + 1, rr, rr + 1)
    return total


def uniform_medium_fluence(S: int, eps: float, sig: float, r: int, c: int) -> float:
    """F at the centre of pixel (r, c) of an S x S grid of constant eps and sig."""
    px, py = c + 0.5, r + 0.5

    def dist(th):
        dx, dy = math.cos(th), math.sin(th)
        tx = (S - px) / dx if dx > 0 else (-px / dx if dx < 0 else math.inf)
        ty = (S - py) / dy if dy > 0 else (-py / dy if dy < 0 else math.inf)
        return min(tx, ty)

    def radiance(th):
        d = dist(th)
        if sig == 0.0:
            return eps * d
        return eps / sig * (-math.expm1(-sig * d))

    corners = sorted(math.atan2(y - py, x - px) % (2 * math.pi)
                     for x, y in ((0, 0), (S, 0), (0, S), (S, S)))
    edges = [0.0] + corners + [2 * math.pi]
    total = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        if b > a:
            val, _ = integrate.quad(radiance, a, b, epsabs=0, epsrel=1e-12, limit=200)
            total += val
    return total
