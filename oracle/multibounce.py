"""FP64 oracle of multiple diffuse bounces (test infrastructure only; see the
package doc).

Section 4.2 obtains further bounces by feeding the output fluence back into
another run of the algorithm; the paper does not say how fluence becomes a
source.  The reading here is isotropic in-scattering in the plane: a pixel with
attenuation sigma_t and albedo a scatters the fraction a of what it attenuates,
evenly over the 2 pi directions, so the emission per unit length seen by the
next bounce is

    eps_{k+1} = eps_0 + a * sigma_t * F_k / (2 pi).

Bounce k solves HRC(eps_k, sigma_t); the result is F_{K-1} after K bounces
(K = 1 is the single-bounce Algorithm 1).  Deep inside a thick uniform medium
each bounce gives F = 2 pi eps / sigma_t, so F_K = (2 pi eps_0 / sigma_t) *
sum_{j<K} a^j, a closed form the tests use.
"""
from __future__ import annotations

import math

import numpy as np

from . import hrc
from . import hrc_vjp


def scatter_source(eps0, sigma, albedo, F):
    """eps_0 + a sigma_t F / (2 pi)."""
    return np.asarray(eps0, np.float64) + (np.asarray(albedo, np.float64) *
                                           np.asarray(sigma, np.float64) *
                                           np.asarray(F, np.float64)) / (2 * math.pi)


def fluence(eps0, sigma, albedo, bounces: int, environment=None):
    """F_{K-1} of K = ``bounces`` >= 1 bounces (module doc)."""
    if bounces < 1:
        raise ValueError("bounces must be >= 1")
    e = np.asarray(eps0, np.float64)
    F = hrc.fluence(e, sigma, environment=environment)
    for _ in range(1, bounces):
        e = scatter_source(eps0, sigma, albedo, F)
        F = hrc.fluence(e, sigma, environment=environment)
    return F


def fluence_vjp(eps0, sigma, albedo, bounces: int, dF, environment=None):
    """(dLoss/d eps_0, dLoss/d sigma_t, dLoss/d albedo) given dLoss/dF of
    ``fluence``: the bounces reversed, each through ``hrc_vjp.fluence_vjp`` at
    its own source, plus the source's dependence on F, sigma_t and albedo."""
    eps0 = np.asarray(eps0, np.float64)
    sigma = np.asarray(sigma, np.float64)
    albedo = np.asarray(albedo, np.float64)
    # forward, keeping every bounce's source and result
    srcs, Fs = [eps0], [hrc.fluence(eps0, sigma, environment=environment)]
    for _ in range(1, bounces):
        srcs.append(scatter_source(eps0, sigma, albedo, Fs[-1]))
        Fs.append(hrc.fluence(srcs[-1], sigma, environment=environment))
    d_eps0 = np.zeros_like(eps0)
    d_sig = np.zeros_like(eps0)
    d_alb = np.zeros_like(eps0)
    g = np.asarray(dF, np.float64)
    for k in range(bounces - 1, -1, -1):
        dE, dS = hrc_vjp.fluence_vjp(srcs[k], sigma, g, environment=environment)
        d_sig += dS
        d_eps0 += dE
        if k >= 1:
            Fp = Fs[k - 1]
            d_sig += albedo * Fp * dE / (2 * math.pi)
            d_alb += sigma * Fp * dE / (2 * math.pi)
            g = albedo * sigma * dE / (2 * math.pi)
    return d_eps0, d_sig, d_alb
