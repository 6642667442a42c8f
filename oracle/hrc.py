"""FP64 oracle of the HRC forward pass (test infrastructure only; see package doc).

Conventions (the paper's notation, with the readings the paper leaves open):

* One quadrant solve works in a frame (u, w) whose facing axis is +u
  (Section 4, "assume we only consider the angular fluence between -pi/4 and
  pi/4").  Pixel (u, w) is the unit square [u, u+1) x [w, w+1) with uniform
  emission E[u][w] and attenuation Sg[u][w] (Section 5).
* Probe (n, x, y) sits at the pixel centre P = (x*2^n + 1/2, y + 1/2)
  (Section 4 places probes at (x*2^n, y); the centre is our reading).
* v_n(k) = (2^n, 2k - 2^n), k = 0..2^n (Section 4, Section 4.1).
* Cone ii = i - 1/2 of level n spans the edges v_n(ii) and v_n(ii+1), ii = 0..2^n-1.
* ``E`` is emission per unit length (the integrand of Eq. 3).  A uniform cell
  crossed over length l contributes <E*(1-exp(-Sg*l))/Sg, exp(-Sg*l)>.
* Everything outside the grid is vacuum with no light (Section 4.2: no lights
  beyond the region), so an out-of-grid interval lookup is <0, 1> and an
  out-of-grid angular fluence lookup is 0.

Arrays: ``T`` levels are pairs (TL, TT) of shape [S/2^n, 2^n+1, S] indexed
[x][k][y]; ``R`` levels have shape [S/2^n, 2^n, S] indexed [x][ii][y].
"""
from __future__ import annotations

from fractions import Fraction
import math

import numpy as np

QUADRANTS = ("+x", "-x", "+y", "-y")


# --------------------------------------------------------------------------
# Interval algebra (Section 3, Eq. 2-9)
# --------------------------------------------------------------------------

def cell_interval(eps, sig, ell):
    """<L, T> of a straight chord of length ``ell`` through a uniform cell.

    Eq. 2 gives T = exp(-sig*ell); Eq. 4 with a constant integrand gives
    L = int_0^ell exp(-sig*t) eps dt = eps*ell*phi(sig*ell), phi(tau) = (1-e^-tau)/tau.
    """
    eps = np.asarray(eps, dtype=np.float64)
    sig = np.asarray(sig, dtype=np.float64)
    tau = sig * ell
    small = tau < 1e-5
    safe = np.where(small, 1.0, tau)
    phi = np.where(small, 1.0 - tau / 2.0 + tau * tau / 6.0, -np.expm1(-safe) / safe)
    return eps * ell * phi, np.exp(-tau)


def merge(near, far):
    """Eq. 7: Merge(<Ln,Tn>, <Lf,Tf>) = <Ln + Tn*Lf, Tn*Tf> (near interval first)."""
    (ln, tn), (lf, tf) = near, far
    return ln + tn * lf, tn * tf


def merge_r(near, rf):
    """Eq. 8: Merge_r(<Ln,Tn>, rf) = Ln + Tn*rf."""
    ln, tn = near
    return ln + tn * rf


def cone_angle(m: int, jj: int) -> float:
    """Eq. 13: A_m(i) = angle(v_m(i+1/2)) - angle(v_m(i-1/2)) with i = jj + 1/2,
    i.e. the arc between the edges v_m(jj) and v_m(jj+1)."""
    a = 2 ** m
    return math.atan2(2 * (jj + 1) - a, a) - math.atan2(2 * jj - a, a)


# --------------------------------------------------------------------------
# Trace (Eq. 9) by a generic segment/grid traversal
# --------------------------------------------------------------------------

def segment_cells(P, Q):
    """Cells crossed by the segment P->Q, in order from P, with exact chord lengths.

    The segment is cut at every crossing of an integer u or w line; each piece
    lies in one cell, found from its midpoint.  Rational arithmetic keeps
    crossings that coincide (corners) exact, so corner touches give no piece.
    Returns a list of (cell_u, cell_w, length).
    """
    pu, pw = Fraction(P[0]), Fraction(P[1])
    qu, qw = Fraction(Q[0]), Fraction(Q[1])
    du, dw = qu - pu, qw - pw
    ts = {Fraction(0), Fraction(1)}
    for p0, d in ((pu, du), (pw, dw)):
        if d != 0:
            lo, hi = sorted((p0, p0 + d))
            m = math.floor(lo) + 1
            while m < hi:
                ts.add((m - p0) / d)
                m += 1
    ts = sorted(ts)
    length = math.hypot(float(du), float(dw))
    out = []
    for t0, t1 in zip(ts[:-1], ts[1:]):
        tm = (t0 + t1) / 2
        cu = math.floor(pu + tm * du)
        cw = math.floor(pw + tm * dw)
        out.append((cu, cw, float(t1 - t0) * length))
    return out


def trace(E, Sg, P, Q):
    """Eq. 9: Trace(P, Q) = <L_r(P<-Q), T_r(P<-Q)>, folding Eq. 7 over the cells
    crossed from P outwards.  Cells outside the grid are vacuum: <0, 1>."""
    S0, S1 = E.shape
    acc = (0.0, 1.0)
    for cu, cw, ell in segment_cells(P, Q):
        if 0 <= cu < S0 and 0 <= cw < S1:
            c = cell_interval(E[cu, cw], Sg[cu, cw], ell)
            acc = merge(acc, (float(c[0]), float(c[1])))
    return acc


def probe_offsets(n: int, k: int):
    """Cells (du, dw, length) crossed by Trace(P, P + v_n(k)) relative to the
    probe's own pixel, for a probe at a pixel centre (translation invariant)."""
    a = 2 ** n
    return segment_cells((0.5, 0.5), (0.5 + a, 0.5 + 2 * k - a))


# --------------------------------------------------------------------------
# Frames: the four quadrant solves (Algorithm 1, Lighting)
# --------------------------------------------------------------------------

def to_frame(img, d):
    """Image [row r][col c] -> frame [u][w] whose +u axis faces quadrant d.
    +x faces increasing c, +y increasing r.  Only flips and transposes."""
    if d == "+x":
        return img.T
    if d == "-x":
        return img[:, ::-1].T
    if d == "+y":
        return img
    if d == "-y":
        return img[::-1, :]
    raise ValueError(d)


def from_frame(Q, d):
    """Inverse of ``to_frame``."""
    if d == "+x":
        return Q.T
    if d == "-x":
        return Q.T[:, ::-1]
    if d == "+y":
        return Q
    if d == "-y":
        return Q[::-1, :]
    raise ValueError(d)


# --------------------------------------------------------------------------
# Helpers
# --------------------------------------------------------------------------

def shifted(A, s, fill):
    """B[..., y] = A[..., y+s] where 0 <= y+s < S, else ``fill`` (last axis)."""
    S = A.shape[-1]
    B = np.full_like(A, fill)
    if s >= 0:
        if s < S:
            B[..., : S - s] = A[..., s:]
    else:
        if -s < S:
            B[..., -s:] = A[..., : S + s]
    return B


def log2_size(S: int) -> int:
    N = S.bit_length() - 1
    if S != 1 << N:
        raise ValueError("grid side must be a power of two")
    return N


# --------------------------------------------------------------------------
# One quadrant: Algorithm 1, procedure HRC
# --------------------------------------------------------------------------

def seed_level(E, Sg, n: int):
    """T_n(p, k) = Trace(p, p + v_n(k)) for every probe of level n (Algorithm 1,
    the traced levels; Section 5 traces them with per-pixel analytic integration).
    Vectorised over probes: the cells crossed are the same for every probe up to
    translation, and cells outside the grid are vacuum."""
    S = E.shape[0]
    a = 2 ** n
    X = S // a
    TL = np.zeros((X, a + 1, S))
    TT = np.ones((X, a + 1, S))
    # pad the fields with vacuum so that every probe's cells can be sliced
    pad = 2 * a + 2
    Ep = np.zeros((S + 2 * pad, S + 2 * pad))
    Sp = np.zeros_like(Ep)
    Ep[pad:pad + S, pad:pad + S] = E
    Sp[pad:pad + S, pad:pad + S] = Sg
    us = np.arange(X) * a
    ys = np.arange(S)
    for k in range(a + 1):
        acc = (np.zeros((X, S)), np.ones((X, S)))
        for du, dw, ell in probe_offsets(n, k):
            e = Ep[np.ix_(us + du + pad, ys + dw + pad)]
            g = Sp[np.ix_(us + du + pad, ys + dw + pad)]
            acc = merge(acc, cell_interval(e, g, ell))
        TL[:, k, :], TT[:, k, :] = acc
    return TL, TT


def merge_up(prev, n: int):
    """T_n from T_{n-1} (Section 4.1; Algorithm 1's second loop).

    The probe (x*2^n, y) of level n is column 2x of level n-1; the point
    p + v_{n-1}(k') is column 2x+1 of level n-1 at row y + 2k' - 2^(n-1).
    Even k (Eq. 18): Merge(T_{n-1}(p, k/2), T_{n-1}(p + v_{n-1}(k/2), k/2)).
    Odd k (Eq. 19-20): the mean, componentwise on L and T, of the two bent paths
    Merge(T_{n-1}(p, k'), T_{n-1}(p + v_{n-1}(k'), k - k')) for k' = (k+-1)/2.
    An out-of-grid far start is vacuum <0, 1>.
    """
    PL, PT = prev
    S = PL.shape[-1]
    h = 2 ** (n - 1)
    X = S // (2 * h)
    nearL, nearT = PL[0::2], PT[0::2]
    farL, farT = PL[1::2], PT[1::2]
    TL = np.zeros((X, 2 * h + 1, S))
    TT = np.zeros((X, 2 * h + 1, S))

    def bent(ka, kb):
        shift = 2 * ka - h
        far = (shifted(farL[:, kb], shift, 0.0), shifted(farT[:, kb], shift, 1.0))
        return merge((nearL[:, ka], nearT[:, ka]), far)

    for k in range(2 * h + 1):
        if k % 2 == 0:
            TL[:, k], TT[:, k] = bent(k // 2, k // 2)
        else:
            l1, t1 = bent((k + 1) // 2, (k - 1) // 2)
            l2, t2 = bent((k - 1) // 2, (k + 1) // 2)
            TL[:, k] = (l1 + l2) / 2
            TT[:, k] = (t1 + t2) / 2
    return TL, TT


def merge_down(Rnext, Tn, Tn1, n: int, env_next=None):
    """R_n from R_{n+1}, T_n and T_{n+1} (Eq. 14-17; Algorithm 1's third loop).

    For cone ii of probe (x*2^n, y), the upper (s=+1) and lower (s=-1) halves are
    cones jj = 2ii+[s>0] of level n+1, with arc A_{n+1}(jj).
    Odd x (Eq. 14): trace the half-cone's outer edge e = ii+[s>0] to
      q = p + v_n(e), the level n+1 probe in column (x+1)/2 at row y + 2e - 2^n:
      F_s = A*T_n(p,e).L + T_n(p,e).T * R_{n+1}(q, jj).
    Even x (Eq. 15-17): p is the level n+1 probe in column x/2; with
      e2 = 2ii+1+s, q = p + v_{n+1}(e2) is column x/2+1 at row y + 2*e2 - 2^(n+1):
      F_s = ( R_{n+1}(p, jj) + A*T_{n+1}(p,e2).L + T_{n+1}(p,e2).T * R_{n+1}(q, jj) ) / 2.
    R_n = F_+ + F_-.  Lookups of R beyond the last column or row are 0, or,
    with an environment, ``env_next[jj]``: the environment's angular fluence in
    cone jj of level n+1 (``environment_fluence``).
    """
    TnL, TnT = Tn
    T1L, T1T = Tn1
    S = TnL.shape[-1]
    a = 2 ** n
    X = S // a
    env_next = np.zeros(2 * a) if env_next is None else np.asarray(env_next, np.float64)
    # pad R_{n+1} with one column beyond the grid (column S/2^(n+1))
    beyond = np.broadcast_to(env_next[None, :, None], (1,) + Rnext.shape[1:])
    Rp = np.concatenate([Rnext, beyond], axis=0)
    R = np.zeros((X, a, S))
    for ii in range(a):
        for s in (-1, 1):
            up = 1 if s > 0 else 0
            jj = 2 * ii + up
            A = cone_angle(n + 1, jj)
            # odd x = 1, 3, ...: (x+1)/2 = 1, 2, ...
            e = ii + up
            far = shifted(Rp[1:, jj], 2 * e - a, env_next[jj])
            R[1::2, ii] += merge_r((A * TnL[1::2, e], TnT[1::2, e]), far)
            # even x = 0, 2, ...: x/2 = 0, 1, ...; x/2+1 = 1, 2, ...
            e2 = 2 * ii + 1 + s
            far2 = shifted(Rp[1:, jj], 2 * e2 - 2 * a, env_next[jj])
            f1 = merge_r((A * T1L[:, e2], T1T[:, e2]), far2)
            R[0::2, ii] += (Rp[:-1, jj] + f1) / 2
    return R


def build_pyramid(E, Sg, seed_levels: int = 3):
    """T_0..T_N: levels below ``seed_levels`` traced, the rest merged up
    (Section 4.2 traces levels 0, 1, 2 and merges 3..N)."""
    S = E.shape[0]
    N = log2_size(S)
    T = []
    for n in range(N + 1):
        if n < seed_levels:
            T.append(seed_level(E, Sg, n))
        else:
            T.append(merge_up(T[n - 1], n))
    return T


def cascades_from_pyramid(T, env=None):
    """R_{N-1}..R_0 from a T pyramid, with R_N = 0 (Section 4.2), or, with an
    environment (``env[m]`` = its angular fluence per cone of level m), R_N
    looked up from it (the footnote to Section 4.2) and so is every lookup
    outside the grid.  Returns the list R with R[n] = R_n for n = 0..N-1."""
    N = len(T) - 1
    S = T[0][0].shape[-1]
    R = [None] * (N + 1)
    R[N] = np.zeros((1, 2 ** N, S))
    if env is not None:
        R[N] += np.asarray(env[N], np.float64)[None, :, None]
    for n in range(N - 1, -1, -1):
        R[n] = merge_down(R[n + 1], T[n], T[n + 1], n, None if env is None else env[n + 1])
    return R[:N]


def gather(R0, env0: float = 0.0):
    """Algorithm 1, Lighting: the quadrant's contribution to pixel [u, w] is
    R_0([u+1, w], 0); the last column looks beyond the grid and gets 0, or the
    environment's fluence over the quadrant, ``env0``."""
    S = R0.shape[-1]
    Q = np.full((S, S), float(env0))
    Q[: S - 1] = R0[1:, 0, :]
    return Q


def quadrant(E, Sg, seed_levels: int = 3, env=None):
    """One HRC(X, Y) solve plus its gather, in the frame of the quadrant; ``env``
    as for ``cascades_from_pyramid``."""
    T = build_pyramid(np.asarray(E, np.float64), np.asarray(Sg, np.float64), seed_levels)
    R = cascades_from_pyramid(T, env)
    return gather(R[0], 0.0 if env is None else float(env[0][0]))


# --------------------------------------------------------------------------
# Environment (the footnote to Section 4.2): light from beyond the grid
# --------------------------------------------------------------------------

def frame_to_world(d, du, dw):
    """World direction (dc, dr) of the frame vector (du, dw) of quadrant d
    (c: column, increasing +x; r: row, increasing +y), as in ``to_frame``."""
    if d == "+x":
        return du, dw
    if d == "-x":
        return -du, dw
    if d == "+y":
        return dw, du
    if d == "-y":
        return dw, -du
    raise ValueError(d)


def environment_radiance(samples, theta: float) -> float:
    """Radiance of an environment map given as K samples at world angles
    2 pi k / K (angle from +x towards +y), looked up at the nearest sample
    (halfway between two samples: the next one counter-clockwise)."""
    K = len(samples)
    k = math.floor(theta * K / (2 * math.pi) + 0.5) % K
    return float(samples[k])


def environment_fluence(samples, d, N: int):
    """env[m][jj] = A_m(jj) times the environment's radiance in the direction of
    v_m(jj + 1/2), the cone's centre (the map is looked up in the direction of
    v_N(i), footnote to Section 4.2), for m = 0..N in the frame of quadrant d."""
    env = []
    for m in range(N + 1):
        a = 2 ** m
        row = np.zeros(a)
        for jj in range(a):
            dc, dr = frame_to_world(d, a, 2 * jj + 1 - a)
            row[jj] = cone_angle(m, jj) * environment_radiance(samples, math.atan2(dr, dc))
        env.append(row)
    return env


def fluence(eps, sigma, seed_levels: int = 3, environment=None):
    """Per-pixel fluence F of a square power-of-two scene (Algorithm 1, Lighting):
    the sum of the four quadrant solves, before any blur.  ``environment``: K
    radiance samples of an environment map lighting the grid from outside
    (``environment_radiance``), or None for no light beyond the grid."""
    eps = np.asarray(eps, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    if eps.shape != sigma.shape or eps.ndim != 2 or eps.shape[0] != eps.shape[1]:
        raise ValueError("eps and sigma must be equal square 2-D arrays")
    log2_size(eps.shape[0])
    N = log2_size(eps.shape[0])
    F = np.zeros(eps.shape)
    for d in QUADRANTS:
        env = None if environment is None else environment_fluence(environment, d, N)
        Q = quadrant(to_frame(eps, d), to_frame(sigma, d), seed_levels, env)
        F += from_frame(Q, d)
    return F


def entry_counts(S: int):
    """Entries per level of one quadrant solve (Section 4.3): #T_n, #R_n."""
    N = log2_size(S)
    t = [(S >> n) * (2 ** n + 1) * S for n in range(N + 1)]
    r = [(S >> n) * (2 ** n) * S for n in range(N)]
    return t, r
