"""FP64 oracle of the reverse pass of HRC (test infrastructure only).

``fluence_vjp(eps, sigma, dF)`` returns (d eps, d sigma) = J^T dF for the
forward map ``oracle.hrc.fluence``.  Every function is the transpose of the
forward step of the same name in ``oracle.hrc``, written in scatter form; it is
pinned by FP64 central differences of the forward pass, not by itself.

Adjoints of the interval algebra (from Eq. 7 and Eq. 8):
  Merge:   Ln' += gL;  Tn' += gL*Lf + gT*Tf;  Lf' += gL*Tn;  Tf' += gT*Tn
  Merge_r: Ln' += g;   Tn' += g*rf;           rf' += g*Tn
Cell interval <eps*l*phi(tau), exp(-tau)>, tau = sig*l:
  dL/deps = l*phi(tau), dL/dsig = eps*l^2*phi'(tau), dT/dsig = -l*exp(-tau),
  phi'(tau) = (exp(-tau)*(1+tau) - 1)/tau^2, with phi'(0) = -1/2.
"""
from __future__ import annotations

import numpy as np

from .hrc import (QUADRANTS, build_pyramid, cascades_from_pyramid, cell_interval,
                  cone_angle, environment_fluence, from_frame, log2_size, probe_offsets,
                  shifted, to_frame)


def cell_interval_grad(eps, sig, ell):
    """Partial derivatives of ``cell_interval``: (dL/deps, dL/dsig, dT/dsig)."""
    eps = np.asarray(eps, dtype=np.float64)
    sig = np.asarray(sig, dtype=np.float64)
    tau = sig * ell
    tiny = tau < 1e-5
    t1 = np.where(tiny, 1.0, tau)
    phi = np.where(tiny, 1.0 - tau / 2.0 + tau * tau / 6.0, -np.expm1(-t1) / t1)
    # Taylor series of phi' below 1e-2, where the closed form cancels
    small = tau < 1e-2
    t2 = np.where(small, 1.0, tau)
    series = -0.5 + tau * (1 / 3 + tau * (-1 / 8 + tau * (1 / 30 - tau / 144)))
    dphi = np.where(small, series, (np.exp(-t2) * (1.0 + t2) - 1.0) / (t2 * t2))
    return ell * phi, eps * ell * ell * dphi, -ell * np.exp(-tau)


def unshift(B, s):
    """Transpose of ``shifted(A, s, fill)`` with respect to A (fill is a constant)."""
    return shifted(B, -s, 0.0)


def gather_vjp(dQ):
    """Transpose of ``gather``: dR_0[u+1][0][w] = dQ[u][w]."""
    S = dQ.shape[-1]
    dR0 = np.zeros((S, 1, S))
    dR0[1:, 0, :] = dQ[: S - 1]
    return dR0


def merge_down_vjp(dR, Rnext, Tn, Tn1, n, dRnext, dTn, dTn1, env_next=None):
    """Transpose of ``merge_down`` at level n: accumulate into dR_{n+1}
    (``dRnext``, padded with the out-of-grid column), dT_n and dT_{n+1}.  The
    out-of-grid values (0, or the environment's ``env_next``) are constants."""
    TnL, TnT = Tn
    T1L, T1T = Tn1
    dTnL, dTnT = dTn
    dT1L, dT1T = dTn1
    S = TnL.shape[-1]
    a = 2 ** n
    env_next = np.zeros(2 * a) if env_next is None else np.asarray(env_next, np.float64)
    beyond = np.broadcast_to(env_next[None, :, None], (1,) + Rnext.shape[1:])
    Rp = np.concatenate([Rnext, beyond], axis=0)
    for ii in range(a):
        for s in (-1, 1):
            up = 1 if s > 0 else 0
            jj = 2 * ii + up
            A = cone_angle(n + 1, jj)
            # odd x
            g = dR[1::2, ii]
            e = ii + up
            sh = 2 * e - a
            far = shifted(Rp[1:, jj], sh, env_next[jj])
            dTnL[1::2, e] += A * g
            dTnT[1::2, e] += g * far
            dRnext[1:, jj] += unshift(g * TnT[1::2, e], sh)
            # even x
            g = dR[0::2, ii] / 2
            e2 = 2 * ii + 1 + s
            sh2 = 2 * e2 - 2 * a
            far2 = shifted(Rp[1:, jj], sh2, env_next[jj])
            dRnext[:-1, jj] += g
            dT1L[:, e2] += A * g
            dT1T[:, e2] += g * far2
            dRnext[1:, jj] += unshift(g * T1T[:, e2], sh2)


def merge_up_vjp(dT, prev, n, dprev):
    """Transpose of ``merge_up`` at level n: accumulate dT_n into dT_{n-1}."""
    PL, PT = prev
    dTL, dTT = dT
    dPL, dPT = dprev
    S = PL.shape[-1]
    h = 2 ** (n - 1)
    nearL, nearT = PL[0::2], PT[0::2]
    farL, farT = PL[1::2], PT[1::2]

    def bent_vjp(ka, kb, gL, gT):
        sh = 2 * ka - h
        fL = shifted(farL[:, kb], sh, 0.0)
        fT = shifted(farT[:, kb], sh, 1.0)
        tn = nearT[:, ka]
        dPL[0::2, ka] += gL
        dPT[0::2, ka] += gL * fL + gT * fT
        dPL[1::2, kb] += unshift(gL * tn, sh)
        dPT[1::2, kb] += unshift(gT * tn, sh)

    for k in range(2 * h + 1):
        gL, gT = dTL[:, k], dTT[:, k]
        if k % 2 == 0:
            bent_vjp(k // 2, k // 2, gL, gT)
        else:
            bent_vjp((k + 1) // 2, (k - 1) // 2, gL / 2, gT / 2)
            bent_vjp((k - 1) // 2, (k + 1) // 2, gL / 2, gT / 2)


def seed_level_vjp(E, Sg, n, dT, dE, dS):
    """Transpose of ``seed_level``: each trace is a fold of cell intervals
    c_1..c_m, so L = sum_j P_j L_j and T = prod_j T_j with prefix transmittance
    P_j = prod_{i<j} T_i; then dL/dL_j = P_j, dL/dT_j = P_j * L(c_{j+1..m}),
    dT/dT_j = P_j * T(c_{j+1..m})."""
    S = E.shape[0]
    a = 2 ** n
    X = S // a
    pad = 2 * a + 2
    Ep = np.zeros((S + 2 * pad, S + 2 * pad))
    Sp = np.zeros_like(Ep)
    Ep[pad:pad + S, pad:pad + S] = E
    Sp[pad:pad + S, pad:pad + S] = Sg
    dEp = np.zeros_like(Ep)
    dSp = np.zeros_like(Ep)
    us = np.arange(X) * a
    ys = np.arange(S)
    dTL, dTT = dT
    for k in range(a + 1):
        cells = probe_offsets(n, k)
        idx = [np.ix_(us + du + pad, ys + dw + pad) for du, dw, _ in cells]
        ivals = [cell_interval(Ep[ix], Sp[ix], ell) for ix, (_, _, ell) in zip(idx, cells)]
        m = len(cells)
        prefix = [np.ones((X, S))]
        for j in range(m):
            prefix.append(prefix[-1] * ivals[j][1])
        # suffix folds: suf[j] = fold of cells j..m-1
        suf = [None] * (m + 1)
        suf[m] = (np.zeros((X, S)), np.ones((X, S)))
        for j in range(m - 1, -1, -1):
            lj, tj = ivals[j]
            sl, st = suf[j + 1]
            suf[j] = (lj + tj * sl, tj * st)
        gL, gT = dTL[:, k], dTT[:, k]
        for j, (ix, (_, _, ell)) in enumerate(zip(idx, cells)):
            sl, st = suf[j + 1]
            dLj = gL * prefix[j]
            dTj = prefix[j] * (gL * sl + gT * st)
            de, dsL, dsT = cell_interval_grad(Ep[ix], Sp[ix], ell)
            dEp[ix] += dLj * de
            dSp[ix] += dLj * dsL + dTj * dsT
    dE += dEp[pad:pad + S, pad:pad + S]
    dS += dSp[pad:pad + S, pad:pad + S]


def quadrant_vjp(E, Sg, dQ, seed_levels=3, env=None):
    """Reverse of one quadrant solve: forward values are recomputed, then the
    merge down is reversed from level 0 upwards, the merge up from level N
    downwards, and finally the traced levels.  ``env`` as for
    ``cascades_from_pyramid`` (constant: it has no adjoint here)."""
    E = np.asarray(E, np.float64)
    Sg = np.asarray(Sg, np.float64)
    S = E.shape[0]
    N = log2_size(S)
    T = build_pyramid(E, Sg, seed_levels)
    RN = np.zeros((1, 2 ** N, S))
    if env is not None:
        RN += np.asarray(env[N], np.float64)[None, :, None]
    R = cascades_from_pyramid(T, env) + [RN]
    dT = [(np.zeros_like(t[0]), np.zeros_like(t[1])) for t in T]
    dRn = gather_vjp(dQ)
    for n in range(N):
        dRp = np.zeros((R[n + 1].shape[0] + 1,) + R[n + 1].shape[1:])
        merge_down_vjp(dRn, R[n + 1], T[n], T[n + 1], n, dRp, dT[n], dT[n + 1],
                       None if env is None else env[n + 1])
        dRn = dRp[:-1]
    for n in range(N, seed_levels - 1, -1):
        if n >= 1:
            merge_up_vjp(dT[n], T[n - 1], n, dT[n - 1])
    dE = np.zeros((S, S))
    dS = np.zeros((S, S))
    for n in range(min(seed_levels, N + 1)):
        seed_level_vjp(E, Sg, n, dT[n], dE, dS)
    return dE, dS


def fluence_vjp(eps, sigma, dF, seed_levels=3, environment=None):
    """(dLoss/d eps, dLoss/d sigma) given dLoss/dF, for ``oracle.hrc.fluence``
    (with the same ``environment``)."""
    eps = np.asarray(eps, np.float64)
    sigma = np.asarray(sigma, np.float64)
    dF = np.asarray(dF, np.float64)
    N = log2_size(eps.shape[0])
    dE = np.zeros(eps.shape)
    dS = np.zeros(eps.shape)
    for d in QUADRANTS:
        env = None if environment is None else environment_fluence(environment, d, N)
        de, ds = quadrant_vjp(to_frame(eps, d), to_frame(sigma, d), to_frame(dF, d),
                              seed_levels, env)
        dE += from_frame(de, d)
        dS += from_frame(ds, d)
    return dE, dS
