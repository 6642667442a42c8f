"""Algorithmic HBM bytes of each pass (the roofline's numerator).

Every data-structure entry a pass is defined to consume is counted as read
once, and every entry it produces as written once, over the four quadrant
solves, in FP32: an interval <L, T> is 8 bytes, an angular fluence 4 bytes, a
scene value 4 bytes.  Re-reads that a cache may or may not absorb (neighbouring
outputs sharing an input row) are not counted: they are what the kernels must
keep on chip to reach the roofline.

Counts per quadrant follow Section 4.3: T_n has X^2 (1 + 2^-n) entries, R_n has
X^2, with X = S = 2^N.  ``iv`` is the bytes of a stored interval: 8 in FP32, 4
with the 16-bit storage of the forward's ``HRC_FLAG_HALF_INTERVALS``.
"""
from __future__ import annotations

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, AMD's published figure


def _t(S: int, n: int) -> float:
    return S * S * (1.0 + 2.0 ** -n)


def pass_bytes(name: str, N: int, n: int = -1, iv: int = 8) -> float:
    S = 1 << N
    SS = float(S * S)
    q = 4
    if name == "seed":
        # the two fields read once for all four quadrants, T_2 written (the
        # forward's tail folds T_0 and T_1 itself)
        return 8 * SS + q * iv * _t(S, 2)
    if name == "seed_all":
        # the reverse's recomputed forward: T_0..T_2 written
        return 8 * SS + q * 8 * (_t(S, 0) + _t(S, 1) + _t(S, 2))
    if name == "merge_up":
        # levels 3 .. N-1 (the top level is built inside the merge down)
        return q * iv * (_t(S, n - 1) + _t(S, n))
    if name == "merge_down":
        # half of T_n (odd columns) and the even directions of T_{n+1}: together
        # X^2 (1 + 2^-n) intervals (at n = N-1: all of T_{N-1}, from which the
        # even directions of T_N are built, the same count); R_{n+1} read
        # unless n + 1 = N; R_n written
        return q * iv * _t(S, n) + (q * 4 * SS if n + 1 < N else 0.0) + q * 4 * SS
    if name == "tail":
        # the two fields once, R_2 of the four quadrants, F written
        return 8 * SS + q * 4 * SS + 4 * SS
    if name == "gather_adj":
        return q * 4 * SS + q * 4 * SS
    if name == "merge_down_adj":
        # dR_n read, transmittances (4 bytes) of the same intervals as the merge
        # down, dR_{n+1} written
        return q * 4 * SS + q * 4 * _t(S, n) + q * 4 * SS
    if name == "interval_adj":
        b = q * 8 * _t(S, n) * 2  # T_n read, dT_n written
        if 3 <= n + 1 <= N:
            b += q * 8 * _t(S, n + 1)  # dT_{n+1}
        if n < N:
            b += q * 4 * SS  # odd columns of dR_n and R_{n+1}
        if n >= 1:
            b += q * 4 * SS  # even columns of dR_{n-1} and R_n
        return b
    if name == "seed_adj":
        # fields read once, dT_0..dT_2 of the four quadrants read, d eps and d sigma written
        return 8 * SS + q * 8 * (_t(S, 0) + _t(S, 1) + _t(S, 2)) + 8 * SS
    raise ValueError(name)


def forward_passes(N: int):
    """(name, level) of every pass of one forward solve, in order."""
    out = [("seed", -1)]
    out += [("merge_up", n) for n in range(3, N)]
    out += [("merge_down", n) for n in range(N - 1, 1, -1)]
    out += [("tail", -1)]
    return out


def forward_bytes(N: int, iv: int = 8) -> float:
    return sum(pass_bytes(k, N, n, iv) for k, n in forward_passes(N))


def backward_bytes(N: int) -> float:
    """hrc_backward: the forward recomputed down to R_1 (every traced level
    stored, no gather) plus the reverse."""
    b = pass_bytes("seed_all", N)
    b += sum(pass_bytes("merge_up", N, n) for n in range(3, N))
    b += sum(pass_bytes("merge_down", N, n) for n in range(N - 1, 0, -1))
    b += pass_bytes("gather_adj", N)
    b += sum(pass_bytes("merge_down_adj", N, n) for n in range(N - 1))
    b += sum(pass_bytes("interval_adj", N, n) for n in range(N, -1, -1))
    b += pass_bytes("seed_adj", N)
    return b


def forward_bytes_rgb(N: int, iv: int = 16) -> float:
    """hrc_forward_rgb: three emission planes and sigma read (16 bytes a pixel),
    intervals (L_r, L_g, L_b, T) of ``iv`` bytes (16 in FP32, 8 with the 16-bit
    storage), cascade levels and fluence as three planes (12 bytes an entry)."""
    S = 1 << N
    SS = float(S * S)
    q = 4
    b = 16 * SS + q * iv * _t(S, 2)
    b += sum(q * iv * (_t(S, n - 1) + _t(S, n)) for n in range(3, N))
    for n in range(N - 1, 1, -1):
        b += q * iv * _t(S, n) + (q * 12 * SS if n + 1 < N else 0.0) + q * 12 * SS
    b += 16 * SS + q * 12 * SS + 12 * SS
    return b
