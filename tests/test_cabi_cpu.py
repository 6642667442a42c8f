"""The C-ABI library on a machine without a GPU: it loads, exports every
function include/hrc.h declares, and rejects bad arguments on the host before
any device call."""
import ctypes
import os
import re

import pytest

from paper_2505_02041_amd import _lib
from paper_2505_02041_amd._lib import (HRC_ERR_INVALID_ARG, HRC_ERR_SHAPE, HRC_ERR_UNSUPPORTED,
                                       HRC_ERR_WORKSPACE, HRC_OK)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hrc.h")

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                                reason="libhrc.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hrc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_names():
    assert declared_functions() == sorted(_lib.SIGNATURES)


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    lib = _lib.load()
    for s in range(-6, 1):
        assert lib.hrc_status_string(s).decode().startswith("HRC")
    assert b"unknown" in lib.hrc_status_string(-99)


def _ws(N, flags=0):
    f = ctypes.c_size_t(0)
    b = ctypes.c_size_t(0)
    st = _lib.load().hrc_workspace_bytes(N, flags, ctypes.byref(f), ctypes.byref(b))
    return st, f.value, b.value


@pytest.mark.parametrize("N", [3, 6, 10, 12])
def test_workspace_sizes_follow_the_memory_analysis(N):
    """Section 4.3.2: the pyramid holds (N + 3 - 2^-N) S^2 interval entries per
    quadrant.  No solve stores the top level T_N ((2^N + 1) S entries: the
    merge down builds the part it reads).  A forward keeps the pyramids of G
    quadrants at once (8 bytes per entry) without T_0 and T_1 (2 S^2 and 1.5 S^2
    entries, which its tail folds on chip), two cascade levels of G quadrants
    and one spare S^2 field; the backward keeps all four pyramids, every
    cascade level and their adjoints (dT_N included), up to alignment."""
    S = 1 << N
    full = 8 * sum((S >> n) * (2 ** n + 1) * S for n in range(N + 1))
    assert full == pytest.approx(8 * (N + 3 - 2.0 ** -N) * S * S)
    one = full - 8 * (2 ** N + 1) * S
    fwd_one = one - 8 * (2 + 1.5) * S * S
    for flags, G in ((_lib.HRC_FLAG_QUADRANTS_1, 1), (_lib.HRC_FLAG_QUADRANTS_2, 2),
                     (_lib.HRC_FLAG_QUADRANTS_4, 4), (0, 4)):
        st, f, b = _ws(N, flags)
        assert st == HRC_OK
        fwd_min = G * fwd_one + 2 * G * 4 * S * S + 4 * S * S
        assert fwd_min <= f <= fwd_min + 256 * (2 * N + 8), (flags, f, fwd_min)
    bwd_min = 4 * one + 4 * full + 2 * N * 4 * 4 * S * S
    assert bwd_min <= b <= bwd_min + 256 * (4 * N + 10)


@pytest.mark.parametrize("N", [3, 6, 10, 12])
def test_half_interval_workspace(N):
    """With HRC_FLAG_HALF_INTERVALS the forward stores the same interval
    entries in 4 bytes instead of 8 (the 16-bit pairs of Section 5), and so
    does the backward's recomputed forward; the cascade levels, the spare field
    and every adjoint stay FP32."""
    S = 1 << N
    full = sum((S >> n) * (2 ** n + 1) * S for n in range(N + 1))
    one = full - (2 ** N + 1) * S
    fwd_entries = one - (2 + 1.5) * S * S
    for group_flag, G in ((_lib.HRC_FLAG_QUADRANTS_1, 1), (0, 4)):
        st, f, b = _ws(N, group_flag | _lib.HRC_FLAG_HALF_INTERVALS)
        assert st == HRC_OK
        fwd_min = G * 4 * fwd_entries + 2 * G * 4 * S * S + 4 * S * S
        assert fwd_min <= f <= fwd_min + 256 * (2 * N + 8), (group_flag, f, fwd_min)
        bwd_min = 4 * 4 * one + 4 * 8 * full + 2 * N * 4 * 4 * S * S
        assert bwd_min <= b <= bwd_min + 256 * (4 * N + 10), (b, bwd_min)
        assert b < _ws(N, group_flag)[2]


def test_half_intervals_where_taken():
    """The bounce calls and the batch reject the 16-bit storage flag before
    touching the device; the forward and the backward take it and then need
    only the smaller workspaces."""
    lib = _lib.load()
    buf = (ctypes.c_float * 1024)()
    p = ctypes.addressof(buf)
    H = _lib.HRC_FLAG_HALF_INTERVALS
    st, f, b = _ws(5)
    _, fh, bh = _ws(5, H)
    assert fh < f and bh < b
    assert lib.hrc_backward(None, 5, p, p, p, p, p, p, bh - 1, None, H) == HRC_ERR_WORKSPACE
    assert lib.hrc_backward(None, 5, p, p, p, p, p, p, bh, None, H) == HRC_ERR_INVALID_ARG
    assert lib.hrc_forward(None, 5, p, p, p, p, fh - 1, None, H) == HRC_ERR_WORKSPACE
    assert lib.hrc_forward(None, 5, p, p, p, p, fh, None, H) == HRC_ERR_INVALID_ARG  # no context
    fb = ctypes.c_size_t(0)
    assert lib.hrc_multibounce_workspace_bytes(5, 3, H, ctypes.byref(fb), None) == HRC_ERR_UNSUPPORTED
    sc = (_lib.hrc_scene * 1)()
    sc[0].log2_size = 5
    sc[0].emission = sc[0].sigma_t = sc[0].fluence = p
    out = ctypes.c_void_p(0)
    assert lib.hrc_batch_plan(None, sc, 1, H, None, ctypes.byref(out)) == HRC_ERR_UNSUPPORTED


def test_keep_and_reuse_flags_where_taken():
    """HRC_FLAG_KEEP_PYRAMID: the forward's workspace becomes the backward's
    (with or without 16-bit intervals), all four quadrants at once;
    HRC_FLAG_REUSE_PYRAMID only on the backward; the RGB calls take the pair
    alike; every other call rejects both before touching the device."""
    lib = _lib.load()
    buf = (ctypes.c_float * 1024)()
    p = ctypes.addressof(buf)
    K, R = _lib.HRC_FLAG_KEEP_PYRAMID, _lib.HRC_FLAG_REUSE_PYRAMID
    H = _lib.HRC_FLAG_HALF_INTERVALS
    for extra in (0, H):
        st, f, b = _ws(5, extra)
        stk, fk, bk = _ws(5, extra | K)
        assert st == stk == HRC_OK and fk == bk == b and f < b
        assert _ws(5, extra | R)[1:] == (f, b)
        # the kept forward needs the backward's size
        assert lib.hrc_forward(None, 5, p, p, p, p, b - 1, None, extra | K) == HRC_ERR_WORKSPACE
        assert lib.hrc_forward(None, 5, p, p, p, p, b, None, extra | K) == HRC_ERR_INVALID_ARG
        assert lib.hrc_backward(None, 5, p, p, p, p, p, p, b - 1, None, extra | R) == \
            HRC_ERR_WORKSPACE
        assert lib.hrc_backward(None, 5, p, p, p, p, p, p, b, None, extra | R) == \
            HRC_ERR_INVALID_ARG
    st, f, b = _ws(5)
    # quadrant groups other than four, and the flags on the wrong call
    for g in (_lib.HRC_FLAG_QUADRANTS_1, _lib.HRC_FLAG_QUADRANTS_2):
        assert _ws(5, K | g)[0] == HRC_ERR_UNSUPPORTED
        assert lib.hrc_forward(None, 5, p, p, p, p, b, None, K | g) == HRC_ERR_UNSUPPORTED
    assert lib.hrc_forward(None, 5, p, p, p, p, b, None, K | _lib.HRC_FLAG_QUADRANTS_4) == \
        HRC_ERR_INVALID_ARG
    assert lib.hrc_forward(None, 5, p, p, p, p, b, None, R) == HRC_ERR_UNSUPPORTED
    assert lib.hrc_backward(None, 5, p, p, p, p, p, p, b, None, K) == HRC_ERR_UNSUPPORTED
    assert lib.hrc_forward_static(None, 5, p, p, p, None, K) == HRC_ERR_UNSUPPORTED
    # the RGB calls: the kept forward takes the RGB reverse's workspace (smaller
    # with the 16-bit storage)
    fr, br = ctypes.c_size_t(0), ctypes.c_size_t(0)
    frk, brk = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.hrc_workspace_bytes_rgb(5, 0, ctypes.byref(fr), ctypes.byref(br)) == HRC_OK
    assert lib.hrc_workspace_bytes_rgb(5, K, ctypes.byref(frk), ctypes.byref(brk)) == HRC_OK
    assert frk.value == brk.value == br.value and fr.value < br.value
    frh, brh = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.hrc_workspace_bytes_rgb(5, K | H, ctypes.byref(frh), ctypes.byref(brh)) == HRC_OK
    assert frh.value == brh.value < br.value
    assert lib.hrc_forward_rgb(None, 5, p, p, p, p, brh.value, None, K | H) == HRC_ERR_INVALID_ARG
    assert lib.hrc_backward_rgb(None, 5, p, p, p, p, p, p, brh.value - 1, None, H) == \
        HRC_ERR_WORKSPACE
    assert lib.hrc_forward_rgb(None, 5, p, p, p, p, br.value - 1, None, K) == HRC_ERR_WORKSPACE
    assert lib.hrc_forward_rgb(None, 5, p, p, p, p, br.value, None, K) == HRC_ERR_INVALID_ARG
    assert lib.hrc_forward_rgb(None, 5, p, p, p, p, br.value, None, R) == HRC_ERR_UNSUPPORTED
    assert lib.hrc_backward_rgb(None, 5, p, p, p, p, p, p, br.value, None, R) == HRC_ERR_INVALID_ARG
    assert lib.hrc_backward_rgb(None, 5, p, p, p, p, p, p, br.value, None, K) == HRC_ERR_UNSUPPORTED
    assert lib.hrc_backward_rgb(None, 5, p, p, p, p, p, p, br.value, None, H) == HRC_ERR_INVALID_ARG
    assert lib.hrc_backward_rgb(None, 5, p, p, p, p, p, p, br.value, None, 0x10) == \
        HRC_ERR_UNSUPPORTED
    fb = ctypes.c_size_t(0)
    for flag in (K, R):
        assert lib.hrc_multibounce_workspace_bytes(5, 3, flag, ctypes.byref(fb), None) == \
            HRC_ERR_UNSUPPORTED


@pytest.mark.parametrize("N", [0, 2, 13, -1])
def test_bad_sizes_are_rejected(N):
    assert _ws(N)[0] == HRC_ERR_SHAPE
    lib = _lib.load()
    buf = (ctypes.c_float * 64)()
    p = ctypes.addressof(buf)
    assert lib.hrc_forward(None, N, p, p, p, p, 1 << 40, None, 0) == HRC_ERR_SHAPE


def test_unknown_flags_are_rejected():
    lib = _lib.load()
    f = ctypes.c_size_t(0)
    assert lib.hrc_workspace_bytes(5, 0x80, ctypes.byref(f), None) == HRC_ERR_UNSUPPORTED


def test_argument_checks_run_before_any_device_call():
    """Host pointers stand in for device pointers: every check below fails
    before the library touches the (absent) GPU."""
    lib = _lib.load()
    buf = (ctypes.c_float * 1024)()
    p = ctypes.addressof(buf)
    assert p % 16 == 0
    st, f, b = _ws(5)
    # NULL and misaligned pointers
    assert lib.hrc_forward(None, 5, None, p, p, p, f, None, 0) == HRC_ERR_INVALID_ARG
    assert lib.hrc_forward(None, 5, p + 4, p, p, p, f, None, 0) == HRC_ERR_INVALID_ARG
    assert lib.hrc_backward(None, 5, p, p, p, p, None, p, b, None, 0) == HRC_ERR_INVALID_ARG
    # workspace too small
    assert lib.hrc_forward(None, 5, p, p, p, p, f - 1, None, 0) == HRC_ERR_WORKSPACE
    assert lib.hrc_backward(None, 5, p, p, p, p, p, p, b - 1, None, 0) == HRC_ERR_WORKSPACE
    # forward workspace is not enough for the backward
    assert lib.hrc_backward(None, 5, p, p, p, p, p, p, f, None, 0) == HRC_ERR_WORKSPACE
    # everything valid but no context
    assert lib.hrc_forward(None, 5, p, p, p, p, f, None, 0) == HRC_ERR_INVALID_ARG
    assert lib.hrc_backward(None, 5, p, p, p, p, p, p, b, None, 0) == HRC_ERR_INVALID_ARG
    # unknown flags
    assert lib.hrc_forward(None, 5, p, p, p, p, f, None, 0x100) == HRC_ERR_UNSUPPORTED
    # a quadrant grouping that needs a larger workspace than the one given
    st1, f4, _ = _ws(5, _lib.HRC_FLAG_QUADRANTS_4)
    st2, f1, _ = _ws(5, _lib.HRC_FLAG_QUADRANTS_1)
    assert f1 < f4
    assert lib.hrc_forward(None, 5, p, p, p, p, f1, None, _lib.HRC_FLAG_QUADRANTS_4) == HRC_ERR_WORKSPACE


def test_batch_argument_checks():
    lib = _lib.load()
    out = ctypes.c_void_p(0)
    assert lib.hrc_batch_plan(None, None, 0, 0, None, ctypes.byref(out)) == HRC_ERR_INVALID_ARG
    assert lib.hrc_batch_plan(None, None, 1, 0, None, None) == HRC_ERR_INVALID_ARG
    buf = (ctypes.c_float * 64)()
    p = ctypes.addressof(buf)
    sc = (_lib.hrc_scene * 1)()
    sc[0].log2_size = 2
    sc[0].emission = sc[0].sigma_t = sc[0].fluence = p
    assert lib.hrc_batch_plan(None, sc, 1, 0, None, ctypes.byref(out)) == HRC_ERR_SHAPE
    sc[0].log2_size = 5
    sc[0].grad_fluence = p  # partial gradient set
    assert lib.hrc_batch_plan(None, sc, 1, 0, None, ctypes.byref(out)) == HRC_ERR_INVALID_ARG
    sc[0].grad_fluence = None
    assert lib.hrc_batch_plan(None, sc, 1, 0, None, ctypes.byref(out)) == HRC_ERR_INVALID_ARG
    assert out.value is None
    assert lib.hrc_batch_launch(None, None) == HRC_ERR_INVALID_ARG
    assert lib.hrc_batch_workspace_bytes(None) == 0
    assert lib.hrc_batch_describe(None, None, None, None, None, None) == HRC_ERR_INVALID_ARG
    sc[0].grad_fluence = None
    for bad in (0x1, 0x300, 0x700, 0x800):  # unknown, or both kernel variants forced
        assert lib.hrc_batch_plan(None, sc, 1, bad, None, ctypes.byref(out)) == \
            HRC_ERR_UNSUPPORTED
    lib.hrc_batch_destroy(None)
    lib.hrc_destroy(None)


def test_environment_argument_checks():
    lib = _lib.load()
    one = (ctypes.c_float * 1)(1.0)
    assert lib.hrc_set_environment(None, one, 1) == HRC_ERR_INVALID_ARG
    assert lib.hrc_set_environment(None, None, 0) == HRC_ERR_INVALID_ARG


def test_multibounce_argument_checks():
    lib = _lib.load()
    f, b = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.hrc_multibounce_workspace_bytes(5, 0, 0, ctypes.byref(f), None) == HRC_ERR_INVALID_ARG
    assert lib.hrc_multibounce_workspace_bytes(5, 65, 0, ctypes.byref(f), None) == HRC_ERR_INVALID_ARG
    assert lib.hrc_multibounce_workspace_bytes(5, 3, 0x2, ctypes.byref(f), None) == HRC_ERR_UNSUPPORTED
    assert lib.hrc_multibounce_workspace_bytes(5, 3, 0, ctypes.byref(f), ctypes.byref(b)) == 0
    single_f, single_b = _ws(5, 0)[1:]
    S2 = 4 * 32 * 32
    assert f.value >= single_f + S2 and b.value >= single_b + (4 + 2) * S2
    f3 = f.value
    assert lib.hrc_multibounce_workspace_bytes(5, 5, 0, ctypes.byref(f), ctypes.byref(b)) == 0
    assert f.value == f3  # the forward does not keep bounces
    buf = (ctypes.c_float * 64)()
    p = ctypes.addressof(buf)
    assert lib.hrc_multibounce_forward(None, 5, p, p, p, 3, p, p, f3, None, 0) == HRC_ERR_INVALID_ARG
    assert lib.hrc_multibounce_forward(None, 5, p, p, p, 3, p, p, f3 - 1, None, 0) == HRC_ERR_WORKSPACE
    assert lib.hrc_multibounce_forward(None, 5, p, p, p, 0, p, p, f3, None, 0) == HRC_ERR_INVALID_ARG
    assert lib.hrc_multibounce_forward(None, 5, p, p, p, 3, p, p, f3, None, 0x2) == HRC_ERR_UNSUPPORTED
    assert lib.hrc_multibounce_backward(None, 5, p, p, p, 3, p, p, p, p, p, 1, None, 0) == HRC_ERR_WORKSPACE
