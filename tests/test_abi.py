"""Host-side checks of the C ABI (no GPU needed: no call below reaches a launch)."""
import ctypes
import os
import re

import pytest

from paper_1805_01759_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "l1ls.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(l1ls_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    return _lib.load()


def test_every_declared_symbol_is_exported(L):
    names = header_functions()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(_lib.EXPORTS) <= set(names)


def test_options_default(L):
    o = L.l1ls_options_default()
    assert (o.max_iter, round(o.tol, 8), o.c_alpha, o.precision) == (500, 1e-4, 0.5, 0)
    assert o.backtracking == 1 and o.monotone == 1 and o.fp64_polish == 1 and o.warm_start == 0
    assert o.fp64_continue == 1


def _ws(L, n, l, p, o=None):
    sz = ctypes.c_size_t(0)
    st = L.l1ls_workspace_size(n, l, p, ctypes.byref(o) if o else None, ctypes.byref(sz))
    return st, sz.value


def test_workspace_sizes(L):
    st, a = _ws(L, 25, 256, 1 << 20)
    assert st == 0 and a > (1 << 20) * 12
    st, b = _ws(L, 25, 256, 0)
    assert st == 0 and 0 < b < a
    assert _ws(L, 0, 10, 1)[0] == -1
    assert _ws(L, 10, 0, 1)[0] == -1
    assert _ws(L, 10, 10, -1)[0] == -1
    assert _ws(L, 129, 100, 1)[0] == -2
    assert b"supported sizes" in L.l1ls_last_error()
    assert _ws(L, 10, 4097, 1)[0] == -2
    assert _ws(L, 128, 4096, 1)[0] == 0
    o = L.l1ls_options_default()
    o.iteration_kernel = 2  # the wave-per-pixel kernel stops at 1,024 bins
    assert _ws(L, 10, 1024, 1, o)[0] == 0
    assert _ws(L, 10, 1025, 1, o)[0] == -2


def _solve(L, n=4, l=8, p=3, o=None, A=16, B=32, lam=64, X=128, ws=256, wsb=1 << 20, stride=0):
    o = o or L.l1ls_options_default()
    return L.l1ls_solve(n, l, p, ctypes.c_void_p(A), ctypes.c_void_p(B), ctypes.c_void_p(lam),
                        stride, ctypes.byref(o), ctypes.c_void_p(X), None, ctypes.c_void_p(ws),
                        wsb, None)


def test_argument_errors_before_any_launch(L):
    # pointers are fake: every case below must be rejected by validation
    assert _solve(L, A=0) == -1
    assert _solve(L, X=0) == -1
    assert _solve(L, A=12) == -1               # misaligned
    assert _solve(L, ws=128) == -1             # workspace alignment
    assert _solve(L, wsb=16) == -3             # workspace too small
    assert _solve(L, stride=-1) == -1
    for field, val in [("tol", 0.0), ("tol", float("nan")), ("c_alpha", 1.0), ("c_alpha", 0.0),
                       ("max_iter", -1), ("precision", 7), ("warm_start", 2), ("fp64_polish", 3),
                       ("fp64_continue", 2)]:
        o = L.l1ls_options_default()
        setattr(o, field, val)
        assert _solve(L, o=o) == -1, field
    assert _solve(L, n=200) == -2
    assert L.l1ls_status_string(-3) == b"L1LS_ERR_WORKSPACE"


def test_empty_batch_is_a_noop(L):
    assert _solve(L, p=0, A=0, B=0, lam=0, X=0, ws=0, wsb=0) == 0


def test_noalloc_size_limit_checked_on_host(L):
    # l1ls_solve_noalloc refuses, before any device call, a stack whose workspace
    # exceeds its fixed scratch array; the pointers are never read
    o = L.l1ls_options_default()
    big = _lib.NOALLOC_SCRATCH_BYTES // (8 * 25)
    st = L.l1ls_solve_noalloc(25, 256, big, None, None, None, 0, ctypes.byref(o), None, None, None)
    assert st == -3
    assert b"scratch" in L.l1ls_last_error()
    assert L.l1ls_solve_noalloc(25, 256, 10, None, None, None, 0, None, None, None, None) == -1
    assert L.l1ls_solve_noalloc(200, 256, 10, None, None, None, 0, ctypes.byref(o), None, None,
                                None) == -2


def test_warm_start_refused_where_unsupported(L):
    # Algorithm 1 from X runs in the split re/im MFMA kernels and the wave kernel;
    # the block form refuses it before any launch
    o = L.l1ls_options_default()
    o.warm_start = 1
    st = L.l1ls_solve_blocks(4, 8, 3, ctypes.c_void_p(16), ctypes.c_void_p(32), ctypes.c_void_p(64), 0,
                             ctypes.byref(o), 2, ctypes.c_void_p(512), ctypes.c_void_p(128), None,
                             ctypes.c_void_p(256), 1 << 20, None)
    assert st == -2 and b"block form" in L.l1ls_last_error()


def test_split_bf16_refused_without_an_mfma_kernel(L):
    # split-BF16 exists in the MFMA tiles (the register tile up to n = 64, l = 512,
    # the streamed tile for every supported shape); the wave-per-pixel kernel and
    # the block form refuse it instead of computing in FP32
    o = L.l1ls_options_default()
    o.precision = 1
    for n, l in ((64, 512), (65, 256), (50, 513), (128, 1024)):
        assert _ws(L, n, l, 1, o)[0] == 0
    o.iteration_kernel = 2
    for n, l in ((20, 100), (128, 1024)):
        assert _ws(L, n, l, 1, o)[0] == -2
        assert b"split-BF16" in L.l1ls_last_error()
        assert _solve(L, n=n, l=l, o=o, wsb=1 << 26) == -2
    o.iteration_kernel = 0
    st = L.l1ls_solve_blocks(4, 8, 3, ctypes.c_void_p(16), ctypes.c_void_p(32), ctypes.c_void_p(64), 0,
                             ctypes.byref(o), 2, ctypes.c_void_p(512), ctypes.c_void_p(128), None,
                             ctypes.c_void_p(256), 1 << 20, None)
    assert st == -2 and b"FP32 only" in L.l1ls_last_error()


def test_iteration_kernel_option(L):
    # the streamed MFMA tile keeps each persistent workgroup's iterate in the workspace:
    # l_pad x 640 bytes for each of min(tiles of 16 pixels, 512) workgroups
    o = L.l1ls_options_default()
    assert o.iteration_kernel == 0
    st, auto_big = _ws(L, 100, 1024, 1 << 16, o)
    o.iteration_kernel = 2  # the wave kernel keeps no such state
    st2, wave_big = _ws(L, 100, 1024, 1 << 16, o)
    assert st == 0 and st2 == 0 and auto_big - wave_big == 512 * 1024 * 640
    o.iteration_kernel = 3  # streamed tile on a register-tile shape: 7 tiles of 16 pixels
    _, s_small = _ws(L, 50, 512, 100, o)
    o.iteration_kernel = 1
    _, m_small = _ws(L, 50, 512, 100, o)
    assert s_small - m_small == 7 * 512 * 640
    # the automatic choice: the streamed tile in FP32 for 384 < l <= 512, the
    # register tile up to l = 384
    o.iteration_kernel = 0
    assert _ws(L, 50, 512, 100, o)[1] == s_small
    o.iteration_kernel = 1
    _, m_mid = _ws(L, 50, 384, 100, o)
    o.iteration_kernel = 0
    assert _ws(L, 50, 384, 100, o)[1] == m_mid
    o.precision = 1  # the same choice in split-BF16
    assert _ws(L, 50, 512, 100, o)[1] == s_small
    assert _ws(L, 50, 384, 100, o)[1] == m_mid
    o.precision = 0
    o.iteration_kernel = 1  # the register tile takes n <= 64, l <= 512 only
    assert _ws(L, 65, 256, 1, o)[0] == -2
    assert _solve(L, n=50, l=600, o=o, wsb=1 << 26) == -2
    assert _ws(L, 64, 512, 1, o)[0] == 0
    o.iteration_kernel = 4
    assert _ws(L, 10, 10, 1, o)[0] == -1
    assert _solve(L, o=o) == -1
    o.precision = 1  # split-BF16 on the MFMA tiles, not the wave kernel
    o.iteration_kernel = 2
    assert _ws(L, 50, 512, 1, o)[0] == -2
    assert b"split-BF16" in L.l1ls_last_error()
    o.iteration_kernel = 3
    assert _ws(L, 50, 512, 1, o)[0] == 0
    o.iteration_kernel = 0  # beyond the register tile the streamed tile takes split-BF16 too
    _, bf_big = _ws(L, 100, 1024, 1 << 16, o)
    assert bf_big == auto_big
    o.precision = 0
    o.iteration_kernel = 3
    assert _solve(L, o=o, wsb=16) == -3  # workspace checked against the streamed tile's size
