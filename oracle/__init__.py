"""FP64 CPU oracle for the complex L1LS / BPDN problem of arXiv 1805.01759.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the GPU path in ``paper_1805_01759_amd`` and the GPU path never imports it.

The arithmetic lives in ``l1ls_oracle.c`` (plain C, FP64, per-pixel loops);
this module only marshals numpy arrays through ctypes.  ``unrolled_ref`` holds
the plain-PyTorch complex128 version of the unrolled fixed-step map, whose
gradients come from autograd.

Function -> passage of the paper:
  objective      Eq. (1) / Eq. (6)
  prox           Eq. (10), complex form S_tau(v) = v max(0, 1 - tau/|v|)
  lipschitz      the Lipschitz constant of grad f used to bound the step (Eq. (14)-(15))
  rbpg           Algorithm 1 with a single block (J = 1): Eqs. (11), (12), (15)
  exact          the minimiser of Eq. (1): Algorithm 1 + active-set Newton + certificates
  unrolled       Eqs. (11)-(12) with a fixed step, K iterations
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "l1ls_oracle.c")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, FP64, no fast-math)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
             "-o", tmp, _SRC, "-lm", "-pthread"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


class RbpgOpts(ctypes.Structure):
    _fields_ = [("alpha0", ctypes.c_double), ("c_alpha", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("backtracking", ctypes.c_int), ("monotone", ctypes.c_int),
                ("warm_start", ctypes.c_int)]


class RbpgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("backtracks", ctypes.c_int),
                ("alpha", ctypes.c_double), ("kkt_nat", ctypes.c_double),
                ("objective", ctypes.c_double), ("converged", ctypes.c_int)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I, D, I64 = ctypes.c_int, ctypes.c_double, ctypes.c_int64
        L.orc_lipschitz.argtypes = [I, I, P]
        L.orc_lipschitz.restype = D
        L.orc_prox.argtypes = [I, P, D, P]
        L.orc_prox.restype = None
        for name in ("orc_objective", "orc_kkt_sub", "orc_dual_gap"):
            getattr(L, name).argtypes = [I, I, P, P, D, P]
            getattr(L, name).restype = D
        L.orc_kkt_nat.argtypes = [I, I, P, P, D, D, P]
        L.orc_kkt_nat.restype = D
        L.orc_rbpg.argtypes = [I, I, P, P, D, D, ctypes.POINTER(RbpgOpts), P,
                               ctypes.POINTER(RbpgInfo)]
        L.orc_rbpg.restype = None
        L.orc_polish.argtypes = [I, I, P, P, D, D, P]
        L.orc_polish.restype = I
        L.orc_gap_screen.argtypes = [I, I, P, P, D, P, P, P]
        L.orc_gap_screen.restype = I
        L.orc_rbpg_batch.argtypes = [I, I, I64, P, P, P, I64, ctypes.POINTER(RbpgOpts), I,
                                     P, P, P, P]
        L.orc_rbpg_batch.restype = None
        L.orc_exact_batch.argtypes = [I, I, I64, P, P, P, I64, I, P, P, P, P, P]
        L.orc_exact_batch.restype = None
        L.orc_unrolled_batch.argtypes = [I, I, I64, P, P, D, D, I, I, P]
        L.orc_unrolled_batch.restype = None
        L.orc_block_lipschitz.argtypes = [I, I, P, I, I]
        L.orc_block_lipschitz.restype = D
        L.orc_block_pick.argtypes = [I, P, D]
        L.orc_block_pick.restype = I
        L.orc_rbpg_blocks.argtypes = [I, I, P, P, D, D, I, P, P, ctypes.POINTER(RbpgOpts), P,
                                      ctypes.POINTER(RbpgInfo)]
        L.orc_rbpg_blocks.restype = None
        L.orc_rbpg_blocks_batch.argtypes = [I, I, I64, P, P, P, I64, I, P, ctypes.POINTER(RbpgOpts),
                                            I, P, P, P, P]
        L.orc_rbpg_blocks_batch.restype = None
        L.orc_default_threads.argtypes = []
        L.orc_default_threads.restype = I
        _lib = L
    return _lib


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def default_threads() -> int:
    return int(lib().orc_default_threads())


def lipschitz(A) -> float:
    """L_f = 2 lambda_max(A A^H)."""
    A = _c128(A)
    n, l = A.shape
    return float(lib().orc_lipschitz(n, l, _ptr(A)))


def prox(v, tau: float):
    v = _c128(v).ravel()
    out = np.empty_like(v)
    lib().orc_prox(v.size, _ptr(v), float(tau), _ptr(out))
    return out


def objective(A, b, lam, x) -> float:
    A, b, x = _c128(A), _c128(b), _c128(x)
    return float(lib().orc_objective(A.shape[0], A.shape[1], _ptr(A), _ptr(b), float(lam), _ptr(x)))


def kkt_nat(A, b, lam, x, Lf=None) -> float:
    A, b, x = _c128(A), _c128(b), _c128(x)
    Lf = lipschitz(A) if Lf is None else Lf
    return float(lib().orc_kkt_nat(A.shape[0], A.shape[1], _ptr(A), _ptr(b), float(lam),
                                   float(Lf), _ptr(x)))


def kkt_sub(A, b, lam, x) -> float:
    A, b, x = _c128(A), _c128(b), _c128(x)
    return float(lib().orc_kkt_sub(A.shape[0], A.shape[1], _ptr(A), _ptr(b), float(lam), _ptr(x)))


def dual_gap(A, b, lam, x) -> float:
    A, b, x = _c128(A), _c128(b), _c128(x)
    return float(lib().orc_dual_gap(A.shape[0], A.shape[1], _ptr(A), _ptr(b), float(lam), _ptr(x)))


def gap_screen(A, b, lam, x):
    """Gap-safe screening at x: (mask of bins whose minimiser entry is certainly 0,
    duality gap F(x) - D(nu))."""
    A, b, x = _c128(A), _c128(b), _c128(x)
    n, l = A.shape
    mask = np.zeros(l, np.int32)
    gap = ctypes.c_double(0.0)
    lib().orc_gap_screen(n, l, _ptr(A), _ptr(b), float(lam), _ptr(x), _ptr(mask), ctypes.byref(gap))
    return mask.astype(bool), gap.value


def rbpg(A, b, lam, *, tol=1e-4, max_iter=500, c_alpha=0.5, alpha0=0.0,
         backtracking=True, monotone=True, Lf=None, x0=None):
    """Algorithm 1 with one block on a single pixel, from x^(0) = x0 (default 0).
    Returns (x, info dict)."""
    A, b = _c128(A), _c128(b)
    n, l = A.shape
    Lf = lipschitz(A) if Lf is None else Lf
    x = np.zeros(l, np.complex128) if x0 is None else _c128(x0).copy()
    o = RbpgOpts(alpha0, c_alpha, tol, max_iter, int(backtracking), int(monotone), int(x0 is not None))
    info = RbpgInfo()
    lib().orc_rbpg(n, l, _ptr(A), _ptr(b), float(lam), float(Lf), ctypes.byref(o), _ptr(x),
                   ctypes.byref(info))
    return x, {f: getattr(info, f) for f, _ in RbpgInfo._fields_}


def polish(A, b, lam, x, Lf=None):
    A, b = _c128(A), _c128(b)
    x = _c128(x).copy()
    Lf = lipschitz(A) if Lf is None else Lf
    lib().orc_polish(A.shape[0], A.shape[1], _ptr(A), _ptr(b), float(lam), float(Lf), _ptr(x))
    return x


def _lam_array(lam, p):
    lam = np.ascontiguousarray(np.atleast_1d(np.asarray(lam, dtype=np.float64)))
    stride = 0 if lam.size == 1 else 1
    if stride and lam.size != p:
        raise ValueError("lambda must be a scalar or have one value per pixel")
    return lam, stride


def rbpg_batch(A, B, lam, *, tol=1e-4, max_iter=500, c_alpha=0.5, alpha0=0.0,
               backtracking=True, monotone=True, nthreads=0, X0=None):
    """Algorithm 1 (J = 1) on every pixel row of B; threads over pixels.  X0
    (P, L): the initial points x^(0) (default 0)."""
    A, B = _c128(A), _c128(B)
    n, l = A.shape
    p = B.shape[0]
    lam, stride = _lam_array(lam, p)
    X = np.zeros((p, l), np.complex128) if X0 is None else np.ascontiguousarray(_c128(X0)).copy()
    if X.shape != (p, l):
        raise ValueError("X0 must be (P, L)")
    iters = np.zeros(p, np.int32)
    kkt = np.zeros(p, np.float64)
    conv = np.zeros(p, np.int32)
    o = RbpgOpts(alpha0, c_alpha, tol, max_iter, int(backtracking), int(monotone), int(X0 is not None))
    lib().orc_rbpg_batch(n, l, p, _ptr(A), _ptr(B), _ptr(lam), stride, ctypes.byref(o),
                         int(nthreads), _ptr(X), _ptr(iters), _ptr(kkt), _ptr(conv))
    return X, {"iters": iters, "kkt_nat": kkt, "converged": conv.astype(bool)}


def block_lipschitz(A, J: int):
    """L_j = 2 lambda_max(A_j A_j^H) of the J contiguous column blocks (Eq. (14))."""
    A = _c128(A)
    n, l = A.shape
    return np.array([lib().orc_block_lipschitz(n, l, _ptr(A), int(J), j) for j in range(J)])


def block_pick(Lb, u: float) -> int:
    """The block that the uniform draw u selects with P_j = L_j / sum L (Eq. (14))."""
    Lb = np.ascontiguousarray(Lb, dtype=np.float64)
    return int(lib().orc_block_pick(Lb.size, _ptr(Lb), float(u)))


def rbpg_blocks(A, b, lam, J: int, u, *, tol=1e-4, max_iter=500, c_alpha=0.5, alpha0=0.0,
                backtracking=True, monotone=True, Lf=None):
    """Algorithm 1 with J blocks on one pixel; u[k-1] is the draw of iteration k."""
    A, b = _c128(A), _c128(b)
    n, l = A.shape
    Lf = lipschitz(A) if Lf is None else Lf
    Lb = block_lipschitz(A, J)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.size >= max_iter
    x = np.zeros(l, np.complex128)
    o = RbpgOpts(alpha0, c_alpha, tol, max_iter, int(backtracking), int(monotone))
    info = RbpgInfo()
    lib().orc_rbpg_blocks(n, l, _ptr(A), _ptr(b), float(lam), float(Lf), int(J), _ptr(Lb), _ptr(u),
                          ctypes.byref(o), _ptr(x), ctypes.byref(info))
    return x, {f: getattr(info, f) for f, _ in RbpgInfo._fields_}


def rbpg_blocks_batch(A, B, lam, J: int, u, *, tol=1e-4, max_iter=500, c_alpha=0.5, alpha0=0.0,
                      backtracking=True, monotone=True, nthreads=0):
    """Algorithm 1 with J blocks on every pixel row of B (the draws u are shared)."""
    A, B = _c128(A), _c128(B)
    n, l = A.shape
    p = B.shape[0]
    lam, stride = _lam_array(lam, p)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.size >= max_iter
    X = np.zeros((p, l), np.complex128)
    iters = np.zeros(p, np.int32)
    kkt = np.zeros(p, np.float64)
    conv = np.zeros(p, np.int32)
    o = RbpgOpts(alpha0, c_alpha, tol, max_iter, int(backtracking), int(monotone))
    lib().orc_rbpg_blocks_batch(n, l, p, _ptr(A), _ptr(B), _ptr(lam), stride, int(J), _ptr(u),
                                ctypes.byref(o), int(nthreads), _ptr(X), _ptr(iters), _ptr(kkt),
                                _ptr(conv))
    return X, {"iters": iters, "kkt_nat": kkt, "converged": conv.astype(bool)}


def exact_batch(A, B, lam, *, nthreads=0):
    """The certified minimiser of Eq. (1) per pixel row of B."""
    A, B = _c128(A), _c128(B)
    n, l = A.shape
    p = B.shape[0]
    lam, stride = _lam_array(lam, p)
    X = np.zeros((p, l), np.complex128)
    ks, kn, gap, obj = (np.zeros(p) for _ in range(4))
    lib().orc_exact_batch(n, l, p, _ptr(A), _ptr(B), _ptr(lam), stride, int(nthreads), _ptr(X),
                          _ptr(ks), _ptr(kn), _ptr(gap), _ptr(obj))
    return X, {"kkt_sub": ks, "kkt_nat": kn, "gap": gap, "objective": obj}


def unrolled_batch(A, B, lam: float, alpha: float, K: int, *, nthreads=0):
    """K fixed-step accelerated proximal-gradient iterations per pixel row of B."""
    A, B = _c128(A), _c128(B)
    n, l = A.shape
    p = B.shape[0]
    X = np.zeros((p, l), np.complex128)
    lib().orc_unrolled_batch(n, l, p, _ptr(A), _ptr(B), float(lam), float(alpha), int(K),
                             int(nthreads), _ptr(X))
    return X
