"""PyTorch-facing calls of the gfx950 L1LS solver (marshalling only).

Every step of the solve runs in the HIP kernels of libl1ls.so; PyTorch only
provides device memory and the stream.  If the library is missing this module
raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


ITERATION_KERNELS = {"auto": 0, "mfma": 1, "wave": 2, "stream": 3}


def options(*, max_iter=500, tol=1e-4, c_alpha=0.5, precision="fp32", backtracking=True,
            monotone=True, fp64_polish=1, polish_after=0, warm_start=False,
            fp64_continue=True, iteration_kernel="auto") -> _lib.Options:
    o = _lib.load().l1ls_options_default()
    o.max_iter = int(max_iter)
    o.tol = float(tol)
    o.c_alpha = float(c_alpha)
    o.precision = {"fp32": _lib.L1LS_FP32, "split_bf16": _lib.L1LS_SPLIT_BF16}[precision]
    o.backtracking = int(bool(backtracking))
    o.monotone = int(bool(monotone))
    o.fp64_polish = int(fp64_polish)  # 0 off, 1 pixels above tol, 2 every pixel
    o.polish_after = int(polish_after)
    o.warm_start = int(bool(warm_start))  # X (out) holds the initial points on entry
    o.fp64_continue = int(bool(fp64_continue))  # FP64 Algorithm 1 after the refinement
    # the kernel of the iterations: auto, mfma (register tile), wave, stream (streamed MFMA tile)
    o.iteration_kernel = ITERATION_KERNELS[iteration_kernel]
    return o


def _check_inputs(A, B, lam):
    if A.dtype != torch.complex64 or B.dtype != torch.complex64:
        raise TypeError("A and B must be complex64")
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("A and B must be device tensors")
    if A.dim() != 2 or B.dim() != 2 or B.shape[1] != A.shape[0]:
        raise ValueError(f"shapes: A (N, L), B (P, N); got {tuple(A.shape)}, {tuple(B.shape)}")
    A = A.contiguous()
    B = B.contiguous()
    p = B.shape[0]
    if isinstance(lam, torch.Tensor):
        lam_t = lam.to(device=B.device, dtype=torch.float32).contiguous().reshape(-1)
    else:
        lam_t = torch.tensor([float(lam)], device=B.device, dtype=torch.float32)
    if lam_t.numel() == 1:
        stride = 0
    elif lam_t.numel() == p:
        stride = 1
    else:
        raise ValueError("lambda must be a scalar or have one value per pixel")
    return A, B, lam_t, stride


class Workspace:
    """A reusable device byte buffer (grown on demand, 256-byte aligned)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.buf.data_ptr()) % 256
        return self.buf[off:off + nbytes]


_default_ws = Workspace()


def workspace_size(n: int, l: int, p: int, opts: _lib.Options | None = None) -> int:
    L = _lib.load()
    sz = ctypes.c_size_t(0)
    _lib.check(L.l1ls_workspace_size(n, l, p, ctypes.byref(opts) if opts else None,
                                     ctypes.byref(sz)), "l1ls_workspace_size")
    return sz.value


def solve(A: torch.Tensor, B: torch.Tensor, lam, *, out: torch.Tensor | None = None,
          workspace: Workspace | None = None, stream=None, blocks: int = 0,
          draws: torch.Tensor | None = None, **opts):
    """Solve min ||A x - b_p||^2 + lambda_p ||x||_1 for every row b_p of B.

    With warm_start=True, `out` must hold each pixel's initial point x^(0) of
    Algorithm 1 on entry (it is overwritten by the result).
    Returns (X, diag) with X (P, L) complex64 and diag a dict of device tensors
    (iters int32, kkt float32, objective float32, status int32 bits, nnz int32).
    blocks > 0: Algorithm 1 with that many column blocks (l1ls_solve_blocks),
    draws a float64 device tensor of uniform draws, one per iteration.
    """
    L = _lib.load()
    A, B, lam_t, stride = _check_inputs(A, B, lam)
    n, l = A.shape
    p = B.shape[0]
    o = options(**opts)
    if o.warm_start and out is None:
        raise ValueError("warm_start needs `out` holding the initial points")
    X = out if out is not None else torch.empty((p, l), dtype=torch.complex64, device=B.device)
    diag = {
        "iters": torch.empty(p, dtype=torch.int32, device=B.device),
        "kkt": torch.empty(p, dtype=torch.float32, device=B.device),
        "objective": torch.empty(p, dtype=torch.float32, device=B.device),
        "status": torch.empty(p, dtype=torch.int32, device=B.device),
        "nnz": torch.empty(p, dtype=torch.int32, device=B.device),
    }
    d = _lib.Diag(diag["iters"].data_ptr(), diag["kkt"].data_ptr(), diag["objective"].data_ptr(),
                  diag["status"].data_ptr(), diag["nnz"].data_ptr())
    ws = (workspace or _default_ws).get(workspace_size(n, l, p, o), B.device)
    if blocks:
        if draws is None or draws.dtype != torch.float64 or not draws.is_cuda or not draws.is_contiguous():
            raise TypeError("draws must be a contiguous float64 device tensor")
        if draws.numel() < min(o.max_iter, o.polish_after if o.polish_after > 0 else o.max_iter):
            raise ValueError("draws needs one value per iteration")
        _lib.check(L.l1ls_solve_blocks(n, l, p, _ptr(A), _ptr(B), _ptr(lam_t), stride, ctypes.byref(o),
                                       int(blocks), _ptr(draws), _ptr(X), ctypes.byref(d), _ptr(ws),
                                       ws.numel(), _stream(stream)),
                   "l1ls_solve_blocks")
    else:
        _lib.check(L.l1ls_solve(n, l, p, _ptr(A), _ptr(B), _ptr(lam_t), stride, ctypes.byref(o),
                                _ptr(X), ctypes.byref(d), _ptr(ws), ws.numel(), _stream(stream)),
                   "l1ls_solve")
    diag["_ws"] = ws
    return X, diag


def solve_noalloc(A: torch.Tensor, B: torch.Tensor, lam, *, out: torch.Tensor,
                  diag: dict | None = None, stream=None, **opts):
    """solve() through l1ls_solve_noalloc: no workspace argument, the library's
    fixed scratch array is used (at most NOALLOC_SCRATCH_BYTES of workspace).
    X (out) and the diagnostics (a dict as new_diag returns, or None) are the
    caller's; nothing is allocated on the device here or in the library."""
    L = _lib.load()
    A, B, lam_t, stride = _check_inputs(A, B, lam)
    n, l = A.shape
    p = B.shape[0]
    o = options(**opts)
    d = _lib.Diag(*(diag[k].data_ptr() for k in ("iters", "kkt", "objective", "status", "nnz"))) \
        if diag is not None else None
    _lib.check(L.l1ls_solve_noalloc(n, l, p, _ptr(A), _ptr(B), _ptr(lam_t), stride, ctypes.byref(o),
                                    _ptr(out), ctypes.byref(d) if d is not None else None,
                                    _stream(stream)), "l1ls_solve_noalloc")
    return out, diag


def solve_counters(n: int, l: int, p: int, diag, stream=None):
    """(forward products, adjoint products, pixels refined, refinement FP64 flops,
    refinement FP32 flops) of the solve that made `diag`."""
    out = (ctypes.c_uint64 * 5)()
    _lib.check(_lib.load().l1ls_solve_counters(n, l, p, _ptr(diag["_ws"]), _stream(stream),
                                               ctypes.byref(out)), "l1ls_solve_counters")
    return tuple(int(v) for v in out)


def solve_constants(n: int, l: int, p: int, diag, stream=None):
    """(L_f, alpha_0, power iterations) of the solve that made `diag` (p > 0)."""
    out = (ctypes.c_double * 3)()
    _lib.check(_lib.load().l1ls_solve_constants(n, l, p, _ptr(diag["_ws"]), _stream(stream),
                                                ctypes.byref(out)), "l1ls_solve_constants")
    return tuple(float(v) for v in out)


def timing_enable(on: bool = True) -> None:
    _lib.load().l1ls_timing_enable(int(on))


def timing_read(kernel: str = "iteration"):
    """(total milliseconds, launches) of one kernel class of l1ls_solve since its
    last read: "iteration", "refine" or "certify"."""
    cls = {"iteration": _lib.KERNEL_ITERATION, "refine": _lib.KERNEL_REFINE,
           "certify": _lib.KERNEL_CERTIFY}[kernel]
    tot = ctypes.c_double(0.0)
    cnt = ctypes.c_int32(0)
    _lib.load().l1ls_timing_read_kernel(cls, ctypes.byref(tot), ctypes.byref(cnt))
    return tot.value, cnt.value


class Plan:
    """Batched solve of stacks of uneven shape (each with its own A).

    Built once from the shapes; ``execute`` only enqueues kernels on the
    stream (no allocation, no synchronisation), so it can be captured into a
    torch.cuda.CUDAGraph (a HIP graph).
    """

    def __init__(self, shapes, **opts):
        L = _lib.load()
        self.shapes = [(int(n), int(l), int(p)) for n, l, p in shapes]
        self.opts = options(**opts)
        arr = (_lib.Stack * max(1, len(self.shapes)))()
        for i, (n, l, p) in enumerate(self.shapes):
            arr[i].n, arr[i].l, arr[i].p = n, l, p
        self._ptr = ctypes.c_void_p()
        _lib.check(L.l1ls_plan_create(arr, len(self.shapes), ctypes.byref(self.opts),
                                      ctypes.byref(self._ptr)), "l1ls_plan_create")
        sz = ctypes.c_size_t(0)
        _lib.check(L.l1ls_plan_workspace_size(self._ptr, ctypes.byref(sz)), "plan workspace")
        self.workspace_bytes = sz.value

    def describe(self) -> str:
        L = _lib.load()
        need = L.l1ls_plan_describe(self._ptr, None, 0)
        buf = ctypes.create_string_buffer(max(need, 1))
        L.l1ls_plan_describe(self._ptr, buf, len(buf))
        return buf.value.decode()

    def execute(self, stacks, workspace: torch.Tensor, stream=None):
        """stacks: list of dicts with A, B, lam (tensor), X and diag tensors."""
        L = _lib.load()
        arr = (_lib.Stack * max(1, len(stacks)))()
        keep = []
        for i, st in enumerate(stacks):
            n, l, p = self.shapes[i]
            A, B, lam_t, stride = _check_inputs(st["A"], st["B"], st["lam"])
            keep += [A, B, lam_t]
            d = st["diag"]
            arr[i].n, arr[i].l, arr[i].p = n, l, p
            arr[i].A, arr[i].B, arr[i].lambda_ = A.data_ptr(), B.data_ptr(), lam_t.data_ptr()
            arr[i].lambda_stride = stride
            arr[i].X = st["X"].data_ptr()
            arr[i].diag = _lib.Diag(d["iters"].data_ptr(), d["kkt"].data_ptr(),
                                    d["objective"].data_ptr(), d["status"].data_ptr(),
                                    d["nnz"].data_ptr())
        self._keep = keep
        _lib.check(L.l1ls_plan_execute(self._ptr, arr, _ptr(workspace), workspace.numel(),
                                       _stream(stream)), "l1ls_plan_execute")

    def __del__(self):
        try:
            if getattr(self, "_ptr", None) and self._ptr.value:
                _lib.load().l1ls_plan_destroy(self._ptr)
        except Exception:
            pass


def new_diag(p: int, device):
    return {"iters": torch.empty(p, dtype=torch.int32, device=device),
            "kkt": torch.empty(p, dtype=torch.float32, device=device),
            "objective": torch.empty(p, dtype=torch.float32, device=device),
            "status": torch.empty(p, dtype=torch.int32, device=device),
            "nnz": torch.empty(p, dtype=torch.int32, device=device)}
