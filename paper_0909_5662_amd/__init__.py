"""Python binding of librot: batched DMRG operator rotation on MI355X.

Argument marshalling only: every arithmetic step runs in the HIP kernels of
``librot.so`` (built in-tree by ``paper_0909_5662_amd.build``).  PyTorch
supplies device memory and the current stream.  There is no CPU fallback:
if the library is missing, importing the binding's entry points raises.

The entry points mirror the C ABI (include/librot.h):
  rot_batch, rot_backward, rot_batch_blocked, rot_pair_loss,
  rot_check_isometry, rot_split_bf16, rot_workspace_size
plus tensor-level helpers ``rotate``, ``rotate_backward``, ``pair_loss``,
``check_isometry``, ``rotate_blocked`` and the autograd functions
``RotateFn`` and ``PairLossFn``.

Operation (Sec. 2 step 5 and Sec. 3.2 of the paper): for every stored
operator O_b, out_b = U^T (O_b (x) I_d) U, with U the (m*d) x m' truncation
isometry (row index i*d + s).
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "ROT_FP64", "ROT_FP32", "ROT_SPLIT_BF16", "ROT_ASSUME_SYMMETRIC_O", "RotError",
    "RotProblem", "problem", "RotSector", "RotBlockedProblem", "lib", "library_path",
    "rot_batch", "rot_batch_noalloc", "rot_backward", "rot_batch_blocked", "rot_pair_loss", "rot_check_isometry",
    "rot_split_bf16", "rot_workspace_size", "rot_blocked_workspace_size",
    "rotate", "rotate_backward", "pair_loss", "check_isometry", "split_bf16",
    "RotateFn", "PairLossFn", "precision_code", "profile_enable", "profile_read",
    "blocked_problem", "rotate_blocked", "Plan", "ROT_PLAN_NO_GRAPH", "ROT_PLAN_NO_TUNE", "ROT_PLAN_RETUNE",
    "RotSiteProblem", "ROT_BLOCK_IDENTITY", "ROT_BLOCK_DIAGONAL", "ROT_BLOCK_DENSE", "rot_batch_site",
    "rot_site_workspace_size", "rotate_site", "expect_block", "expect_cross",
    "RotDmSector", "rot_density_basis", "density_workspace_size", "density_basis",
    "RotSbTerm", "RotSbProblem", "SuperblockH",
]

ROT_FP64, ROT_FP32, ROT_SPLIT_BF16 = 0, 1, 2
ROT_ASSUME_SYMMETRIC_O = 1
_STATUS = {0: "ROT_OK", -1: "ROT_ERR_INVALID_ARG", -2: "ROT_ERR_UNSUPPORTED", -3: "ROT_ERR_WORKSPACE",
           -4: "ROT_ERR_HIP", -5: "ROT_ERR_NOT_ISOMETRY", -6: "ROT_ERR_NOT_CONVERGED"}

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "librot.so")


class RotError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{_STATUS.get(status, status)}: {detail}")
        self.status = status


class RotProblem(ctypes.Structure):
    """rot_problem: leading dimensions ldu, ldo, ldout of 0 select the packed values."""
    _fields_ = [("m", ctypes.c_int32), ("d", ctypes.c_int32), ("mp", ctypes.c_int32),
                ("n_ops", ctypes.c_int32), ("U", ctypes.c_void_p), ("ldu", ctypes.c_int64),
                ("O", ctypes.c_void_p), ("ldo", ctypes.c_int64), ("stride_o", ctypes.c_int64),
                ("out", ctypes.c_void_p), ("ldout", ctypes.c_int64), ("stride_out", ctypes.c_int64)]


def problem(m: int, d: int, mp: int, n_ops: int, U: int, O: int, out: int, ldu: int = 0, ldo: int = 0,
            stride_o: int | None = None, ldout: int = 0, stride_out: int | None = None) -> RotProblem:
    """A rot_problem from raw device addresses (packed layouts by default)."""
    lo, lout = ldo or m, ldout or mp
    return RotProblem(m, d, mp, n_ops, U, ldu, O, ldo, (m - 1) * lo + m if stride_o is None else stride_o,
                      out, ldout, (mp - 1) * lout + mp if stride_out is None else stride_out)


ROT_BLOCK_IDENTITY, ROT_BLOCK_DIAGONAL, ROT_BLOCK_DENSE = 0, 1, 2


class RotSiteProblem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("d", ctypes.c_int32), ("mp", ctypes.c_int32),
                ("n_ops", ctypes.c_int32), ("block_kind", ctypes.c_int32), ("U", ctypes.c_void_p),
                ("site", ctypes.POINTER(ctypes.c_double)), ("X", ctypes.c_void_p), ("stride_x", ctypes.c_int64),
                ("out", ctypes.c_void_p), ("stride_out", ctypes.c_int64)]


class RotSector(ctypes.Structure):
    _fields_ = [("n_up", ctypes.c_int32), ("n_dn", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("offset", ctypes.c_int64)]


class RotBlockedProblem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("site_qn", ctypes.POINTER(ctypes.c_int32)),
                ("n_old", ctypes.c_int32), ("old_sec", ctypes.POINTER(RotSector)),
                ("n_new", ctypes.c_int32), ("new_sec", ctypes.POINTER(RotSector)),
                ("U_blk", ctypes.c_void_p), ("U_off", ctypes.POINTER(ctypes.c_int64)),
                ("n_ops", ctypes.c_int32), ("shift", ctypes.POINTER(ctypes.c_int32)),
                ("O_blk", ctypes.c_void_p), ("O_off", ctypes.POINTER(ctypes.c_int64)),
                ("out_blk", ctypes.c_void_p), ("out_off", ctypes.POINTER(ctypes.c_int64))]


class RotDmSector(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("r", ctypes.c_int32), ("psi", ctypes.c_void_p), ("ld_psi", ctypes.c_int64),
                ("w", ctypes.c_void_p), ("V", ctypes.c_void_p), ("ld_v", ctypes.c_int64)]


class RotSbTerm(ctypes.Structure):
    _fields_ = [("coef", ctypes.c_double), ("left_op", ctypes.c_int32), ("right_op", ctypes.c_int32),
                ("site_a", ctypes.POINTER(ctypes.c_double)), ("site_at", ctypes.POINTER(ctypes.c_double))]


class RotSbProblem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("site_qn", ctypes.POINTER(ctypes.c_int32)),
                ("n_left", ctypes.c_int32), ("left", ctypes.POINTER(RotSector)),
                ("n_right", ctypes.c_int32), ("right", ctypes.POINTER(RotSector)),
                ("target", ctypes.c_int32 * 2),
                ("n_left_ops", ctypes.c_int32), ("left_shift", ctypes.POINTER(ctypes.c_int32)),
                ("left_blk", ctypes.c_void_p), ("left_off", ctypes.POINTER(ctypes.c_int64)),
                ("n_right_ops", ctypes.c_int32), ("right_shift", ctypes.POINTER(ctypes.c_int32)),
                ("right_blk", ctypes.c_void_p), ("right_off", ctypes.POINTER(ctypes.c_int64)),
                ("n_terms", ctypes.c_int32), ("terms", ctypes.POINTER(RotSbTerm))]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded librot.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise RuntimeError(f"{library_path} not found: build it with `python -m paper_0909_5662_amd.build`")
        L = ctypes.CDLL(library_path)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        L.rot_batch.argtypes = [ctypes.POINTER(RotProblem), i32, ctypes.c_int, vp, sz, vp]
        L.rot_batch_ex.argtypes = [ctypes.POINTER(RotProblem), i32, ctypes.c_int, ctypes.c_uint32, vp, sz, vp]
        L.rot_batch_noalloc.argtypes = [ctypes.POINTER(RotProblem), i32, ctypes.c_int, ctypes.c_uint32, vp]
        L.rot_batch_noalloc.restype = ctypes.c_int
        L.rot_noalloc_scratch_bytes.argtypes = []
        L.rot_noalloc_scratch_bytes.restype = sz
        L.rot_workspace_size.argtypes = [ctypes.POINTER(RotProblem), i32, ctypes.c_int, i32, i32]
        L.rot_workspace_size.restype = sz
        L.rot_backward.argtypes = [ctypes.POINTER(RotProblem), i32, ctypes.POINTER(vp), ctypes.POINTER(i64),
                                   ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_uint32, ctypes.c_int,
                                   vp, sz, vp]
        L.rot_batch_site.argtypes = [ctypes.POINTER(RotSiteProblem), i32, ctypes.c_int, vp, sz, vp]
        L.rot_site_workspace_size.argtypes = [ctypes.POINTER(RotSiteProblem), i32, ctypes.c_int, i32]
        L.rot_site_workspace_size.restype = sz
        L.rot_expect_block_workspace_size.argtypes = [i32, i32, i64, i32]
        L.rot_expect_block_workspace_size.restype = sz
        L.rot_expect_block.argtypes = [vp, i32, i32, i64, vp, i32, i64, ctypes.c_int, vp, vp, sz, vp]
        L.rot_expect_cross_workspace_size.argtypes = [i32, i32, i32, i32, i32, i32, i32]
        L.rot_expect_cross_workspace_size.restype = sz
        L.rot_expect_cross.argtypes = [vp, i32, i32, i32, i32, vp, i32, i64, vp, i32, i64, vp, vp, sz, vp]
        L.rot_batch_blocked.argtypes = [ctypes.POINTER(RotBlockedProblem), ctypes.c_int, vp, sz, vp]
        L.rot_blocked_workspace_size.argtypes = [ctypes.POINTER(RotBlockedProblem)]
        L.rot_blocked_workspace_size.restype = sz
        L.rot_pair_loss.argtypes = [vp, i32, i32, i64, ctypes.c_int, vp, vp, vp, vp, vp, sz, vp]
        L.rot_pair_loss_workspace_size.argtypes = [i32, i32]
        L.rot_pair_loss_workspace_size.restype = sz
        L.rot_check_isometry.argtypes = [vp, i32, i32, i64, ctypes.c_int, ctypes.c_double,
                                         ctypes.POINTER(ctypes.c_double), vp, sz, vp]
        L.rot_isometry_workspace_size.argtypes = [i32, i32, ctypes.c_int]
        L.rot_isometry_workspace_size.restype = sz
        L.rot_split_bf16.argtypes = [vp, i64, vp, vp, vp]
        L.rot_sb_layout.argtypes = [ctypes.POINTER(RotSbProblem), i32, ctypes.POINTER(i32), vp, vp, vp, vp,
                                    ctypes.POINTER(i64)]
        L.rot_sb_plan_create.argtypes = [ctypes.POINTER(RotSbProblem), ctypes.POINTER(vp)]
        L.rot_sb_apply.argtypes = [vp, vp, vp, vp]
        L.rot_sb_plan_flops.argtypes = [vp]
        L.rot_sb_plan_flops.restype = ctypes.c_double
        L.rot_sb_plan_destroy.argtypes = [vp]
        L.rot_density_workspace_size.argtypes = [ctypes.POINTER(RotDmSector), i32]
        L.rot_density_workspace_size.restype = sz
        L.rot_density_basis.argtypes = [ctypes.POINTER(RotDmSector), i32, i64, vp, vp, vp, sz, vp]
        L.rot_status_string.restype = ctypes.c_char_p
        L.rot_status_string.argtypes = [ctypes.c_int]
        L.rot_last_error.restype = ctypes.c_char_p
        L.rot_last_error.argtypes = []
        L.rot_version.restype = ctypes.c_int32
        L.rot_plan_create.argtypes = [ctypes.POINTER(RotProblem), i32, ctypes.c_int, vp, sz, ctypes.c_uint32, vp,
                                      ctypes.POINTER(vp)]
        L.rot_plan_create.restype = ctypes.c_int
        L.rot_plan_rebind.argtypes = [vp, ctypes.POINTER(RotProblem), i32, vp]
        L.rot_plan_rebind.restype = ctypes.c_int
        L.rot_plan_execute.argtypes = [vp, vp]
        L.rot_plan_execute.restype = ctypes.c_int
        L.rot_plan_describe.argtypes = [vp, ctypes.c_char_p, sz]
        L.rot_plan_describe.restype = i32
        L.rot_plan_destroy.argtypes = [vp]
        L.rot_plan_destroy.restype = ctypes.c_int
        L.rot_profile_enable.argtypes = [i32]
        L.rot_profile_enable.restype = ctypes.c_int
        L.rot_profile_read.argtypes = [ctypes.c_char_p, sz]
        L.rot_profile_read.restype = i32
        for f in ("rot_batch", "rot_backward", "rot_batch_blocked", "rot_pair_loss",
                  "rot_check_isometry", "rot_split_bf16"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def profile_enable(on: bool) -> None:
    """Start (clearing earlier records) or stop per-kernel event timing."""
    _check(lib().rot_profile_enable(int(on)))


def profile_read() -> dict[str, tuple[int, float]]:
    """{kernel kind: (launches, total ms)} since profile_enable(True)."""
    buf = ctypes.create_string_buffer(1 << 16)
    n = lib().rot_profile_read(buf, len(buf))
    if n < 0:
        raise RotError(-4, "rot_profile_read failed")
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


def _check(status: int) -> None:
    if status != 0:
        raise RotError(status, lib().rot_last_error().decode())


def precision_code(precision) -> int:
    if isinstance(precision, int):
        return precision
    return {"fp64": ROT_FP64, "fp32": ROT_FP32, "split_bf16": ROT_SPLIT_BF16, "bf16x3": ROT_SPLIT_BF16}[precision]


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace allocation is not 256-byte aligned")
    return ws


# --------------------------------------------------------------- raw C ABI --

def rot_workspace_size(groups, prec: int, ops_per_chunk: int = 0, for_backward: bool = False) -> int:
    arr = (RotProblem * len(groups))(*groups)
    return lib().rot_workspace_size(arr, len(groups), prec, ops_per_chunk, int(for_backward))


def rot_batch(groups, prec: int, workspace: int, workspace_bytes: int, stream: int, flags: int = 0) -> None:
    arr = (RotProblem * len(groups))(*groups)
    if flags:
        _check(lib().rot_batch_ex(arr, len(groups), prec, flags, workspace, workspace_bytes, stream))
    else:
        _check(lib().rot_batch(arr, len(groups), prec, workspace, workspace_bytes, stream))


def rot_batch_noalloc(groups, prec: int, stream: int, flags: int = 0) -> None:
    """rot_batch_ex on the library's fixed device scratch (no allocation)."""
    arr = (RotProblem * len(groups))(*groups)
    _check(lib().rot_batch_noalloc(arr, len(groups), prec, flags, stream))


def rot_backward(groups, dOut, stride_dout, dO, dU, flags: int, prec: int, workspace: int,
                 workspace_bytes: int, stream: int) -> None:
    n = len(groups)
    arr = (RotProblem * n)(*groups)
    vp = ctypes.c_void_p
    dout_arr = (vp * n)(*dOut)
    sd_arr = (ctypes.c_int64 * n)(*stride_dout)
    do_arr = None if dO is None else (vp * n)(*dO)
    du_arr = None if dU is None else (vp * n)(*dU)
    _check(lib().rot_backward(arr, n, dout_arr, sd_arr, do_arr, du_arr, flags, prec, workspace,
                              workspace_bytes, stream))


def rot_batch_blocked(problem: RotBlockedProblem, prec: int, workspace: int, workspace_bytes: int,
                      stream: int) -> None:
    _check(lib().rot_batch_blocked(ctypes.byref(problem), prec, workspace, workspace_bytes, stream))


def rot_blocked_workspace_size(problem: RotBlockedProblem) -> int:
    return lib().rot_blocked_workspace_size(ctypes.byref(problem))


def rot_pair_loss(X: int, mp: int, n_ops: int, stride_x: int, prec: int, psi: int, loss: int,
                  pairs: int | None, grad: int | None, workspace: int, workspace_bytes: int,
                  stream: int) -> None:
    _check(lib().rot_pair_loss(X, mp, n_ops, stride_x, prec, psi, loss, pairs, grad, workspace,
                               workspace_bytes, stream))


def rot_check_isometry(U: int, rows: int, cols: int, prec: int, tol: float, workspace: int,
                       workspace_bytes: int, stream: int, ldu: int = 0) -> tuple[int, float]:
    dev = ctypes.c_double(float("nan"))
    st = lib().rot_check_isometry(U, rows, cols, ldu, prec, tol, ctypes.byref(dev), workspace,
                                  workspace_bytes, stream)
    if st not in (0, -5):
        _check(st)
    return st, dev.value


def rot_split_bf16(x: int, n: int, hi: int, lo: int, stream: int) -> None:
    _check(lib().rot_split_bf16(x, n, hi, lo, stream))


# ---------------------------------------------------------- tensor helpers --

def _dtype_for(prec: int):
    return torch.float64 if prec == ROT_FP64 else torch.float32


def _row_layout(t: torch.Tensor, name: str) -> tuple[int, int]:
    """(row stride, matrix stride) of a 2-D matrix or 3-D batch of matrices
    whose rows are contiguous (unit last stride), rows and matrices not
    overlapping: the layouts the C ABI's leading dimensions describe."""
    if t.dim() not in (2, 3) or any(n <= 0 for n in t.shape):
        raise ValueError(f"{name}: expected a non-empty 2-D or 3-D tensor, got shape {tuple(t.shape)}")
    rows, cols = t.shape[-2], t.shape[-1]
    if t.stride(-1) != 1 and cols > 1:
        raise ValueError(f"{name}: rows must be contiguous (unit last stride)")
    ld = t.stride(-2) if rows > 1 else cols
    if ld < cols:
        raise ValueError(f"{name}: row stride {ld} below the row length {cols}")
    extent = (rows - 1) * ld + cols
    bs = extent
    if t.dim() == 3:
        bs = t.stride(0) if t.shape[0] > 1 else extent
        if bs < extent:
            raise ValueError(f"{name}: matrices overlap (stride {bs} < {extent})")
    return ld, bs


def _problem(U: torch.Tensor, O: torch.Tensor, out: torch.Tensor, d: int) -> RotProblem:
    n, m, _ = O.shape
    ldu, _ = _row_layout(U, "U")
    ldo, so = _row_layout(O, "O")
    ldout, sout = _row_layout(out, "out")
    return RotProblem(m, d, U.shape[1], n, U.data_ptr(), ldu, O.data_ptr(), ldo, so, out.data_ptr(), ldout, sout)


def _check_inputs(U: torch.Tensor, O: torch.Tensor, d: int, prec: int) -> None:
    dt = _dtype_for(prec)
    if U.dtype != dt or O.dtype != dt:
        raise TypeError(f"precision {prec} needs {dt} tensors, got {U.dtype}/{O.dtype}")
    if not (U.is_cuda and O.is_cuda) or U.device != O.device:
        raise ValueError("U and O must be tensors on one GPU")
    if O.dim() != 3 or O.shape[1] != O.shape[2] or U.dim() != 2 or U.shape[0] != O.shape[1] * d:
        raise ValueError("expected O (n, m, m) and U (m*d, mp)")
    _row_layout(U, "U")
    _row_layout(O, "O")


def _check_like(t: torch.Tensor, U: torch.Tensor, shape: tuple, name: str, contiguous: bool = True) -> None:
    """t must live on U's device with U's dtype and exactly `shape`; checked
    before anything is launched."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if not t.is_cuda or t.device != U.device:
        raise ValueError(f"{name} must be on {U.device}, got {t.device}")
    if t.dtype != U.dtype:
        raise TypeError(f"{name} must have dtype {U.dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if contiguous and not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def rotate(U: torch.Tensor, O: torch.Tensor, d: int, precision="fp32", out: torch.Tensor | None = None,
           workspace: torch.Tensor | None = None, stream=None, symmetric_O: bool = False) -> torch.Tensor:
    """out_b = U^T (O_b (x) I_d) U for O of shape (n, m, m), U (m*d, mp).
    symmetric_O: every O_b is symmetric; only the upper output triangle is
    computed (and mirrored)."""
    prec = precision_code(precision)
    _check_inputs(U, O, d, prec)
    n, m, _ = O.shape
    mp = U.shape[1]
    if out is None:
        out = torch.empty((n, mp, mp), dtype=U.dtype, device=U.device)
    else:
        _check_like(out, U, (n, mp, mp), "out", contiguous=False)
        _row_layout(out, "out")
    p = _problem(U, O, out, d)
    if workspace is None:
        workspace = _workspace(rot_workspace_size([p], prec), U.device)
    rot_batch([p], prec, workspace.data_ptr(), workspace.numel(), _stream(stream),
              ROT_ASSUME_SYMMETRIC_O if symmetric_O else 0)
    return out


def rot_site_workspace_size(groups, prec: int, ops_per_chunk: int = 0) -> int:
    arr = (RotSiteProblem * len(groups))(*groups)
    return lib().rot_site_workspace_size(arr, len(groups), prec, ops_per_chunk)


def rot_batch_site(groups, prec: int, workspace: int, workspace_bytes: int, stream: int) -> None:
    arr = (RotSiteProblem * len(groups))(*groups)
    _check(lib().rot_batch_site(arr, len(groups), prec, workspace, workspace_bytes, stream))


def rotate_site(U: torch.Tensor, X, S, precision="fp32", workspace: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
    """out_b = U^T (X_b (x) S) U for a site operator S (d x d, host array) and
    X = None (identity of the old block: returns (mp, mp)), a vector of m
    values (diagonal, e.g. the block's fermion parity: returns (mp, mp)), or
    block operators of shape (n, m, m) (returns (n, mp, mp))."""
    import numpy as np
    prec = precision_code(precision)
    if prec == ROT_SPLIT_BF16:
        raise ValueError("rotate_site supports fp32 and fp64")
    S_host = np.ascontiguousarray(np.asarray(S, dtype=np.float64))
    d = S_host.shape[0]
    if S_host.shape != (d, d) or U.shape[0] % d:
        raise ValueError("S must be d x d and U must have m*d rows")
    if U.dtype != _dtype_for(prec) or not U.is_contiguous() or not U.is_cuda:
        raise TypeError("U must be a contiguous CUDA tensor of the precision's dtype")
    m, mp = U.shape[0] // d, U.shape[1]
    if X is None:
        kind, n, xp, sx = ROT_BLOCK_IDENTITY, 1, None, 0
    else:
        if X.dtype != U.dtype or not X.is_contiguous() or not X.is_cuda:
            raise TypeError("X must be a contiguous CUDA tensor with the dtype of U")
        if X.dim() == 1:
            if X.shape[0] != m:
                raise ValueError("diagonal X must have m entries")
            kind, n, xp, sx = ROT_BLOCK_DIAGONAL, 1, X.data_ptr(), 0
        else:
            if X.dim() != 3 or X.shape[1:] != (m, m):
                raise ValueError("block operators must have shape (n, m, m)")
            kind, n, xp, sx = ROT_BLOCK_DENSE, X.shape[0], X.data_ptr(), m * m
    out = torch.empty((n, mp, mp), dtype=U.dtype, device=U.device)
    p = RotSiteProblem(m, d, mp, n, kind, U.data_ptr(), S_host.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       xp, sx, out.data_ptr(), mp * mp)
    if workspace is None:
        workspace = _workspace(rot_site_workspace_size([p], prec), U.device)
    rot_batch_site([p], prec, workspace.data_ptr(), workspace.numel(), _stream(stream))
    return out if kind == ROT_BLOCK_DENSE else out[0]


def expect_block(psi: torch.Tensor, Z: torch.Tensor, d: int, stream=None) -> torch.Tensor:
    """<psi| Z_b (x) I |psi> (FP64) for block operators Z (n, m, m), float32 or
    float64, in the superblock state psi ((m*d) x ncols, float64)."""
    if psi.dtype != torch.float64 or not psi.is_contiguous() or not psi.is_cuda:
        raise TypeError("psi must be a contiguous float64 CUDA tensor")
    if Z.dtype not in (torch.float32, torch.float64) or not Z.is_contiguous() or Z.dim() != 3:
        raise TypeError("Z must be a contiguous (n, m, m) float32/float64 tensor")
    n, m, _ = Z.shape
    if psi.shape[0] != m * d:
        raise ValueError("psi must have m*d rows")
    e = torch.empty(n, dtype=torch.float64, device=psi.device)
    ws = _workspace(lib().rot_expect_block_workspace_size(m, d, psi.shape[1], n), psi.device)
    prec = ROT_FP64 if Z.dtype == torch.float64 else ROT_FP32
    _check(lib().rot_expect_block(psi.data_ptr(), m, d, psi.shape[1], Z.data_ptr(), n, m * m, prec, e.data_ptr(),
                                  ws.data_ptr(), ws.numel(), _stream(stream)))
    return e


def density_workspace_size(sectors) -> int:
    arr = (RotDmSector * len(sectors))(*sectors)
    return lib().rot_density_workspace_size(arr, len(sectors))


def rot_density_basis(sectors, m_keep: int, kept: int, eps: int, workspace: int, workspace_bytes: int,
                      stream: int) -> None:
    arr = (RotDmSector * len(sectors))(*sectors)
    _check(lib().rot_density_basis(arr, len(sectors), m_keep, kept, eps, workspace, workspace_bytes, stream))


def density_basis(psi_sectors, m_keep: int, workspace: torch.Tensor | None = None, stream=None):
    """Reduced density matrix of the system per quantum-number sector, its
    eigenpairs and the m_keep kept states (FP64).  psi_sectors: list of
    (n_k, r_k) float64 CUDA tensors (row-major, unit row stride).  Returns
    (w, V, kept, eps): per sector the descending eigenvalues (n_k,) and the
    eigenvectors as columns of V (n_k, n_k); kept (int32, one per sector) and
    eps (the discarded weight) on the device."""
    if not psi_sectors:
        raise ValueError("need at least one sector")
    dev = psi_sectors[0].device
    secs, w_out, v_out = [], [], []
    for p in psi_sectors:
        if p.dtype != torch.float64 or not p.is_cuda or p.dim() != 2 or (p.shape[1] > 0 and p.stride(1) != 1):
            raise TypeError("each psi sector must be a 2-D float64 CUDA tensor with unit column stride")
        n, r = p.shape
        w = torch.empty(n, dtype=torch.float64, device=dev)
        V = torch.empty((n, n), dtype=torch.float64, device=dev)
        secs.append(RotDmSector(n, r, p.data_ptr() if r > 0 else None, max(p.stride(0), r), w.data_ptr(),
                                V.data_ptr(), n))
        w_out.append(w)
        v_out.append(V)
    kept = torch.empty(len(secs), dtype=torch.int32, device=dev)
    eps = torch.empty(1, dtype=torch.float64, device=dev)
    if workspace is None:
        workspace = _workspace(density_workspace_size(secs), dev)
    rot_density_basis(secs, m_keep, kept.data_ptr(), eps.data_ptr(), workspace.data_ptr(), workspace.numel(),
                      _stream(stream))
    return w_out, v_out, kept, eps


class SuperblockH:
    """The superblock Hamiltonian of Eq. (9) over quantum-number blocks, as a
    plan of librot (rot_sb_plan_create); apply(psi) = H psi in FP64.

    site_qn: d (n_up, n_dn) pairs; left / right: lists of ((n_up, n_dn), dim)
    sectors of B and B~; target: total numbers; left_ops / right_ops: lists of
    (shift, {source sector index: dense block (q + shift <- q)}); terms: list
    of (coef, left_op or -1, site_a or None, site_at or None, right_op or -1).
    The layout of psi is self.blocks: (numbers, rows, cols, offset) per
    system sector, self.total elements."""

    def __init__(self, site_qn, left, right, target, left_ops, right_ops, terms, device="cuda",
                 create_plan: bool = True):
        import numpy as np
        self._keep = []
        d = len(site_qn)
        qn = np.ascontiguousarray(site_qn, dtype=np.int32).reshape(-1)
        self._keep.append(qn)

        def sectors(lst):
            arr = (RotSector * len(lst))(*[RotSector(q[0], q[1], dim, 0) for q, dim in lst])
            self._keep.append(arr)
            return arr

        def ops(lst, n_sec):
            shift = np.ascontiguousarray([sh for sh, _ in lst] or [(0, 0)], dtype=np.int32).reshape(-1)
            off = np.full(max(len(lst) * n_sec, 1), -1, dtype=np.int64)
            parts, pos = [], 0
            for b, (_, blocks) in enumerate(lst):
                for k, blk in sorted(blocks.items()):
                    off[b * n_sec + k] = pos
                    parts.append(np.ascontiguousarray(blk, dtype=np.float64).ravel())
                    pos += parts[-1].size
            data = torch.from_numpy(np.concatenate(parts) if parts else np.zeros(1)).to(device)
            self._keep += [shift, off, data]
            return shift, off, data

        lsh, loff, ldata = ops(left_ops, len(left))
        rsh, roff, rdata = ops(right_ops, len(right))
        tarr = (RotSbTerm * max(len(terms), 1))()
        for i, (coef, lo, sa, sat, ro) in enumerate(terms):
            mats = []
            for S in (sa, sat):
                if S is None:
                    mats.append(None)
                else:
                    a = np.ascontiguousarray(S, dtype=np.float64).reshape(d, d)
                    self._keep.append(a)
                    mats.append(a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
            tarr[i] = RotSbTerm(coef, lo, ro, mats[0], mats[1])
        self._keep.append(tarr)
        P = RotSbProblem()
        P.d = d
        P.site_qn = qn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        P.n_left, P.left = len(left), sectors(left)
        P.n_right, P.right = len(right), sectors(right)
        P.target[0], P.target[1] = target
        P.n_left_ops, P.left_shift = len(left_ops), lsh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        P.left_blk, P.left_off = ldata.data_ptr(), loff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        P.n_right_ops, P.right_shift = len(right_ops), rsh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        P.right_blk, P.right_off = rdata.data_ptr(), roff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        P.n_terms, P.terms = len(terms), tarr
        self.problem = P
        nb, total = ctypes.c_int32(), ctypes.c_int64()
        _check(lib().rot_sb_layout(ctypes.byref(P), 0, ctypes.byref(nb), None, None, None, None, ctypes.byref(total)))
        n = nb.value
        bq = np.zeros(2 * max(n, 1), dtype=np.int32)
        br = np.zeros(max(n, 1), dtype=np.int32)
        bc = np.zeros(max(n, 1), dtype=np.int32)
        bo = np.zeros(max(n, 1), dtype=np.int64)
        _check(lib().rot_sb_layout(ctypes.byref(P), n, ctypes.byref(nb), bq.ctypes.data, br.ctypes.data,
                                   bc.ctypes.data, bo.ctypes.data, ctypes.byref(total)))
        self.blocks = [((int(bq[2 * k]), int(bq[2 * k + 1])), int(br[k]), int(bc[k]), int(bo[k])) for k in range(n)]
        self.total = total.value
        self.device = device
        self._plan = None
        if create_plan:
            plan = ctypes.c_void_p()
            _check(lib().rot_sb_plan_create(ctypes.byref(P), ctypes.byref(plan)))
            self._plan = plan

    @property
    def flops(self) -> float:
        return lib().rot_sb_plan_flops(self._plan)

    def apply(self, psi: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if psi.dtype != torch.float64 or not psi.is_contiguous() or psi.numel() != self.total:
            raise TypeError("psi must be a contiguous float64 tensor of the layout's length")
        if out is None:
            out = torch.empty_like(psi)
        _check(lib().rot_sb_apply(self._plan, psi.data_ptr(), out.data_ptr(), _stream(stream)))
        return out

    def close(self) -> None:
        if getattr(self, "_plan", None):
            lib().rot_sb_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def expect_cross(psi: torch.Tensor, Z: torch.Tensor, W: torch.Tensor, d: int, dR: int,
                 ops_per_chunk: int = 0, stream=None) -> torch.Tensor:
    """<psi| (Z_b (x) I_a) (x) (I_a~ (x) W_k) |psi> (FP64, shape (nL, nR)) for
    Z (nL, m, m) on the left block and W (nR, mR, mR) on the right block, all
    float64; psi is (m*d) x (dR*mR)."""
    for t in (psi, Z, W):
        if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
            raise TypeError("psi, Z and W must be contiguous float64 CUDA tensors")
    nL, m, _ = Z.shape
    nR, mR, _ = W.shape
    if psi.shape != (m * d, dR * mR):
        raise ValueError("psi must be (m*d) x (dR*mR)")
    c = torch.empty((nL, nR), dtype=torch.float64, device=psi.device)
    ws = _workspace(lib().rot_expect_cross_workspace_size(m, d, mR, dR, nL, nR, ops_per_chunk), psi.device)
    _check(lib().rot_expect_cross(psi.data_ptr(), m, d, mR, dR, Z.data_ptr(), nL, m * m, W.data_ptr(), nR, mR * mR,
                                  c.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return c


def rotate_backward(U: torch.Tensor, O: torch.Tensor, d: int, dOut: torch.Tensor, precision="fp32",
                    need_dO: bool = True, need_dU: bool = True, symmetric_O: bool = False,
                    workspace: torch.Tensor | None = None, stream=None):
    """(dO, dU) of the rotation for upstream gradient dOut ((mp, mp), broadcast
    to every operator, or (n, mp, mp))."""
    prec = precision_code(precision)
    _check_inputs(U, O, d, prec)
    n, m, _ = O.shape
    mp = U.shape[1]
    _check_like(dOut, U, (mp, mp) if dOut.dim() == 2 else (n, mp, mp), "dOut")
    sd = 0 if dOut.dim() == 2 else mp * mp
    # the adjoint writes packed outputs: dO (n, m, m) and dU (m*d, mp)
    dO = torch.empty((n, m, m), dtype=O.dtype, device=O.device) if need_dO else None
    dU = torch.empty((m * d, mp), dtype=U.dtype, device=U.device) if need_dU else None
    dummy = torch.empty((1, mp, mp), dtype=U.dtype, device=U.device)
    p = _problem(U, O, dummy, d)
    if workspace is None:
        workspace = _workspace(rot_workspace_size([p], prec, for_backward=True), U.device)
    rot_backward([p], [dOut.data_ptr()], [sd], None if dO is None else [dO.data_ptr()],
                 None if dU is None else [dU.data_ptr()], ROT_ASSUME_SYMMETRIC_O if symmetric_O else 0,
                 prec, workspace.data_ptr(), workspace.numel(), _stream(stream))
    return dO, dU


def pair_loss(X: torch.Tensor, psi: torch.Tensor, want_pairs: bool = False, want_grad: bool = False,
              precision=None, stream=None):
    """Eq. (11) summed over pairs, in FP64 on the GPU.  X: (n, mp, mp) float or
    double; psi: (mp,) double.  Returns (loss (0-d double), pairs, grad)."""
    prec = precision_code(precision) if precision is not None else (
        ROT_FP64 if X.dtype == torch.float64 else ROT_FP32)
    if X.dtype != _dtype_for(prec) or psi.dtype != torch.float64 or not X.is_contiguous():
        raise TypeError("X must be contiguous float32/float64 matching precision; psi float64")
    if not X.is_cuda or X.dim() != 3 or X.shape[1] != X.shape[2] or X.shape[0] < 1:
        raise ValueError("X must be a (n, mp, mp) device tensor with n >= 1")
    n, mp, _ = X.shape
    if not psi.is_cuda or psi.device != X.device or tuple(psi.shape) != (mp,):
        raise ValueError(f"psi must be a ({mp},) float64 tensor on {X.device}")
    loss = torch.empty((), dtype=torch.float64, device=X.device)
    pairs = torch.empty((n, n), dtype=torch.float64, device=X.device) if want_pairs else None
    grad = torch.empty((mp, mp), dtype=X.dtype, device=X.device) if want_grad else None
    ws = _workspace(lib().rot_pair_loss_workspace_size(mp, n), X.device)
    rot_pair_loss(X.data_ptr(), mp, n, mp * mp, prec, psi.contiguous().data_ptr(), loss.data_ptr(),
                  _ptr(pairs), _ptr(grad), ws.data_ptr(), ws.numel(), _stream(stream))
    return loss, pairs, grad


def check_isometry(U: torch.Tensor, tol: float = 1e-6, stream=None) -> tuple[bool, float]:
    """(ok, max|U^T U - I|) computed in FP64 on the GPU; U may have padded
    rows (unit last stride)."""
    prec = ROT_FP64 if U.dtype == torch.float64 else ROT_FP32
    if U.dtype not in (torch.float32, torch.float64) or not U.is_cuda:
        raise TypeError("U must be a float32/float64 device tensor")
    rows, cols = U.shape
    ldu, _ = _row_layout(U, "U")
    ws = _workspace(lib().rot_isometry_workspace_size(rows, cols, prec), U.device)
    st, dev = rot_check_isometry(U.data_ptr(), rows, cols, prec, tol, ws.data_ptr(), ws.numel(), _stream(stream),
                                 ldu=ldu)
    return st == 0, dev


def split_bf16(x: torch.Tensor, stream=None):
    """(hi, lo) int16 tensors holding the bf16 bit patterns of the split."""
    if x.dtype != torch.float32 or not x.is_contiguous():
        raise TypeError("x must be contiguous float32")
    hi = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    lo = torch.empty_like(hi)
    rot_split_bf16(x.data_ptr(), x.numel(), hi.data_ptr(), lo.data_ptr(), _stream(stream))
    return hi, lo


def _sectors(table) -> ctypes.Array:
    """(n, 3) rows (n_up, n_dn, dim) -> rot_sector array with prefix-sum offsets."""
    arr = (RotSector * len(table))()
    off = 0
    for k, (u, d_, dim) in enumerate(table):
        arr[k] = RotSector(int(u), int(d_), int(dim), off)
        off += int(dim)
    return arr


def blocked_problem(site_qn, old, new, shift, U_blk: torch.Tensor, U_off, O_blk: torch.Tensor, O_off,
                    out_off, out_blk: torch.Tensor):
    """Build the rot_blocked_problem descriptor.  Tables are host sequences
    (kept alive by the returned holder); block data are float32 device tensors."""
    import numpy as np
    i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
    keep = {
        "site_qn": np.ascontiguousarray(site_qn, dtype=np.int32).ravel(),
        "old": _sectors(old), "new": _sectors(new),
        "U_off": np.ascontiguousarray(U_off, dtype=np.int64),
        "shift": np.ascontiguousarray(shift, dtype=np.int32).ravel(),
        "O_off": np.ascontiguousarray(O_off, dtype=np.int64),
        "out_off": np.ascontiguousarray(out_off, dtype=np.int64),
    }
    for t in (U_blk, O_blk, out_blk):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise TypeError("block data must be contiguous float32 device tensors")
    p = RotBlockedProblem(
        len(keep["site_qn"]) // 2, keep["site_qn"].ctypes.data_as(i32p),
        len(old), keep["old"], len(new), keep["new"],
        U_blk.data_ptr(), keep["U_off"].ctypes.data_as(i64p),
        len(keep["shift"]) // 2, keep["shift"].ctypes.data_as(i32p),
        O_blk.data_ptr(), keep["O_off"].ctypes.data_as(i64p),
        out_blk.data_ptr(), keep["out_off"].ctypes.data_as(i64p))
    return p, keep


def rotate_blocked(site_qn, old, new, shift, U_blk, U_off, O_blk, O_off, out_off, out_blk,
                   workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Quantum-number block-sparse rotation (FP32); writes and returns out_blk."""
    p, keep = blocked_problem(site_qn, old, new, shift, U_blk, U_off, O_blk, O_off, out_off, out_blk)
    need = rot_blocked_workspace_size(p)
    if need == 0 and len(shift) > 0:
        # invalid descriptor: let the call report why
        need = 256
    if workspace is None:
        workspace = _workspace(need, U_blk.device)
    rot_batch_blocked(p, ROT_FP32, workspace.data_ptr(), workspace.numel(), _stream(stream))
    del keep
    return out_blk


ROT_PLAN_NO_GRAPH, ROT_PLAN_NO_TUNE, ROT_PLAN_RETUNE = 1, 2, 4


class Plan:
    """A fixed set of rotation groups of different sizes, executed as grouped
    persistent launches replayed from a hipGraph (C ABI: rot_plan_*).

    groups: list of (U, O, out, d) device tensors (FP32).  The tensors and the
    workspace are bound by address: keep them alive and in place while the plan
    exists (the plan holds references)."""

    def __init__(self, groups, workspace_bytes: int | None = None, graph: bool = True, tune: bool = True,
                 retune: bool = False, stream=None):
        self._groups = list(groups)
        probs = []
        for U, O, out, d in self._groups:
            _check_inputs(U, O, d, ROT_FP32)
            probs.append(_problem(U, O, out, d))
        self._probs = (RotProblem * len(probs))(*probs)
        if workspace_bytes is None:
            workspace_bytes = rot_workspace_size(probs, ROT_FP32)  # everything in one chunk per class
        dev = self._groups[0][0].device if self._groups else torch.device("cuda")
        self.workspace = _workspace(workspace_bytes, dev)
        flags = (0 if graph else ROT_PLAN_NO_GRAPH) | (0 if tune else ROT_PLAN_NO_TUNE) | (
            ROT_PLAN_RETUNE if retune else 0)
        h = ctypes.c_void_p()
        _check(lib().rot_plan_create(self._probs, len(probs), ROT_FP32, self.workspace.data_ptr(),
                                     self.workspace.numel(), flags, _stream(stream), ctypes.byref(h)))
        self._h = h

    def execute(self, stream=None) -> None:
        _check(lib().rot_plan_execute(self._h, _stream(stream)))

    def rebind(self, groups, stream=None) -> None:
        """Bind new (U, O, out, d) tensors of the same shapes and layouts
        (rot_plan_rebind): later executions on `stream` use them."""
        groups = list(groups)
        probs = []
        for U, O, out, d in groups:
            _check_inputs(U, O, d, ROT_FP32)
            probs.append(_problem(U, O, out, d))
        arr = (RotProblem * len(probs))(*probs)
        _check(lib().rot_plan_rebind(self._h, arr, len(probs), _stream(stream)))
        self._groups = groups
        self._probs = arr

    def describe(self) -> dict:
        import json
        n = lib().rot_plan_describe(self._h, None, 0)
        buf = ctypes.create_string_buffer(n + 1)
        lib().rot_plan_describe(self._h, buf, n + 1)
        return json.loads(buf.value.decode())

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().rot_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RotateFn(torch.autograd.Function):
    """Differentiable rotation.  Saves only U and O; the backward forms
    U dOut_b (and U dOut_b^T) and contracts them with O_b, so no stage-1
    intermediate is stored."""

    @staticmethod
    def forward(ctx, U, O, d, precision="fp32", symmetric_O=False):
        ctx.save_for_backward(U, O)
        ctx.d = d
        ctx.precision = precision
        ctx.symmetric_O = symmetric_O
        return rotate(U, O, d, precision)

    @staticmethod
    def backward(ctx, dOut):
        U, O = ctx.saved_tensors
        prec = precision_code(ctx.precision)
        if dOut.dim() == 3 and dOut.stride(0) == 0 and dOut[0].is_contiguous():
            dOut = dOut[0]  # one matrix broadcast to every operator: pass stride 0
        # the adjoint runs in the forward's own arithmetic (FP64, FP32 or split-BF16)
        dO, dU = rotate_backward(U, O, ctx.d, dOut.contiguous(), prec, ctx.needs_input_grad[1],
                                 ctx.needs_input_grad[0], ctx.symmetric_O)
        return dU, dO, None, None, None


class PairLossFn(torch.autograd.Function):
    """L = sum_ij <psi|X_i X_j|psi> (FP64 reduction); backward returns the
    closed-form gradient psi (S psi)^T + (S^T psi) psi^T for every X_k."""

    @staticmethod
    def forward(ctx, X, psi):
        loss, _, grad = pair_loss(X, psi, want_grad=True)
        ctx.save_for_backward(grad)
        ctx.n = X.shape[0]
        return loss

    @staticmethod
    def backward(ctx, gl):
        (grad,) = ctx.saved_tensors
        g = grad if bool(gl == 1) else grad * gl.to(grad.dtype)
        return g.unsqueeze(0).expand(ctx.n, *grad.shape), None
